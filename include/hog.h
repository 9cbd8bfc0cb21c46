/*
 * hog.h -- C ABI of the MI355X fast-HOG library (libhog.so).
 *
 * The library implements the method of "A Fast HOG Descriptor Using Lookup
 * Table and Integral Image" (Huang & Huang, arXiv:1703.06256) as
 * hand-written HIP kernels for gfx950:
 *
 *   hog_lut_build     Sec. 2: a 511 x 511 table from every integer (dx, dy)
 *                     to its orientation bin, built once at start-up.
 *   hog_bin_map       Eq. 1 + Sec. 2: central differences per pixel, the
 *                     table lookup, unit magnitude (the oriented gradients
 *                     map of Sec. 3.1).
 *   hog_integral      Eq. 4 + Eq. 5: one integral image per bin.
 *   hog_scan_windows  Eq. 6 + Sec. 3.3 + Sec. 4: per-cell histograms as
 *                     four-corner sums of the integral images, cached once
 *                     per image, concatenated per detection window and
 *                     scored by linear templates (inner products).
 *
 * Conventions shared by every call:
 *   - Device buffers are owned by the caller and passed as plain device
 *     pointers; they must stay valid until the stream's work has finished.
 *     Objects created by the library (hog_lut, hog_plan) own their device
 *     tables and are freed with the matching *_free / *_destroy call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work and return; none of them synchronises.
 *   - Argument errors are found before anything is enqueued: the call
 *     returns HOG_E_INVALID and enqueues nothing. Launch failures return
 *     HOG_E_DEVICE. hog_last_error() gives a message for the calling
 *     thread's last failing call. No C++ exception crosses this boundary.
 *   - Calls on different plans or buffers are re-entrant; concurrent calls
 *     that write the same buffers race.
 *   - Bins are uint8 with 255 meaning "no bin" (image border, zero
 *     gradient); 1 <= n_bins <= 64.
 */
#ifndef HOG_H_
#define HOG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HOG_OK = 0,
    HOG_E_INVALID = 1,   /* bad argument; nothing was enqueued */
    HOG_E_NOMEM = 2,     /* a host or device allocation failed */
    HOG_E_DEVICE = 3,    /* a HIP call or kernel launch failed */
    HOG_E_BUSY = 4,      /* the request queue is full (hog_submit) */
    HOG_E_NOT_READY = 5  /* the request has not finished (hog_poll) */
} hog_status;

#define HOG_NO_BIN 255
#define HOG_MAX_BINS 64
#define HOG_LUT_SIDE 511 /* dx, dy in [-255, 255] */

enum { HOG_NORM_RAW = 0, HOG_NORM_L2 = 1 };

/* Orientation of the table's bins: signed over [0, 2 pi) (the default), or
 * unsigned over [0, pi), where a gradient and its opposite share a bin (the
 * 9-bin, 0..180 degree histograms of Fig. 4's example). */
enum { HOG_ORIENT_SIGNED = 0, HOG_ORIENT_UNSIGNED = 1 };

/* Votes per pixel. HOG_VOTES_HARD: the pixel counts 1 in its bin (Sec. 2's
 * simplest case, which the paper keeps). HOG_VOTES_SOFT: the two-bin vote
 * Sec. 2 attributes to OpenCV, which the paper sets aside -- with a the
 * angle in bin widths minus 1/2, the pixel votes 1 - frac(a) to bin
 * floor(a) mod n and frac(a) to the next bin -- here quantised to whole
 * units of 1/HOG_SOFT_QUANTUM: w1 = floor(frac(a) HOG_SOFT_QUANTUM + 1/2)
 * to the next bin and HOG_SOFT_QUANTUM - w1 to floor(a) mod n, so that the
 * per-bin integral images stay exact integers (in units of
 * 1/HOG_SOFT_QUANTUM) and Eq. 6 stays exact. */
enum { HOG_VOTES_HARD = 0, HOG_VOTES_SOFT = 1 };
#define HOG_SOFT_QUANTUM 32

/* Message for the calling thread's last failing call ("" if none). */
const char *hog_last_error(void);

/* ------------------------------------------------------------------------ */
/* Lookup table (Sec. 2; Fig. 2 shows 8 bins).                              */
/* ------------------------------------------------------------------------ */
typedef struct hog_lut hog_lut;

/* Fill table[(dy+255)*511 + (dx+255)] with the bin of (dx, dy) for every
 * dx, dy in [-255, 255]: the angle of (dx, dy) in [0, 2 pi), measured from
 * +x towards +y (y = row index, growing downwards), falls in the half-open
 * sector [k 2pi/n, (k+1) 2pi/n) and the entry is k; (0, 0) gives 255. The
 * angle is evaluated in FP64 on the host; gradients along the axes and
 * diagonals, the only integer directions that can sit exactly on a sector
 * edge, are binned with exact integer arithmetic. Host-only: table is a
 * caller-owned host buffer of 511*511 bytes. No device call is made. */
hog_status hog_lut_fill_host(int n_bins, uint8_t *table);

/* As hog_lut_fill_host for either orientation. HOG_ORIENT_UNSIGNED: the
 * angle of (dx, dy) is taken mod pi, into [0, pi), and falls in the sector
 * [k pi/n, (k+1) pi/n); axes and diagonals (directions m pi/4) get
 * floor((m mod 4) n / 4), in integers. HOG_E_INVALID for another value. */
hog_status hog_lut_fill_host_ex(int n_bins, int orientation, uint8_t *table);

/* The soft-vote table (HOG_VOTES_SOFT) for either orientation, host-only:
 * table[(dy+255)*511 + (dx+255)] = b0 | w1 << 8 (uint16), b0 the lower of
 * the two bins and w1 the units (0..HOG_SOFT_QUANTUM) that go to bin
 * (b0 + 1) mod n_bins; (0, 0) gives 255 (no vote). Angles as in
 * hog_lut_fill_host_ex, in FP64. */
hog_status hog_lut_fill_soft_host(int n_bins, int orientation, uint16_t *table);

/* Build the table for n_bins once and upload it to the current device.
 * *out is library-owned (host copy + device copy); free with hog_lut_free.
 * Synchronous. */
hog_status hog_lut_build(int n_bins, hog_lut **out);
/* hog_lut_build for either orientation (hog_lut_fill_host_ex). The plans and
 * kernels are the same for both: the orientation lives in the table only. */
hog_status hog_lut_build_ex(int n_bins, int orientation, hog_lut **out);  /* holds both tables */
int hog_lut_orientation(const hog_lut *lut);
void hog_lut_free(hog_lut *lut);
int hog_lut_bins(const hog_lut *lut);
/* Host copy of the table (511*511 bytes, layout as hog_lut_fill_host),
 * valid until hog_lut_free. */
const uint8_t *hog_lut_host(const hog_lut *lut);

/* The device copies a hog_lut holds (Sec. 2's table as the kernels read it):
 *   HOG_LUT_DEVICE_FULL  uint8 [511][511], layout as hog_lut_fill_host_ex;
 *   HOG_LUT_DEVICE_HALF  uint8 [256][511], the dy >= 0 rows that hog_bin_map
 *                        stages in LDS: entry (dx, dy) = bin(dx, dy) | f << 6
 *                        (255 for no bin), where bin(dx, -dy) =
 *                        n_bins - 1 - bin(dx, dy) + f;
 *   HOG_LUT_DEVICE_SOFT  uint16 [511][511], layout as hog_lut_fill_soft_host. */
enum { HOG_LUT_DEVICE_FULL = 0, HOG_LUT_DEVICE_HALF = 1, HOG_LUT_DEVICE_SOFT = 2 };
/* Copy device table `table` of lut into host memory dst (caller-owned,
 * `bytes` must equal that table's size: 261121, 130816 or 522242), reading it
 * back from the device (synchronous; for tests and tools). HOG_E_INVALID for
 * a NULL argument, an unknown table or a wrong size; HOG_E_DEVICE if the
 * copy fails. */
hog_status hog_lut_read_device(const hog_lut *lut, int table, void *dst, int64_t bytes);

/* ------------------------------------------------------------------------ */
/* Plan: level geometry and buffer layout for one image shape.              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t cell;        /* cell side in pixels (Sec. 3.1 "sub areas"); 1..32 */
    int32_t win_cells_x; /* window width in cells; 8 for a 64-pixel window */
    int32_t win_cells_y; /* window height in cells; 16 for 128 pixels; <= 64 */
    int32_t block;       /* L2 blocks: block x block cells, stepping one cell;
                            must be 2 with HOG_NORM_L2 */
    int32_t norm;        /* HOG_NORM_RAW or HOG_NORM_L2 */
    float eps;           /* L2: v / sqrt(|v|^2 + eps^2) */
} hog_scan_params;

typedef struct {
    int32_t width, height; /* source image, pixels; each <= 32767 */
    int32_t channels;      /* 1 (grey) or 3 (interleaved RGB) */
    int32_t n_bins;        /* 1..64 */
    int32_t max_levels;    /* 1: the image only; 0: pyramid down to the window
                              size; k > 1: at most k levels */
    double scale;          /* pyramid step (> 1) when max_levels != 1 */
    int32_t n_templates;   /* K >= 1 linear templates */
    hog_scan_params scan;
    int32_t plane_bits;    /* integral-image element: 32 (or 0) uint32; 16 uint16; 8 uint8.
                              Narrow planes hold ii mod 2^plane_bits (Sec. 4: 16-bit
                              integral images); see hog_integral. 8 needs cell^2 < 256. */
    int32_t votes;         /* HOG_VOTES_HARD (0) or HOG_VOTES_SOFT; soft needs 32-bit planes
                              and width * height * HOG_SOFT_QUANTUM < 2^32 */
} hog_plan_desc;

typedef struct hog_plan hog_plan;

/* One pyramid level. All offsets are from the base pointers passed to the
 * calls below. Level 0 is the source image; level l has scale s_l = s_{l-1}
 * * scale (s_0 = 1, FP64) and size floor(W / s_l) x floor(H / s_l); pixel
 * (x, y) of level l is source pixel (min(W-1, floor(x s_l)),
 * min(H-1, floor(y s_l))) (nearest neighbour). Levels are kept while both
 * sides are at least the window size. */
typedef struct {
    int32_t width, height;
    double scale;
    int64_t bins_offset;     /* bytes; bin (x, y) at bins[bins_offset + y*bins_pitch + x]
                                (soft votes: the uint16 b0 | w1 << 8 at byte offset
                                bins_offset + y*bins_pitch + 2x) */
    int64_t bins_pitch;      /* bytes */
    int64_t ii_offset;       /* elements; ii(x, y) of bin n at ii[ii_offset +
                                n*ii_plane_stride + y*ii_pitch + x] (hog_integral) */
    int64_t ii_pitch;        /* elements between rows; rows are whole 128-byte lines */
    int64_t ii_plane_stride; /* elements between bins' planes */
    int32_t cells_x, cells_y;    /* whole cells: floor(width / cell), ... */
    int32_t windows_x, windows_y;/* window grid; 0 x 0 if the level is smaller than a window */
    int64_t score_offset;    /* elements; scores[score_offset + (wy*windows_x + wx)*K + k] */
    int64_t cell_offset;     /* elements; cell_hist[cell_offset + (cy*cells_x + cx)*n_bins + n] */
    int64_t block_offset;    /* elements; block_feat[block_offset +
                                ((by*(cells_x-1) + bx)*4 + (v*2 + u))*n_bins + n] (L2 only) */
} hog_level_info;

typedef struct {
    int32_t n_levels;
    int64_t bins_bytes;       /* size of the bins buffer */
    int64_t ii_elems;         /* elements (ii_elem_bytes each) of the integral-image buffer */
    int64_t score_elems;      /* float elements of the score buffer */
    int64_t cell_elems;       /* uint32 elements of the optional cell_hist buffer */
    int64_t block_elems;      /* float elements of the optional block_feat buffer */
    int64_t workspace_bytes;  /* scratch needed by hog_integral and hog_scan_windows */
    int32_t feature_dim;      /* window feature length D */
    int64_t total_pixels;     /* sum of level areas */
    int64_t total_windows;    /* sum of window counts */
    int32_t ii_elem_bytes;    /* plane_bits / 8: 4, 2 or 1 */
} hog_plan_sizes;

/* One image of a plan: its levels, and where hog_bin_map reads it. */
typedef struct {
    int32_t first_level, n_levels; /* the image's levels among the plan's */
    int32_t width, height;
    int64_t img_offset;   /* bytes from the input pointer to the image's first pixel */
    int64_t img_pitch;    /* bytes per row; 0: the img_pitch passed to hog_bin_map */
    int64_t total_pixels; /* sum of the image's level areas */
    int64_t total_windows;
} hog_image_info;

/* Validate desc, plan the levels, tiles and buffer layout, and upload the
 * plan's tables to the current device (library-owned; synchronous). */
hog_status hog_plan_create(const hog_plan_desc *desc, hog_plan **out);

/* A batch: n_images images of any sizes (descs[i]: image i's size and
 * pyramid), planned together so that each call below is one launch per kernel
 * for every level of every image -- the scan of Sec. 4 over many images at
 * once. channels, n_bins, n_templates and scan must be equal across the
 * descriptions (HOG_E_INVALID otherwise). The input of hog_bin_map is one
 * device buffer holding the images packed in order, image i at img_offset
 * with rows of width*channels bytes (hog_plan_get_image); pass img_pitch = 0.
 * Levels are numbered image by image; each image's results equal those of a
 * single-image plan of the same description. 1 <= n_images <= 65536. */
hog_status hog_plan_create_batch(const hog_plan_desc *descs, int n_images, hog_plan **out);
int hog_plan_images(const hog_plan *plan);
hog_status hog_plan_get_image(const hog_plan *plan, int image, hog_image_info *out);
void hog_plan_destroy(hog_plan *plan);
hog_status hog_plan_get_sizes(const hog_plan *plan, hog_plan_sizes *out);
hog_status hog_plan_get_level(const hog_plan *plan, int level, hog_level_info *out);

/* ------------------------------------------------------------------------ */
/* The hot path.                                                            */
/* ------------------------------------------------------------------------ */

/* Eq. 1 + Sec. 2. img: device, uint8, row-major, channels interleaved,
 * img_pitch bytes per row (>= width*channels, with (height - 1) * img_pitch +
 * width * channels < 2^32, else HOG_E_INVALID; 0 for a batch plan, whose
 * images are packed as hog_plan_get_image says). For every level, writes the
 * bin map into bins (device, plan layout): for interior pixels, per channel
 * dx = P[x+1][y] - P[x-1][y], dy = P[x][y+1] - P[x][y-1] (on the level's
 * nearest-neighbour image); the channel with the largest dx^2 + dy^2 wins
 * (ties to the lowest index); the bin is lut[(dy+255)*511 + dx+255]. Border
 * pixels and zero gradients get 255. lut must have the plan's n_bins. Soft
 * votes: each pixel gets the uint16 soft-table entry b0 | w1 << 8 instead
 * (255 for no vote). */
hog_status hog_bin_map(const hog_plan *plan, const hog_lut *lut, const uint8_t *img,
                       int64_t img_pitch, uint8_t *bins, void *stream);

/* Eq. 4 + Eq. 5. bins: device, plan layout (as written by hog_bin_map).
 * Writes, for every level and bin n, the integral image
 *   ii[ii_offset + n*ii_plane_stride + y*ii_pitch + x]
 *       = #{ (x', y') : x' <= x, y' <= y, bin(x', y') = n }
 * for 0 <= x < width, 0 <= y < height (uint32, exact). With plane_bits 16
 * or 8 the planes are uint16 / uint8 and hold that count mod 2^plane_bits;
 * since the four-corner sum of Eq. 6 is a sum with signs, taking it mod
 * 2^plane_bits still gives the exact count of any rectangle of fewer than
 * 2^plane_bits pixels, whatever the image size. Values at x < 0 or
 * y < 0 are zero by definition and not stored: a rectangle touching row or
 * column 0 takes them as 0 in the four-corner sum. Elements of a row beyond
 * column width - 1 hold unspecified values. As a by-product it caches every
 * 8 x 8-pixel cell histogram (Eq. 6, the four-corner sums of the planes it
 * writes) in the workspace for hog_scan_windows. workspace: device, at least
 * workspace_bytes, contents on entry ignored. Soft votes: the count becomes
 * the sum of the votes for bin n, in units of 1/HOG_SOFT_QUANTUM (a pixel
 * gives HOG_SOFT_QUANTUM - w1 to b0 and w1 to b0 + 1 mod n_bins), and the
 * cell histograms of every cell size are cached. */
hog_status hog_integral(const hog_plan *plan, const uint8_t *bins, void *ii,
                        void *workspace, void *stream);

/* Eq. 6, Sec. 3.3, Sec. 4. For every level: the histogram of cell (cx, cy),
 * the cell x cell square at (cx*cell, cy*cell), is ii(4) + ii(1) - ii(2) -
 * ii(3) on each bin's plane, computed once per cell and cached. If ii is
 * non-NULL (device, layout and element type as written by hog_integral) the
 * cells are computed from it (mod 2^plane_bits for narrow planes, exact as
 * cell^2 < 2^plane_bits); if ii is NULL the histograms cached by the last
 * hog_integral call on this plan and workspace are used (Sec. 3.3: areas
 * visited more than once are cached before evaluation); that needs 8-pixel
 * cells, otherwise ii is required.
 * Window (wx, wy) covers cells [wx, wx+win_cells_x) x [wy, wy+win_cells_y).
 * Its feature f is, for HOG_NORM_RAW, the cell histograms in row-major cell
 * order, f[(cy*win_cells_x + cx)*n_bins + n]; for HOG_NORM_L2, the 2x2-cell
 * blocks stepping one cell, each normalised as v / sqrt(|v|^2 + eps^2) in
 * FP32, f[((by*(win_cells_x-1) + bx)*4 + (v*2 + u))*n_bins + n]. Scores:
 *   scores[score_offset + (wy*windows_x + wx)*K + k] = bias[k] + sum_d tmpl[k*D + d] f[d]
 * in FP32 arithmetic: the partial dot product over each block (L2) or each
 * cell (raw) is accumulated in FP32, scaled by the block's 1/norm, and the
 * partials are summed in FP64 before the final rounding to FP32.
 * tmpl: device, float[K][D]; bias: device, float[K]; scores: device, float.
 * cell_hist (nullable): device, uint32, receives every cell histogram.
 * block_feat (nullable, L2 only): device, float, receives every normalised
 * block. workspace: the one passed to hog_integral. Soft votes: cells hold
 * vote sums in units of 1/HOG_SOFT_QUANTUM (so does cell_hist); the feature
 * uses them divided by HOG_SOFT_QUANTUM, so a pixel's votes sum to 1. */
hog_status hog_scan_windows(const hog_plan *plan, const void *ii, const float *tmpl,
                            const float *bias, float *scores, uint32_t *cell_hist,
                            float *block_feat, void *workspace, void *stream);

/* ------------------------------------------------------------------------ */
/* Tile shapes.                                                             */
/* ------------------------------------------------------------------------ */
#define HOG_MAX_LEVEL_GROUPS 4
typedef struct {
    int32_t bin_chunk;    /* bins per integral wave, 1..6 (a last, shorter chunk takes the rest) */
    int32_t score_rows;   /* window rows per strip of the one-template matrix-core scorer
                             (L2, 8-cell-wide windows, K < 16, n_bins <= 20); 0 otherwise */
    int32_t level_groups; /* hog_run and hog_graph_create only: the levels (of every image)
                             split into up to this many contiguous ranges of about equal
                             pixel counts, run on concurrent streams, each range starting
                             once the previous one starts writing its planes. 0 or 1: one
                             launch per kernel for all levels; at most HOG_MAX_LEVEL_GROUPS.
                             get_tiles reports the number of ranges in use. Results are the
                             same for every value. */
    int32_t lut_global;   /* where hog_bin_map reads the Sec. 2 table (hard votes): 0, the
                             dy >= 0 half staged in each workgroup's LDS; 1, the full
                             511 x 511 table read through the L1/L2 caches. Results are the
                             same for both. */
} hog_tiles;

hog_status hog_plan_get_tiles(const hog_plan *plan, hog_tiles *out);
/* Install tile shapes (validated: HOG_E_INVALID if out of range). Updates
 * the plan's device tables (synchronous); not to be called while work that
 * uses the plan is in flight. Results do not depend on the tile shapes. */
hog_status hog_plan_set_tiles(hog_plan *plan, const hog_tiles *tiles);

/* Autotuner: times the whole path (hog_run; per candidate, the per-run time
 * of reps back-to-back runs, the best of three such rounds) on the caller's
 * buffers for each candidate tile
 * shape -- bins per integral wave,
 * then window rows per strip, then the table in LDS or through L2, then
 * 1..HOG_MAX_LEVEL_GROUPS level groups --
 * and installs the fastest; *chosen (nullable) receives it. Synchronises the stream; the buffers' contents after the call
 * are those of a hog_run. */
hog_status hog_plan_autotune(hog_plan *plan, const hog_lut *lut, const uint8_t *img,
                             int64_t img_pitch, uint8_t *bins, void *ii, const float *tmpl,
                             const float *bias, float *scores, void *workspace, void *stream,
                             int reps, hog_tiles *chosen);

/* Autotune cache. path names a text file of earlier hog_plan_autotune
 * results, one line per (device architecture and compute-unit count, build of
 * this library, plan shape: every level's size and the plan's bins, channels,
 * templates, scan parameters, plane width and votes); NULL closes the cache.
 * Opening reads the file (it need not exist yet) and resets the counters.
 * While a cache is open, hog_plan_autotune installs a stored result without
 * timing anything (a hit: it runs the path once, so the buffers end as after
 * a tuned call) or times the candidates as usual and appends the result (a
 * miss). Lines that do not parse, and stored tiles the plan rejects, are
 * ignored (the latter are re-tuned). A file that cannot be written keeps the
 * results in memory only. Process-wide and thread-safe; HOG_E_INVALID for an
 * empty path. */
hog_status hog_tune_cache_open(const char *path);
/* Hits and misses of hog_plan_autotune since the cache was opened, and the
 * results it holds (each pointer nullable). */
hog_status hog_tune_cache_stats(int64_t *hits, int64_t *misses, int64_t *entries);

/* ------------------------------------------------------------------------ */
/* The whole path at once.                                                  */
/* ------------------------------------------------------------------------ */

/* hog_bin_map, hog_integral and hog_scan_windows (scores only; cells from the
 * cache for 8-pixel cells, else from ii) in one call, on the same buffers and
 * with the same layouts. Arguments are all checked before anything is
 * enqueued. The scores equal those of the three calls bit for bit; without
 * level groups the one-template matrix-core scorer's weights are prepared in
 * the carry scan's launch rather than a launch of their own. With level
 * groups (hog_tiles) the groups run on the plan's own
 * streams (created on the plan's device by the first such call, freed by
 * hog_plan_destroy), forked from and joined back into `stream`, so the work
 * is ordered on `stream` as without groups; concurrent grouped calls on one
 * plan take turns enqueueing and share those streams. */
hog_status hog_run(const hog_plan *plan, const hog_lut *lut, const uint8_t *img, int64_t img_pitch,
                   uint8_t *bins, void *ii, const float *tmpl, const float *bias, float *scores,
                   void *workspace, void *stream);

/* hog_run without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc). The workspace is a
 * library-owned static device array of HOG_STATIC_SCRATCH_BYTES, one per GPU,
 * held from library load until the process ends; its address is looked up
 * once per device on the first call there. Same buffers, layouts and results
 * as hog_run with one difference: the levels run as one group (the plan's
 * level_groups are not used, since their streams are created on first use),
 * and no kernel timing is recorded. The plan's device must be the current
 * device. HOG_E_INVALID, with nothing enqueued, if the plan's workspace_bytes
 * exceeds HOG_STATIC_SCRATCH_BYTES or an argument is invalid. Every call on a
 * GPU shares that GPU's array, and its contents on entry are ignored: calls
 * whose work overlaps on one GPU (different streams, or threads) race on it
 * and must be ordered by the caller. */
#define HOG_STATIC_SCRATCH_BYTES (64ll << 20)
hog_status hog_run_static(const hog_plan *plan, const hog_lut *lut, const uint8_t *img, int64_t img_pitch,
                          uint8_t *bins, void *ii, const float *tmpl, const float *bias, float *scores,
                          void *stream);

/* hog_run captured once into a HIP graph for these exact buffers, replayed by
 * hog_graph_launch with one launch: for callers that run the same plan on the
 * same buffers again and again (a batch refilled in place, video frames).
 * The buffers' contents are read at replay time; the pointers are fixed. The
 * graph records no memset nodes. Creating it synchronises nothing and
 * launches nothing; hog_graph_destroy frees it (library-owned). */
typedef struct hog_graph hog_graph;
hog_status hog_graph_create(const hog_plan *plan, const hog_lut *lut, const uint8_t *img,
                            int64_t img_pitch, uint8_t *bins, void *ii, const float *tmpl,
                            const float *bias, float *scores, void *workspace, hog_graph **out);
hog_status hog_graph_launch(hog_graph *graph, void *stream);
void hog_graph_destroy(hog_graph *graph);

/* ------------------------------------------------------------------------ */
/* Serving: a request queue with continuous batching.                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t channels, n_bins, n_templates;
    int32_t max_levels;      /* each request's pyramid: 1 = the image only (hog_plan_desc) */
    double scale;
    hog_scan_params scan;
    int32_t max_width, max_height; /* largest image accepted */
    int64_t memory_budget;   /* device bytes for the requests on the device */
    int64_t host_budget;     /* pinned host bytes for the images of queued requests */
    int32_t max_slots;       /* requests on the device at once */
    int32_t max_batch;       /* requests per launch (<= max_slots) */
    int32_t max_queue;       /* requests waiting; hog_submit returns HOG_E_BUSY beyond */
    int32_t streams;         /* batches in flight at once, 1..8 */
    int32_t orientation;     /* HOG_ORIENT_SIGNED or HOG_ORIENT_UNSIGNED */
    int32_t votes;           /* HOG_VOTES_HARD or HOG_VOTES_SOFT (hog_plan_desc) */
    int32_t plane_bits;      /* integral-image element of the server's own buffers
                                (hog_plan_desc; 0 = 32). The scores do not depend on it:
                                8 or 16 cut the device footprint per request. */
    int32_t copy_threads;    /* helper threads that split hog_submit's copies of large
                                images with the caller, 0..32 (0: the caller alone) */
} hog_server_config;

typedef struct hog_server hog_server;

/* A server for one detector: the lookup table and the K templates (host,
 * float[K][D], float[K]; copied) stay on the current device, which also holds
 * an arena of memory_budget bytes for the requests' buffers. A worker thread
 * forms a batch from the oldest waiting request and the waiting requests of
 * the same image size behind it, while slots and arena memory allow -- a
 * request's footprint is that of its plan's buffers (bins, N_b uint32
 * integral images per level, workspace, scores, image) -- and runs it as one
 * batch plan (hog_plan_create_batch, cached per size and count: at most
 * 4 max_batch + 16 plans, the least recently used idle ones dropped beyond
 * that; a batch that cannot be planned is retried with fewer requests) on one of
 * `streams` non-blocking streams: copy in from the pinned host arena
 * (host_budget bytes), hog_run, each request's scores out into its own
 * region of a pinned output arena (room for 2 * max_slots results of the
 * largest image; a finished request holds its region until hog_poll takes
 * it, and admission waits while the arena is full). Requests that arrive while
 * batches are running form the next batches as slots and memory free up,
 * and run concurrently with them. Each
 * request's scores equal those of running its image alone with
 * hog_plan_create (bit for bit). Library-owned; hog_server_destroy waits for
 * the batches on the device and drops requests that never started. */
hog_status hog_server_create(const hog_server_config *cfg, const float *tmpl_host,
                             const float *bias_host, hog_server **out);
void hog_server_destroy(hog_server *server);

/* Builds the batch plans for 1..max_batch images of w x h now, so that the
 * first batches of that size do not wait for them (a plan's tables are
 * allocated and copied synchronously). Optional. HOG_E_INVALID if w x h is
 * outside max_width x max_height or cannot be planned. Thread-safe. */
hog_status hog_server_warm(hog_server *server, int w, int h);

/* Queue an image (host, w x h x channels uint8, rows packed; copied into the
 * server's pinned host memory before returning) and get its ticket.
 * HOG_E_INVALID if the image is larger than max_width x max_height or alone
 * needs more than memory_budget; HOG_E_BUSY if max_queue requests are waiting
 * or host_budget is in use by queued and running requests. Thread-safe. */
hog_status hog_submit(hog_server *server, const uint8_t *host_img, int w, int h, uint64_t *ticket);

/* HOG_E_NOT_READY while the request is waiting or running. Once it is done:
 * copies its scores (every level of its pyramid, in level order, each as
 * hog_scan_windows lays them out: [wy][wx][K]) into scores (cap floats;
 * HOG_E_INVALID if too small, the request is kept), sets the level-0 window
 * grid and the latency from hog_submit to completion (seconds, host clock),
 * and forgets the ticket. HOG_E_INVALID for an unknown ticket. Thread-safe. */
hog_status hog_poll(hog_server *server, uint64_t ticket, float *scores, size_t cap, int *nwx,
                    int *nwy, double *latency_s);

/* Completion queue: writes into tickets[] (cap >= 1 entries) the tickets of
 * requests that finished, succeeded or failed, since the last call, in the
 * order they finished, and their number into *count; waits up to timeout_us
 * microseconds (0: no wait) while there are none. Each ticket is reported
 * once, and not at all if hog_poll has already taken it; take its result
 * with hog_poll. HOG_E_INVALID for NULL pointers, cap <
 * 1 or a negative timeout. Thread-safe. */
hog_status hog_wait_any(hog_server *server, uint64_t *tickets, int cap, int64_t timeout_us,
                        int *count);

/* ------------------------------------------------------------------------ */
/* Kernel timing. When enabled, every kernel launch of the calls above is   */
/* bracketed by a pair of HIP events recorded on the launch stream; totals  */
/* accumulate per kernel name until hog_timing_reset. Not thread-safe.      */
/* Names: "bin_map", "integral_reduce", "integral_scan", "integral_emit",   */
/* "integral_soft" (soft votes: tile reduce, prefixes and plane writer, the */
/* writer also caching 8-pixel cells), "cells", "score", "block_features",  */
/* and, for hog_run with level groups, "score_prep" (the template weights,  */
/* prepared once); there each kernel is timed per level group.              */
/* ------------------------------------------------------------------------ */
hog_status hog_timing_enable(int on);
hog_status hog_timing_reset(void);
/* Waits for the recorded events, then reports launches and total ms. */
hog_status hog_timing_get(const char *kernel, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* HOG_H_ */
