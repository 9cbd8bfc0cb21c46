// Internal interface between the host half of libhog (hog_api.cpp) and the
// gfx950 kernels (hog_kernels.hip). Not installed; not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hogk {

constexpr int kNoBin = 255;

// Bin map: a wave owns 64 consecutive level columns (62 outputs plus one
// halo column each side, so left/right neighbours come from adjacent lanes)
// and walks kBinRows rows, rolling the up/centre/down samples in registers.
constexpr int kBinCols = 62;
constexpr int kBinRows = 16;
// dy >= 0 half of the 511 x 511 lookup table, as staged in LDS.
constexpr int kLutHalfBytes = 256 * 511;
constexpr int kLutEntries = 511 * 511;  // the full (dx, dy) table

// Integral images: a tile is kTile x kTile pixels, one wave per tile and per
// chunk of at most kMaxBinChunk bins; bins are read kRowBatch rows at a time.
constexpr int kTile = 64;
constexpr int kRowBatch = 16;
constexpr int kMaxBinChunk = 6;

// Matrix-core window scorer: one wave per strip of kStripW window columns and
// kStripTH window rows; windows kStripMaxBX + 1 cells wide.
constexpr int kStripW = 16;
constexpr int kStripTH = 16;
constexpr int kStripMaxBX = 7;

// Many-template scorer (K >= 16): one workgroup per kWgW x kWgTH windows and
// 32 templates.
constexpr int kWgW = 64;
constexpr int kWgTH = 8;
// Levels at most kWgW / 2 windows wide take tiles of kWgW / 2 x 2 kWgTH
// windows instead, so that they do not leave half of each tile empty.
constexpr bool wgemm_narrow(int win_x) { return win_x <= kWgW / 2; }

// Workspace bytes of one template's prepared weights for nbp bin slots per
// cell: fragments [bx][slot][lane] of 16 bytes (nbp / 4 slots: the fp16 hi and
// lo halves of the products' steps, or the FP32 weights in exact mode), then
// the column scales [lane] (float), then the template's mode (int, padded).
constexpr int64_t strip_prep_bytes(int nbp)
{
    return (int64_t)kStripMaxBX * (nbp / 4) * 64 * 16 + 64 * 4 + 256;
}

// Kernel indices into the per-kernel prefix tables.
enum {
    KB_BINMAP = 0,  // waves
    KB_ITILE,       // integral tiles
    KB_CSCAN,       // threads of the column-prefix scan: 16 round_up(tiles_x, 4) * n_bins (4 columns each)
    KB_ESCAN,       // threads of the row-carry scan: 16 round_up(tiles_y, 4) * n_bins (4 rows each)
    KB_PSCAN,       // waves of the tile-total prefix: n_bins
    KB_CELL,        // threads of the cell kernel: cells
    KB_STILE,       // workgroups of the scorer: window tiles
    KB_BLOCK,       // threads of the block-feature kernel: blocks
    KB_SSEG,        // soft votes: waves of the tile reduce, one per integral tile
    KB_SSCAN,       // soft votes: threads of the prefixes, one per (bin, tile-rounded row) then per (bin, column)
    KB_SEMIT,       // soft votes: waves of the plane writer, one per (integral tile, pair of bins)
    KB_COUNT
};

// One pyramid level as the kernels see it. Offsets are in elements of the
// buffer they index (bytes for uint8 buffers).
struct Level {
    int32_t w, h;
    int32_t cells_x, cells_y;
    int32_t win_x, win_y;
    int32_t tiles_x, tiles_y;  // integral tiles: ceil(w / kTile) x ceil(h / kTile)
    int32_t bm_gx, bm_gy;      // bin-map waves
    int32_t st_x, st_y;        // scorer tiles
    int32_t cbx, cby;          // 8 x 8-cell blocks of the cell cache: ceil(cells / 8)
    int32_t src_w, src_h;      // the level's source image (nearest-neighbour maps index it)
    int64_t src_off;           // bytes: the source image in the input buffer
    int64_t src_pitch;         // bytes per source row; 0: the pitch passed to the call
    int64_t mapx_off, mapy_off;
    int64_t bins_off, bins_pitch;
    int64_t ii_off, ii_pitch, ii_plane;
    int64_t score_off, cell_off, block_off;
    // workspace (bytes from the workspace base); hp = 64 tiles_y, wp = 64 tiles_x
    int64_t ws_rowtot;  // uint8  [tiles_x][nb][hp]   count of bin n in row y of tile column tx
    int64_t ws_coltot;  // uint8  [tiles_y][nb][wp]   count of bin n in column x of tile row ty
    int64_t ws_tiletot; // uint32 [tiles_y][tiles_x][nb]  count of bin n in each tile
    int64_t ws_e;       // uint16 [tiles_x][nb][hp]   row y's count left of tile column tx
    int64_t ws_cs;      // uint16 [tiles_y][nb][wp]   column x's count above tile row ty
    int64_t ws_p;       // uint32 [tiles_y][tiles_x][nb]  count above and left of the tile
    int64_t ws_cache;   // uint16 [nb][cby][cbx][8][8] cell histogram cache
    int64_t ws_stot;    // soft votes: uint32 [nb][tiles_x][hp] votes of each tile in row y, then left of it
    int64_t ws_scol;    // soft votes: uint32 [nb][tiles_y][wp] votes of each tile in column x, then above it
};

struct PlanDev {
    const Level *levels;   // device [n_levels]
    const int32_t *first;  // device [KB_COUNT][n_levels + 1]
    const int32_t *mapx;   // device
    const int32_t *mapy;   // device
    int32_t n_levels;
    int32_t n_bins;
    int32_t channels;
    int32_t n_templates;
    int32_t cell, win_cells_x, win_cells_y, block, norm;
    float eps;                 // L2 epsilon in feature units
    float eps_counts;          // the same in units of the cached cell values
    float vscale;              // feature units per cached cell unit: 1, or 1 / HOG_SOFT_QUANTUM
    int32_t votes;             // HOG_VOTES_HARD or HOG_VOTES_SOFT
    int32_t feat_dim;
    int32_t st_tw, st_th;      // scorer tile (windows)
    int32_t scorer;            // 0: vector units; 1: strips (one template per wave); 2: window GEMM (K >= 16);
                               // 3: raw features on the vector units, 64 windows per workgroup
    int32_t st_waves;          // raw scorer: waves per workgroup (they split the window's cell rows)
    int32_t mfma_ks;           // matrix-core scorers: bin slots per cell (8, 16 or 20)
    int32_t st_lds_bytes;      // scorer dynamic LDS
    int32_t cell_stride;       // floats per staged cell in the scorer's LDS
    int32_t plane_bytes;       // bytes per integral-image element: 4, 2 or 1 (ii mod 2^(8 bytes))
    int32_t bin_chunk;         // bins per integral wave
    int32_t lut_global;        // bin map: 0 the LDS half table, 1 the full table through L2
    int32_t n_chunks;
    int32_t n_cu;              // compute units of the device (persistent grids)
    int64_t tprep_off;         // workspace bytes: prepared template fragments (matrix-core scorer)
    int64_t tprep_stride;      // bytes per template
    int64_t total[KB_COUNT];   // totals (= first[k][n_levels])
};

// Sets the calling thread's hog_last_error() message (hog_api.cpp).
void set_last_error(const char *msg);

// Four-wave workgroups per CU that the bin map's cache-read forms keep
// resident (the full table through L2, or the soft table), from the
// runtime's occupancy calculator, asked once per form. The plan builder asks
// first, so that no launch makes that call under stream capture.
int bin_map_blocks_per_cu(bool soft, int channels);

// Launchers (hog_kernels.hip). Each enqueues one kernel on `stream` and
// returns the launch status.
hipError_t launch_bin_map(const PlanDev &p, const uint8_t *lut_half, const uint8_t *lut_full,
                          const uint8_t *img, int64_t img_pitch, uint8_t *bins, hipStream_t stream);
hipError_t launch_int_reduce(const PlanDev &p, const uint8_t *bins, uint8_t *ws,
                             hipStream_t stream);
// Soft votes: bin map from the uint16 soft table, and the weighted integral
// images (segment totals, their row prefix, one top-down writer per segment).
hipError_t launch_bin_map_soft(const PlanDev &p, const uint16_t *soft_lut, const uint8_t *img,
                               int64_t img_pitch, uint8_t *bins, hipStream_t stream);
// With cells, the writer also fills the cell cache (8-pixel cells only).
hipError_t launch_soft_integral(const PlanDev &p, const uint8_t *bins, uint8_t *ws, uint32_t *ii,
                                bool cells, hipStream_t stream);
// With tmpl (the one-template strip scorer's weights), the launch also runs
// that scorer's template prep, so launch_score can then skip it.
hipError_t launch_int_scan(const PlanDev &p, uint8_t *ws, hipStream_t stream, const float *tmpl = nullptr);
// Whether launch_int_scan runs the template prep for this plan when given tmpl.
bool scan_runs_prep(const PlanDev &p);
hipError_t launch_int_emit(const PlanDev &p, const uint8_t *bins, uint8_t *ws, void *ii,
                           hipStream_t stream);
hipError_t launch_cells(const PlanDev &p, const void *ii, uint8_t *ws, uint32_t *cell_hist,
                        hipStream_t stream);
hipError_t launch_cache_export(const PlanDev &p, const uint8_t *ws, uint32_t *cell_hist,
                               hipStream_t stream);
// The matrix-core scorers' prepared template weights (rewritten in the
// workspace; the vector scorer has none).
hipError_t launch_score_prep(const PlanDev &p, uint8_t *ws, const float *tmpl, hipStream_t stream);
// Window scores; prep = false when launch_score_prep has already run on this
// workspace for these templates.
hipError_t launch_score(const PlanDev &p, const uint8_t *ws, const float *tmpl, const float *bias,
                        float *scores, hipStream_t stream, bool prep = true);
hipError_t launch_block_features(const PlanDev &p, const uint8_t *ws, float *block_feat,
                                 hipStream_t stream);

}  // namespace hogk
