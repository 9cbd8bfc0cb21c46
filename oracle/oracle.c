/*
 * CPU oracle for the fast-HOG hot path.  TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct code written from the paper "A Fast HOG
 * Descriptor Using Lookup Table and Integral Image" (Huang & Huang,
 * arXiv:1703.06256).  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the product path
 * (the HIP library and its binding) never does, and this file shares no
 * code, header, table or constant with it.
 *
 * What it computes, and how it differs from the fast method on purpose:
 *   - bins:      atan2 in FP64 for every pixel (Sec. 2 describes a lookup
 *                table filled with exactly these polar values; the oracle
 *                evaluates the conversion directly instead of tabulating).
 *   - integrals: the recurrence form of Eq. 5 in 64-bit integers, and, for
 *                tiny inputs, the literal double sum of Eq. 5.
 *   - cells:     brute-force counting of the pixels of each area by bin
 *                (the plain definition of the histogram in Sec. 3.2), with
 *                no integral image and no cache.
 *   - features:  per-window concatenation of cell histograms (Sec. 3.1,
 *                Fig. 4), raw or L2-normalised per 2x2-cell block, in FP64.
 *   - scores:    the inner product of Sec. 4, in FP64.
 *
 * Readings of points the paper leaves open (zero gradient and the image
 * border carry no bin, bin 0 starts at +x, colour channel choice, window
 * and block geometry, the L2 form) are listed in the design notes and
 * restated at each function.
 *
 * Parity pins: every function here is pinned by the CPU test suite against
 * exact integer rules, closed forms, invariants or brute force; none is
 * "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NO_BIN 255

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------------- */
/* Sec. 2: orientation bin of one gradient.                               */
/*                                                                        */
/* The angle of (dx, dy) is taken in [0, 2 pi), measured from +x towards  */
/* +y (y is the row index, growing downwards), and split into n_bins      */
/* equal half-open sectors [k 2pi/n, (k+1) 2pi/n); Fig. 2 shows n = 8.    */
/* The magnitude is dropped (unit magnitude, Sec. 2).  A zero gradient    */
/* has no direction and gets no bin.                                      */
/* ---------------------------------------------------------------------- */
int orc_bin(int dx, int dy, int n_bins)
{
    if (n_bins < 1 || n_bins > 64) return -1;
    if (dx == 0 && dy == 0) return ORC_NO_BIN;
    /* Exact sector edges.  An integer gradient points exactly along a      */
    /* multiple of pi/4 only on the axes and the diagonals (by Niven's      */
    /* theorem the tangent of a rational multiple of pi is rational only    */
    /* at 0 and +-1), and only there can the angle sit exactly on a sector  */
    /* edge.  There theta = m pi/4 and the sector is floor(m n / 8), taken  */
    /* in integers: the FP64 product below can round across the edge (for   */
    /* n = 20 at theta = 3 pi/2 it gives 14.999...).                        */
    int m = -1;
    if (dy == 0) m = dx > 0 ? 0 : 4;
    else if (dx == 0) m = dy > 0 ? 2 : 6;
    else if (dx == dy) m = dx > 0 ? 1 : 5;
    else if (dx == -dy) m = dx < 0 ? 3 : 7;
    if (m >= 0) return (m * n_bins) / 8;
    double theta = atan2((double)dy, (double)dx); /* (-pi, pi] */
    if (theta < 0.0) theta += 2.0 * M_PI;           /* [0, 2 pi) */
    int b = (int)floor((theta * (double)n_bins) / (2.0 * M_PI));
    if (b < 0 || b >= n_bins) return -2; /* cannot happen for |dx|,|dy| <= 255 */
    return b;
}

/* ---------------------------------------------------------------------- */
/* Unsigned orientation: the variant Fig. 4's example uses (9 bins over   */
/* 0..180 degrees), where a gradient and its opposite share a bin.  The   */
/* angle is taken mod pi, into [0, pi), and split into n_bins half-open   */
/* sectors [k pi/n, (k+1) pi/n).  On the axes and diagonals the direction */
/* m pi/4 folds to (m mod 4) pi/4, sector floor((m mod 4) n / 4), taken   */
/* in integers for the same reason as above.                              */
/* ---------------------------------------------------------------------- */
int orc_bin_unsigned(int dx, int dy, int n_bins)
{
    if (n_bins < 1 || n_bins > 64) return -1;
    if (dx == 0 && dy == 0) return ORC_NO_BIN;
    int m = -1;
    if (dy == 0) m = 0;                 /* 0 or pi */
    else if (dx == 0) m = 2;            /* pi/2 or 3 pi/2 */
    else if (dx == dy) m = 1;           /* pi/4 or 5 pi/4 */
    else if (dx == -dy) m = 3;          /* 3 pi/4 or 7 pi/4 */
    if (m >= 0) return (m * n_bins) / 4;
    double theta = atan2((double)dy, (double)dx); /* (-pi, pi] */
    if (theta < 0.0) theta += M_PI;                /* [0, pi) */
    int b = (int)floor((theta * (double)n_bins) / M_PI);
    if (b < 0 || b >= n_bins) return -2; /* cannot happen for |dx|,|dy| <= 255 */
    return b;
}

static int orc_bin_oriented(int dx, int dy, int n_bins, int unsigned_orientation)
{
    return unsigned_orientation ? orc_bin_unsigned(dx, dy, n_bins) : orc_bin(dx, dy, n_bins);
}

/* orc_bin (or orc_bin_unsigned) for every (dx, dy) in [-255, 255]^2:     */
/* out[(dy+255)*511 + dx+255].                                            */
int orc_bin_table_ex(int n_bins, int unsigned_orientation, uint8_t *out)
{
    if (n_bins < 1 || n_bins > 64) return -1;
    for (int dy = -255; dy <= 255; ++dy)
        for (int dx = -255; dx <= 255; ++dx)
            out[(dy + 255) * 511 + (dx + 255)] =
                (uint8_t)orc_bin_oriented(dx, dy, n_bins, unsigned_orientation);
    return 0;
}

int orc_bin_table(int n_bins, uint8_t *out) { return orc_bin_table_ex(n_bins, 0, out); }

/* ---------------------------------------------------------------------- */
/* Eq. 1 + Sec. 2: bin map of one image.                                  */
/*                                                                        */
/* img is row-major, channels interleaved: pixel (x, y) channel c is at   */
/* img[y * pitch + x * channels + c]; x is the column (horizontal).       */
/* dx = P[x+1][y] - P[x-1][y], dy = P[x][y+1] - P[x][y-1] per channel.    */
/* With several channels the one with the largest dx^2 + dy^2 gives the   */
/* gradient; equal magnitudes go to the lowest channel index.  The        */
/* one-pixel border, where Eq. 1 has no neighbour, gets no bin.           */
/* out is w*h bytes, row-major, no padding.                               */
/* ---------------------------------------------------------------------- */
int orc_bin_map_ex(const uint8_t *img, int w, int h, int channels, int64_t pitch,
                   int n_bins, int unsigned_orientation, uint8_t *out)
{
    if (w < 1 || h < 1 || channels < 1 || n_bins < 1 || n_bins > 64) return -1;
    for (int y = 0; y < h; ++y) {
        for (int x = 0; x < w; ++x) {
            uint8_t bin = ORC_NO_BIN;
            if (x > 0 && x < w - 1 && y > 0 && y < h - 1) {
                int best = -1, bdx = 0, bdy = 0;
                for (int c = 0; c < channels; ++c) {
                    int right = img[(int64_t)y * pitch + (int64_t)(x + 1) * channels + c];
                    int left  = img[(int64_t)y * pitch + (int64_t)(x - 1) * channels + c];
                    int down  = img[(int64_t)(y + 1) * pitch + (int64_t)x * channels + c];
                    int up    = img[(int64_t)(y - 1) * pitch + (int64_t)x * channels + c];
                    int dx = right - left;
                    int dy = down - up;
                    int mag = dx * dx + dy * dy;
                    if (mag > best) { best = mag; bdx = dx; bdy = dy; }
                }
                if (best > 0) bin = (uint8_t)orc_bin_oriented(bdx, bdy, n_bins, unsigned_orientation);
            }
            out[(int64_t)y * w + x] = bin;
        }
    }
    return 0;
}

int orc_bin_map(const uint8_t *img, int w, int h, int channels, int64_t pitch,
                int n_bins, uint8_t *out)
{
    return orc_bin_map_ex(img, w, h, channels, pitch, n_bins, 0, out);
}

/* ---------------------------------------------------------------------- */
/* Image pyramid (not in the paper; used to score windows at several      */
/* sizes).  Level 0 is the image itself.  Level l >= 1 has scale          */
/* s_l = s_{l-1} * scale (s_0 = 1, repeated FP64 multiplication), size    */
/* floor(w / s_l) x floor(h / s_l), and is kept while l < max_levels      */
/* (max_levels <= 0: no limit) and both sides are at least min_w, min_h.  */
/* Returns the level count; fills lw, lh, ls (caller gives room for cap). */
/* ---------------------------------------------------------------------- */
int orc_pyramid(int w, int h, double scale, int min_w, int min_h, int max_levels,
                int cap, int *lw, int *lh, double *ls)
{
    if (w < 1 || h < 1 || cap < 1) return -1;
    if (!(scale > 1.0) && max_levels != 1) return -1;
    int n = 0;
    double s = 1.0;
    for (;;) {
        if (max_levels > 0 && n >= max_levels) break;
        int lwv = (int)floor((double)w / s);
        int lhv = (int)floor((double)h / s);
        if (n > 0 && (lwv < min_w || lhv < min_h)) break;
        if (n > 0 && (lwv < 1 || lhv < 1)) break;
        if (n >= cap) return -2;
        lw[n] = lwv; lh[n] = lhv; ls[n] = s;
        ++n;
        s = s * scale;
    }
    return n;
}

/* Nearest-neighbour level image: pixel (x, y) of the level copies source  */
/* pixel (min(w-1, floor(x s)), min(h-1, floor(y s))), all channels.      */
/* out is lw*lh*channels bytes, row-major, no padding.                    */
int orc_resize_nn(const uint8_t *img, int w, int h, int channels, int64_t pitch,
                  double s, int lw, int lh, uint8_t *out)
{
    if (w < 1 || h < 1 || lw < 1 || lh < 1 || channels < 1) return -1;
    for (int y = 0; y < lh; ++y) {
        int64_t sy = (int64_t)floor((double)y * s);
        if (sy > h - 1) sy = h - 1;
        for (int x = 0; x < lw; ++x) {
            int64_t sx = (int64_t)floor((double)x * s);
            if (sx > w - 1) sx = w - 1;
            for (int c = 0; c < channels; ++c)
                out[((int64_t)y * lw + x) * channels + c] = img[sy * pitch + sx * channels + c];
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Eq. 4 + Eq. 5: one integral image per bin, by the recurrence           */
/*   ii_n(x,y) = i_n(x,y) + ii_n(x-1,y) + ii_n(x,y-1) - ii_n(x-1,y-1)     */
/* with ii_n(-1, .) = ii_n(., -1) = 0 and i_n(x,y) = [bin(x,y) == n].     */
/* Output layout: out[n][y+1][x+1] = ii_n(x, y); row 0 and column 0 are   */
/* zero.  Shape n_bins x (h+1) x (w+1), uint32.  Sums are formed in       */
/* 64-bit and then stored; every value is at most w*h.                    */
/* ---------------------------------------------------------------------- */
int orc_integral(const uint8_t *bins, int w, int h, int n_bins, uint32_t *out)
{
    if (w < 1 || h < 1 || n_bins < 1 || n_bins > 64) return -1;
    const int64_t W1 = (int64_t)w + 1, H1 = (int64_t)h + 1;
    uint64_t *prev = (uint64_t *)calloc((size_t)W1, sizeof(uint64_t));
    uint64_t *cur = (uint64_t *)calloc((size_t)W1, sizeof(uint64_t));
    if (!prev || !cur) { free(prev); free(cur); return -3; }
    for (int n = 0; n < n_bins; ++n) {
        uint32_t *plane = out + (int64_t)n * H1 * W1;
        memset(prev, 0, (size_t)W1 * sizeof(uint64_t));
        for (int64_t c = 0; c < W1; ++c) plane[c] = 0;
        for (int y = 0; y < h; ++y) {
            cur[0] = 0;
            for (int x = 0; x < w; ++x) {
                uint64_t one = (bins[(int64_t)y * w + x] == n) ? 1u : 0u;
                cur[x + 1] = one + cur[x] + prev[x + 1] - prev[x];
            }
            for (int64_t c = 0; c < W1; ++c) plane[(int64_t)(y + 1) * W1 + c] = (uint32_t)cur[c];
            uint64_t *t = prev; prev = cur; cur = t;
        }
    }
    free(prev); free(cur);
    return 0;
}

/* Eq. 5 written out literally: ii_n(x,y) = sum over x' <= x, y' <= y of   */
/* i_n(x', y').  O(w^2 h^2) per bin: tiny inputs only.  Same layout as     */
/* orc_integral.                                                           */
int orc_integral_literal(const uint8_t *bins, int w, int h, int n_bins, uint32_t *out)
{
    if (w < 1 || h < 1 || n_bins < 1 || n_bins > 64) return -1;
    if ((int64_t)w * h > 64 * 64) return -1;
    const int64_t W1 = (int64_t)w + 1, H1 = (int64_t)h + 1;
    for (int n = 0; n < n_bins; ++n) {
        uint32_t *plane = out + (int64_t)n * H1 * W1;
        for (int64_t c = 0; c < W1; ++c) plane[c] = 0;
        for (int y = 0; y < h; ++y) {
            plane[(int64_t)(y + 1) * W1] = 0;
            for (int x = 0; x < w; ++x) {
                uint32_t s = 0;
                for (int yp = 0; yp <= y; ++yp)
                    for (int xp = 0; xp <= x; ++xp)
                        s += (bins[(int64_t)yp * w + xp] == n) ? 1u : 0u;
                plane[(int64_t)(y + 1) * W1 + x + 1] = s;
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Sec. 3.2: histogram of one area, by counting.  Cells are cell x cell   */
/* squares anchored at the image origin; cell (cx, cy) covers columns     */
/* [cx*cell, cx*cell+cell) and rows [cy*cell, cy*cell+cell).  There are   */
/* floor(w/cell) x floor(h/cell) whole cells; a partial strip at the      */
/* right or bottom belongs to no cell.  Pixels with no bin are not        */
/* counted.  out[cy][cx][n], uint32.                                      */
/* ---------------------------------------------------------------------- */
int orc_cell_hist(const uint8_t *bins, int w, int h, int n_bins, int cell, uint32_t *out)
{
    if (w < 1 || h < 1 || n_bins < 1 || n_bins > 64 || cell < 1) return -1;
    const int wc = w / cell, hc = h / cell;
    for (int cy = 0; cy < hc; ++cy)
        for (int cx = 0; cx < wc; ++cx) {
            uint32_t *hist = out + ((int64_t)cy * wc + cx) * n_bins;
            for (int n = 0; n < n_bins; ++n) hist[n] = 0;
            for (int y = cy * cell; y < cy * cell + cell; ++y)
                for (int x = cx * cell; x < cx * cell + cell; ++x) {
                    uint8_t b = bins[(int64_t)y * w + x];
                    if (b != ORC_NO_BIN) hist[b] += 1;
                }
        }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Soft votes.  Sec. 2 notes that OpenCV shares each pixel's vote between */
/* two bins, and that the paper keeps to one bin per pixel because the    */
/* shared vote does not fit the one-hot decomposition.  The variant here  */
/* quantises the shared vote so that integral images stay exact: with t   */
/* the angle (signed [0, 2 pi) or unsigned [0, pi)), the bin width        */
/* range / n and a = t / width - 1/2, the pixel gives                      */
/*     w1 = floor(frac(a) * ORC_SOFT_Q + 1/2)                              */
/* units to bin (floor(a) + 1) mod n and ORC_SOFT_Q - w1 to floor(a) mod n */
/* (ORC_SOFT_Q units = one pixel).  On the axes and diagonals t / width   */
/* is the rational m n / 8 (signed) or (m mod 4) n / 4 (unsigned), and a  */
/* is taken in integers there; elsewhere a is FP64.                        */
/* ---------------------------------------------------------------------- */
#define ORC_SOFT_Q 32

int orc_soft_vote(int dx, int dy, int n_bins, int unsigned_orientation, int *b0, int *w1)
{
    if (n_bins < 1 || n_bins > 64 || !b0 || !w1) return -1;
    if (dx == 0 && dy == 0) { *b0 = ORC_NO_BIN; *w1 = 0; return ORC_NO_BIN; }
    int m = -1;
    if (dy == 0) m = dx > 0 ? 0 : 4;
    else if (dx == 0) m = dy > 0 ? 2 : 6;
    else if (dx == dy) m = dx > 0 ? 1 : 5;
    else if (dx == -dy) m = dx < 0 ? 3 : 7;
    long fl;
    double frac_q; /* frac(a) * ORC_SOFT_Q */
    if (m >= 0) {
        /* a * den = num exactly */
        const long den = unsigned_orientation ? 4 : 8;
        const long num = unsigned_orientation ? (long)(m % 4) * n_bins - 2 : (long)m * n_bins - 4;
        fl = num >= 0 ? num / den : -((-num + den - 1) / den);
        frac_q = (double)((num - fl * den) * ORC_SOFT_Q) / (double)den;
    } else {
        double t = atan2((double)dy, (double)dx);
        const double range = unsigned_orientation ? M_PI : 2.0 * M_PI;
        if (t < 0.0) t += range;
        const double a = (t * (double)n_bins) / range - 0.5;
        const double f = floor(a);
        fl = (long)f;
        frac_q = (a - f) * ORC_SOFT_Q;
    }
    *b0 = (int)(((fl % n_bins) + n_bins) % n_bins);
    *w1 = (int)floor(frac_q + 0.5);
    return 0;
}

/* The soft vote of every (dx, dy) in [-255, 255]^2, as b0 and w1 tables. */
int orc_soft_table(int n_bins, int unsigned_orientation, uint8_t *b0_out, uint8_t *w1_out)
{
    if (n_bins < 1 || n_bins > 64) return -1;
    for (int dy = -255; dy <= 255; ++dy)
        for (int dx = -255; dx <= 255; ++dx) {
            int b0, w1;
            orc_soft_vote(dx, dy, n_bins, unsigned_orientation, &b0, &w1);
            b0_out[(dy + 255) * 511 + (dx + 255)] = (uint8_t)b0;
            w1_out[(dy + 255) * 511 + (dx + 255)] = (uint8_t)w1;
        }
    return 0;
}

/* Eq. 1 and the channel choice as in orc_bin_map, then the soft vote.    */
int orc_soft_bin_map(const uint8_t *img, int w, int h, int channels, int64_t pitch, int n_bins,
                     int unsigned_orientation, uint8_t *b0_out, uint8_t *w1_out)
{
    if (w < 1 || h < 1 || channels < 1 || n_bins < 1 || n_bins > 64) return -1;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int b0 = ORC_NO_BIN, w1 = 0;
            if (x > 0 && x < w - 1 && y > 0 && y < h - 1) {
                int best = -1, bdx = 0, bdy = 0;
                for (int c = 0; c < channels; ++c) {
                    int dx = img[(int64_t)y * pitch + (int64_t)(x + 1) * channels + c] -
                             img[(int64_t)y * pitch + (int64_t)(x - 1) * channels + c];
                    int dy = img[(int64_t)(y + 1) * pitch + (int64_t)x * channels + c] -
                             img[(int64_t)(y - 1) * pitch + (int64_t)x * channels + c];
                    int mag = dx * dx + dy * dy;
                    if (mag > best) { best = mag; bdx = dx; bdy = dy; }
                }
                if (best > 0) orc_soft_vote(bdx, bdy, n_bins, unsigned_orientation, &b0, &w1);
            }
            b0_out[(int64_t)y * w + x] = (uint8_t)b0;
            w1_out[(int64_t)y * w + x] = (uint8_t)w1;
        }
    return 0;
}

/* The votes pixel (x, y) gives bin n, in units of 1 / ORC_SOFT_Q.         */
static uint32_t soft_votes_for(const uint8_t *b0, const uint8_t *w1, int64_t i, int n, int n_bins)
{
    if (b0[i] == ORC_NO_BIN) return 0;
    const int lo = b0[i], hi = (b0[i] + 1) % n_bins;
    uint32_t v = 0;
    if (lo == n) v += ORC_SOFT_Q - w1[i];
    if (hi == n) v += w1[i];
    return v;
}

/* Eq. 5 over the soft votes: out[n][y+1][x+1] = sum of bin n's votes over */
/* x' <= x, y' <= y (64-bit running sums; guard row and column are 0).     */
int orc_soft_integral(const uint8_t *b0, const uint8_t *w1, int w, int h, int n_bins, uint32_t *out)
{
    if (w < 1 || h < 1 || n_bins < 1 || n_bins > 64) return -1;
    const int64_t W1 = w + 1, plane = W1 * (h + 1);
    for (int n = 0; n < n_bins; ++n) {
        uint32_t *P = out + n * plane;
        for (int x = 0; x <= w; ++x) P[x] = 0;
        for (int y = 0; y < h; ++y) {
            uint64_t row = 0;
            P[(y + 1) * W1] = 0;
            for (int x = 0; x < w; ++x) {
                row += soft_votes_for(b0, w1, (int64_t)y * w + x, n, n_bins);
                P[(y + 1) * W1 + x + 1] = (uint32_t)(P[y * W1 + x + 1] + row);
            }
        }
    }
    return 0;
}

/* Brute-force vote sums of every cell, in units of 1 / ORC_SOFT_Q.        */
int orc_soft_cell_hist(const uint8_t *b0, const uint8_t *w1, int w, int h, int n_bins, int cell,
                       uint32_t *out)
{
    if (w < 1 || h < 1 || n_bins < 1 || n_bins > 64 || cell < 1) return -1;
    const int wc = w / cell, hc = h / cell;
    for (int cy = 0; cy < hc; ++cy)
        for (int cx = 0; cx < wc; ++cx) {
            uint32_t *hist = out + ((int64_t)cy * wc + cx) * n_bins;
            for (int n = 0; n < n_bins; ++n) {
                uint32_t sum = 0;
                for (int y = cy * cell; y < cy * cell + cell; ++y)
                    for (int x = cx * cell; x < cx * cell + cell; ++x)
                        sum += soft_votes_for(b0, w1, (int64_t)y * w + x, n, n_bins);
                hist[n] = sum;
            }
        }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Sec. 3.1 / Fig. 4: feature of one detection window.                    */
/*                                                                        */
/* The window has its top-left corner at pixel (wx*cell, wy*cell) and     */
/* covers wcx x wcy cells (windows step by one cell).  Its cell           */
/* histograms are counted afresh here, pixel by pixel (no integral image, */
/* no cache).  norm == 0 (raw): the feature is the cell histograms in     */
/* row-major cell order, f[(cy*wcx + cx)*n_bins + n].  norm == 1 (L2):    */
/* the window is covered by block x block-cell blocks stepping one cell,  */
/* (wcx-block+1) x (wcy-block+1) of them; each block's vector v (its      */
/* cells in row-major order, each cell's n_bins counts) becomes           */
/*   v / sqrt(sum v^2 + eps^2)                                            */
/* and the feature is f[((by*nbx + bx)*block^2 + (v*block + u))*n_bins+n] */
/* with (u, v) the cell inside the block.  FP64 throughout.               */
/* Returns the feature length, or < 0 on bad arguments.                   */
/* ---------------------------------------------------------------------- */
int orc_feature_dim(int n_bins, int wcx, int wcy, int block, int norm)
{
    if (n_bins < 1 || wcx < 1 || wcy < 1) return -1;
    if (norm == 0) return wcx * wcy * n_bins;
    if (norm != 1 || block < 1 || block > wcx || block > wcy) return -1;
    return (wcx - block + 1) * (wcy - block + 1) * block * block * n_bins;
}

int orc_window_feature(const uint8_t *bins, int w, int h, int n_bins, int cell,
                       int wcx, int wcy, int block, int norm, double eps,
                       int wx, int wy, double *f)
{
    const int dim = orc_feature_dim(n_bins, wcx, wcy, block, norm);
    if (dim < 0 || cell < 1 || wx < 0 || wy < 0) return -1;
    if ((wx + wcx) * cell > w || (wy + wcy) * cell > h) return -1;
    uint32_t *cnt = (uint32_t *)calloc((size_t)wcx * wcy * n_bins, sizeof(uint32_t));
    if (!cnt) return -3;
    for (int cy = 0; cy < wcy; ++cy)
        for (int cx = 0; cx < wcx; ++cx) {
            uint32_t *hist = cnt + ((int64_t)cy * wcx + cx) * n_bins;
            const int x0 = (wx + cx) * cell, y0 = (wy + cy) * cell;
            for (int y = y0; y < y0 + cell; ++y)
                for (int x = x0; x < x0 + cell; ++x) {
                    uint8_t b = bins[(int64_t)y * w + x];
                    if (b != ORC_NO_BIN) hist[b] += 1;
                }
        }
    if (norm == 0) {
        for (int i = 0; i < dim; ++i) f[i] = (double)cnt[i];
    } else {
        const int nbx = wcx - block + 1, nby = wcy - block + 1;
        for (int by = 0; by < nby; ++by)
            for (int bx = 0; bx < nbx; ++bx) {
                double ss = 0.0;
                for (int v = 0; v < block; ++v)
                    for (int u = 0; u < block; ++u)
                        for (int n = 0; n < n_bins; ++n) {
                            double c = (double)cnt[((int64_t)(by + v) * wcx + (bx + u)) * n_bins + n];
                            ss += c * c;
                        }
                const double inv = 1.0 / sqrt(ss + eps * eps);
                double *fb = f + ((int64_t)(by * nbx + bx) * block * block) * n_bins;
                for (int v = 0; v < block; ++v)
                    for (int u = 0; u < block; ++u)
                        for (int n = 0; n < n_bins; ++n)
                            fb[(v * block + u) * n_bins + n] =
                                (double)cnt[((int64_t)(by + v) * wcx + (bx + u)) * n_bins + n] * inv;
            }
    }
    free(cnt);
    return dim;
}

/* Window grid: windows whose wcx x wcy cells lie inside the image.        */
int orc_window_grid(int w, int h, int cell, int wcx, int wcy, int *nwx, int *nwy)
{
    if (w < 1 || h < 1 || cell < 1 || wcx < 1 || wcy < 1) return -1;
    int a = w / cell - wcx + 1, b = h / cell - wcy + 1;
    *nwx = a > 0 ? a : 0;
    *nwy = b > 0 ? b : 0;
    if (*nwx == 0 || *nwy == 0) { *nwx = 0; *nwy = 0; }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Sec. 4: objectness by inner product.  For each listed window and each  */
/* template k: s_k = bias_k + sum_d tmpl[k][d] * f[d], in FP64 (the       */
/* FP32 template values are widened exactly).  scores[i*k_n + k];         */
/* feats (optional) receives each window's feature, feats[i*dim + d];     */
/* absterms (optional) receives |bias_k| + sum_d |tmpl[k][d] f[d]|, the   */
/* scale against which a score's rounding error is judged.                */
/* ---------------------------------------------------------------------- */
int orc_score_windows(const uint8_t *bins, int w, int h, int n_bins, int cell,
                      int wcx, int wcy, int block, int norm, double eps,
                      const float *tmpl, const float *bias, int k_n,
                      int n_win, const int *wxs, const int *wys,
                      double *scores, double *feats, double *absterms)
{
    const int dim = orc_feature_dim(n_bins, wcx, wcy, block, norm);
    if (dim < 0 || k_n < 1) return -1;
    double *f = (double *)malloc((size_t)dim * sizeof(double));
    if (!f) return -3;
    for (int i = 0; i < n_win; ++i) {
        int r = orc_window_feature(bins, w, h, n_bins, cell, wcx, wcy, block, norm, eps,
                                   wxs[i], wys[i], f);
        if (r < 0) { free(f); return r; }
        if (feats) memcpy(feats + (int64_t)i * dim, f, (size_t)dim * sizeof(double));
        for (int k = 0; k < k_n; ++k) {
            const float *t = tmpl + (int64_t)k * dim;
            double s = (double)bias[k], a = fabs((double)bias[k]);
            for (int d = 0; d < dim; ++d) {
                double p = (double)t[d] * f[d];
                s += p;
                a += fabs(p);
            }
            scores[(int64_t)i * k_n + k] = s;
            if (absterms) absterms[(int64_t)i * k_n + k] = a;
        }
    }
    free(f);
    return 0;
}
