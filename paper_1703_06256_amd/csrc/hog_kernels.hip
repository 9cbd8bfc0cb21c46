// gfx950 kernels of the fast-HOG path (arXiv:1703.06256).
//
// Every kernel covers all pyramid levels of a plan in one launch: each
// level owns a contiguous range of the launch's waves, workgroups or
// threads (the plan's per-kernel prefix table `first`), and a wave finds
// its level by a binary search over that table.
//
//   k_bin_map         Eq. 1 + Sec. 2    gradients, channel choice, table lookup
//   k_int_reduce      Eq. 5 (pass 1)    per-tile row and column bin counts
//   k_int_scan_rows   Eq. 5 (pass 2)    row carries from the tiles on the left
//   k_int_scan_cols   Eq. 5 (pass 2)    plane row just above every tile row
//   k_int_emit        Eq. 4 + Eq. 5     one-hot in registers, write the planes
//   k_cells           Eq. 6, Sec. 3.3   four-corner cell histograms, cached
//   k_score           Sec. 3.1, Sec. 4  window features and inner products
//   k_block_features  (optional output) normalised block vectors
#include "hog_internal.h"

namespace hogk {
namespace {

__device__ __forceinline__ int wave_id_in_block()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// Largest l with first[l] <= g (levels with no items are skipped).
__device__ __forceinline__ int find_level(const int32_t *__restrict__ first, int n, int g)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ float inv_block_norm(float ss, float eps)
{
    // v / sqrt(|v|^2 + eps^2): the sum of squares of integer counts is exact
    // in FP32 (at most 16 * cell^4 <= 2^24); sqrt and the reciprocal round.
    return 1.0f / sqrtf(ss + eps * eps);
}

// ---------------------------------------------------------------------------
// Eq. 1 + Sec. 2: bin map. A wave owns level columns x0-1 .. x0+62 (lane L
// is column x0-1+L) and kBinRows rows. Each lane reads one sample per row
// (the nearest-neighbour source pixel of its column); left and right come
// from the adjacent lanes, up and down from the previous and next row kept
// in registers. Lanes 1..62 write bins.
// ---------------------------------------------------------------------------
template <int C>
__global__ __launch_bounds__(256) void k_bin_map(const Level *__restrict__ lv,
                                                 const int32_t *__restrict__ first, int n_levels,
                                                 const int32_t *__restrict__ mapx,
                                                 const int32_t *__restrict__ mapy,
                                                 const uint8_t *__restrict__ img, int64_t pitch,
                                                 const uint8_t *__restrict__ lut,
                                                 uint8_t *__restrict__ bins)
{
    const int wave = (int)blockIdx.x * 4 + wave_id_in_block();
    const int lane = threadIdx.x & 63;
    if (wave >= first[n_levels]) return;
    const int l = find_level(first, n_levels, wave);
    const Level &v = lv[l];
    const int W = v.w, H = v.h;
    const int t = wave - first[l];
    const int gx = t % v.bm_gx, gy = t / v.bm_gx;
    const int x = gx * kBinCols - 1 + lane;
    const bool col_ok = x >= 0 && x < W;
    const int32_t *my = mapy + v.mapy_off;
    const uint8_t *colp = img + (int64_t)(col_ok ? mapx[v.mapx_off + x] : 0) * C;

    auto sample = [&](int r) -> uint32_t {
        if (!col_ok || r < 0 || r >= H) return 0u;
        const uint8_t *p = colp + (int64_t)my[r] * pitch;
        if constexpr (C == 1) {
            return p[0];
        } else {
            return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16);
        }
    };

    const int y0 = gy * kBinRows;
    const int y1 = min(y0 + kBinRows, H);
    uint32_t up = sample(y0 - 1);
    uint32_t cur = sample(y0);
    uint8_t *out = bins + v.bins_off + x;
    const bool writer = lane >= 1 && lane <= kBinCols && col_ok;
    const bool col_interior = x >= 1 && x <= W - 2;
    for (int y = y0; y < y1; ++y) {
        const uint32_t down = sample(y + 1);
        const uint32_t left = __shfl_up(cur, 1u);
        const uint32_t right = __shfl_down(cur, 1u);
        uint8_t b = (uint8_t)kNoBin;
        if (col_interior && y >= 1 && y <= H - 2) {
            int best = 0, bdx = 0, bdy = 0;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int dx = (int)((right >> (8 * c)) & 255u) - (int)((left >> (8 * c)) & 255u);
                const int dy = (int)((down >> (8 * c)) & 255u) - (int)((up >> (8 * c)) & 255u);
                const int m = dx * dx + dy * dy;
                if (m > best) { best = m; bdx = dx; bdy = dy; }  // ties keep the lower channel
            }
            if (best > 0) b = lut[(bdy + 255) * 511 + (bdx + 255)];
        }
        if (writer) out[(int64_t)y * v.bins_pitch] = b;
        up = cur;
        cur = down;
    }
}

// ---------------------------------------------------------------------------
// Eq. 5, pass 1. Tile (tx, ty): padded columns [64 tx, 64 tx + 64), padded
// rows [TH ty, TH ty + TH); padded (r, c) holds pixel (c-1, r-1), and row 0
// / column 0 hold nothing. For the wave's chunk of bins, count per tile row
// (a ballot per bin) and per column (registers).
// ---------------------------------------------------------------------------
template <int NBC>
__global__ __launch_bounds__(256) void k_int_reduce(const Level *__restrict__ lv,
                                                    const int32_t *__restrict__ first, int n_levels,
                                                    int nb, const uint8_t *__restrict__ bins,
                                                    uint8_t *__restrict__ ws)
{
    const int tile = (int)blockIdx.x * 4 + wave_id_in_block();
    const int lane = threadIdx.x & 63;
    if (tile >= first[n_levels]) return;
    const int l = find_level(first, n_levels, tile);
    const Level &v = lv[l];
    const int t = tile - first[l];
    const int tx = t % v.tiles_x, ty = t / v.tiles_x;
    const int b0 = (int)blockIdx.y * NBC;
    const int nbh = min(NBC, nb - b0);
    const int c = tx * kIntTileCols + lane;
    const int x = c - 1;
    const bool cin = x >= 0 && x < v.w;
    const int r0 = ty * kIntTileRows, r1 = min(r0 + kIntTileRows, v.h + 1);
    const uint8_t *bcol = bins + v.bins_off + x;
    uint8_t *rowtot = ws + v.ws_rowtot + (int64_t)tx * (v.h + 1) * nb + b0;

    uint32_t colcnt[NBC];
#pragma unroll
    for (int j = 0; j < NBC; ++j) colcnt[j] = 0;

    for (int r = r0; r < r1; ++r) {
        const int y = r - 1;
        const int bin = (cin && y >= 0) ? (int)bcol[(int64_t)y * v.bins_pitch] : kNoBin;
        const int rel = bin - b0;
        uint32_t mine = 0;
#pragma unroll
        for (int j = 0; j < NBC; ++j) {
            if (j < nbh) {
                const bool hit = rel == j;
                colcnt[j] += hit ? 1u : 0u;
                const uint32_t cnt = (uint32_t)__popcll(__ballot(hit));
                mine = (lane == j) ? cnt : mine;
            }
        }
        if (lane < nbh) rowtot[(int64_t)r * nb + lane] = (uint8_t)mine;
    }
    if (c <= v.w) {
        uint8_t *coltot = ws + v.ws_coltot + ((int64_t)ty * nb + b0) * (v.w + 1) + c;
#pragma unroll
        for (int j = 0; j < NBC; ++j)
            if (j < nbh) coltot[(int64_t)j * (v.w + 1)] = (uint8_t)colcnt[j];
    }
}

// Eq. 5, pass 2a: for every padded row r and bin n, the number of n-pixels
// of row r in the tiles left of tile column tx (exclusive scan over tx).
__global__ __launch_bounds__(256) void k_int_scan_rows(const Level *__restrict__ lv,
                                                       const int32_t *__restrict__ first,
                                                       int n_levels, int nb,
                                                       uint8_t *__restrict__ ws)
{
    const int g = (int)(blockIdx.x * 256 + threadIdx.x);
    if (g >= first[n_levels]) return;
    const int l = find_level(first, n_levels, g);
    const Level &v = lv[l];
    const int rel = g - first[l];  // r * nb + n
    const int64_t stride = (int64_t)(v.h + 1) * nb;
    const uint8_t *rt = ws + v.ws_rowtot + rel;
    uint32_t *e = reinterpret_cast<uint32_t *>(ws + v.ws_e) + rel;
    uint32_t acc = 0;
    for (int tx = 0; tx < v.tiles_x; ++tx) {
        e[tx * stride] = acc;
        acc += rt[tx * stride];
    }
}

// Eq. 5, pass 2b: for tile row ty and bin n, the plane row just above the
// tile row, T(c) = ii at padded row TH ty - 1, padded column c: the inclusive
// prefix over c of the column counts of all tile rows above.
__global__ __launch_bounds__(256) void k_int_scan_cols(const Level *__restrict__ lv,
                                                       const int32_t *__restrict__ first,
                                                       int n_levels, int nb,
                                                       uint8_t *__restrict__ ws)
{
    const int wg = (int)blockIdx.x;
    if (wg >= first[n_levels]) return;
    const int l = find_level(first, n_levels, wg);
    const Level &v = lv[l];
    const int rel = wg - first[l];
    const int ty = rel / nb, n = rel % nb;
    const int W1 = v.w + 1;
    const uint8_t *ct = ws + v.ws_coltot + (int64_t)n * W1;
    const int64_t ct_stride = (int64_t)nb * W1;
    uint32_t *T = reinterpret_cast<uint32_t *>(ws + v.ws_t) + ((int64_t)ty * nb + n) * W1;
    __shared__ uint32_t wsum[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int base = 0; base < W1; base += 256) {
        const int c = base + (int)threadIdx.x;
        uint32_t a = 0;
        if (c < W1)
            for (int k = 0; k < ty; ++k) a += ct[k * ct_stride + c];
        uint32_t s = a;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(s, (unsigned)d);
            if (lane >= d) s += o;
        }
        if (lane == 63) wsum[wv] = s;
        __syncthreads();
        uint32_t off = carry;
        for (int k = 0; k < wv; ++k) off += wsum[k];
        const uint32_t tot = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        if (c < W1) T[c] = off + s;
        carry += tot;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Eq. 4 + Eq. 5, pass 3. Each lane owns one padded column of the tile and
// keeps, per bin of the wave's chunk, the running plane value of its column
// in a register, seeded with the plane row above the tile. Per row: the
// one-hot image of Eq. 4 is a ballot per bin, its inclusive prefix along the
// row is a masked popcount (mbcnt), the row carry of the tiles on the left
// is added, and the running value is stored: ii(r, c) = ii(r-1, c) + R(r, c).
// ---------------------------------------------------------------------------
template <int NBC>
__global__ __launch_bounds__(256) void k_int_emit(const Level *__restrict__ lv,
                                                  const int32_t *__restrict__ first, int n_levels,
                                                  int nb, const uint8_t *__restrict__ bins,
                                                  const uint8_t *__restrict__ ws,
                                                  uint32_t *__restrict__ ii)
{
    const int tile = (int)blockIdx.x * 4 + wave_id_in_block();
    const int lane = threadIdx.x & 63;
    if (tile >= first[n_levels]) return;
    const int l = find_level(first, n_levels, tile);
    const Level &v = lv[l];
    const int t = tile - first[l];
    const int tx = t % v.tiles_x, ty = t / v.tiles_x;
    const int b0 = (int)blockIdx.y * NBC;
    const int nbh = min(NBC, nb - b0);
    const int c = tx * kIntTileCols + lane;
    const int x = c - 1;
    const bool cin = x >= 0 && x < v.w;
    const int W1 = v.w + 1;
    const bool cst = c < W1;
    const int r0 = ty * kIntTileRows, r1 = min(r0 + kIntTileRows, v.h + 1);

    const uint32_t *T = reinterpret_cast<const uint32_t *>(ws + v.ws_t) +
                        ((int64_t)ty * nb + b0) * W1 + c;
    uint32_t run[NBC];
#pragma unroll
    for (int j = 0; j < NBC; ++j) run[j] = (j < nbh && cst) ? T[(int64_t)j * W1] : 0u;

    const uint32_t *E = reinterpret_cast<const uint32_t *>(ws + v.ws_e) +
                        (int64_t)tx * (v.h + 1) * nb + b0;
    uint32_t *out = ii + v.ii_off + (int64_t)b0 * v.ii_plane + c;
    const uint8_t *bcol = bins + v.bins_off + x;

    for (int r = r0; r < r1; ++r) {
        const int y = r - 1;
        const int bin = (cin && y >= 0) ? (int)bcol[(int64_t)y * v.bins_pitch] : kNoBin;
        const int rel = bin - b0;
        const uint32_t *Er = E + (int64_t)r * nb;
        uint32_t *orow = out + (int64_t)r * v.ii_pitch;
#pragma unroll
        for (int j = 0; j < NBC; ++j) {
            if (j < nbh) {
                const bool hit = rel == j;
                const uint64_t m = __ballot(hit);
                const uint32_t pre = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                run[j] += Er[j] + pre + (hit ? 1u : 0u);
                if (cst) orow[(int64_t)j * v.ii_plane] = run[j];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Eq. 6 + Sec. 3.3: the histogram of cell (cx, cy) is, on each bin's plane,
// P(r1, c1) + P(r0, c0) - P(r0, c1) - P(r1, c0) with (r0, c0) = cell * (cy, cx)
// and (r1, c1) = (r0, c0) + cell in padded coordinates. Computed once per
// cell and cached (uint16, [bin][cy][cx]) for every window that uses it.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cells(const Level *__restrict__ lv,
                                               const int32_t *__restrict__ first, int n_levels,
                                               int nb, int cell, const uint32_t *__restrict__ ii,
                                               uint8_t *__restrict__ ws,
                                               uint32_t *__restrict__ cell_hist)
{
    const int g = (int)(blockIdx.x * 256 + threadIdx.x);
    if (g >= first[n_levels]) return;
    const int l = find_level(first, n_levels, g);
    const Level &v = lv[l];
    const int rel = g - first[l];
    const int cy = rel / v.cells_x, cx = rel % v.cells_x;
    const uint32_t *P = ii + v.ii_off;
    const int64_t r0 = (int64_t)cy * cell * v.ii_pitch;
    const int64_t r1 = r0 + (int64_t)cell * v.ii_pitch;
    const int64_t c0 = (int64_t)cx * cell, c1 = c0 + cell;
    const int64_t cstride = (int64_t)v.cells_x * v.cells_y;
    uint16_t *cache = reinterpret_cast<uint16_t *>(ws + v.ws_cache) + rel;
    uint32_t *ch = cell_hist ? cell_hist + v.cell_off + (int64_t)rel * nb : nullptr;
    for (int n = 0; n < nb; ++n) {
        const uint32_t *p = P + (int64_t)n * v.ii_plane;
        const uint32_t h = p[r1 + c1] + p[r0 + c0] - p[r0 + c1] - p[r1 + c0];
        cache[n * cstride] = (uint16_t)h;
        if (ch) ch[n] = h;
    }
}

struct ScoreArgs {
    int nb, wcx, wcy, norm, k, dim, tw, th, nbp;
    float eps;
};

// Load one staged cell (nb floats at hp) into registers.
template <int NB>
__device__ __forceinline__ void load_cell(const float *hp, float (&h)[NB])
{
#pragma unroll
    for (int b = 0; b < NB; ++b) h[b] = hp[b];
}

template <int NB>
__device__ __forceinline__ float dot_acc(const float *__restrict__ w, const float (&h)[NB], float g)
{
#pragma unroll
    for (int b = 0; b < NB; ++b) g = fmaf(w[b], h[b], g);
    return g;
}

// ---------------------------------------------------------------------------
// Sec. 3.1 / Fig. 4 + Sec. 4: window scores. A workgroup scores a tile of
// tw x th windows of one level; it stages the (tw+wcx-1) x (th+wcy-1) cells
// they use from the cache into LDS as floats (plus, for L2, each block's
// 1/sqrt(|v|^2 + eps^2)); each thread then scores one window.
//
// L2 (block 2, window 8 cells wide): the thread walks the window's cell rows
// q; a cell at (q, qx) belongs to the blocks (q-1|q, qx-1|qx); each block
// gathers its 4*nb products in one FP32 accumulator, is scaled by its
// inverse norm when its second cell row is done, and added in FP64.
// Raw: each cell's nb products form one FP32 partial, added in FP64.
// ---------------------------------------------------------------------------
template <int NB, int WCX>
__global__ __launch_bounds__(256) void k_score(const Level *__restrict__ lv,
                                               const int32_t *__restrict__ first, int n_levels,
                                               ScoreArgs a, const uint8_t *__restrict__ ws,
                                               const float *__restrict__ tmpl,
                                               const float *__restrict__ bias,
                                               float *__restrict__ scores)
{
    extern __shared__ float lds[];
    const int wg = (int)blockIdx.x;
    if (wg >= first[n_levels]) return;
    const int l = find_level(first, n_levels, wg);
    const Level &v = lv[l];
    const int rel = wg - first[l];
    const int stx = rel % v.st_x, sty = rel / v.st_x;
    const int wx0 = stx * a.tw, wy0 = sty * a.th;
    const int nb = NB > 0 ? NB : a.nb;
    const int nbp = a.nbp;
    const int wcx = WCX > 0 ? WCX : a.wcx;
    const int CW = a.tw + wcx - 1, CH = a.th + a.wcy - 1;
    float *hc = lds;
    float *inv = lds + (int64_t)CH * CW * nbp;

    // Stage the tile's cells (zero outside the level's cell grid).
    const uint16_t *cache = reinterpret_cast<const uint16_t *>(ws + v.ws_cache);
    const int64_t cstride = (int64_t)v.cells_x * v.cells_y;
    const int total = CH * CW * nb;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        const int j = i % CW;
        const int rest = i / CW;
        const int r = rest % CH, n = rest / CH;
        const int cy = wy0 + r, cx = wx0 + j;
        float val = 0.f;
        if (cy < v.cells_y && cx < v.cells_x)
            val = (float)cache[n * cstride + (int64_t)cy * v.cells_x + cx];
        hc[(r * CW + j) * nbp + n] = val;
    }
    __syncthreads();
    if (a.norm == 1) {
        const int BW = CW - 1, BH = CH - 1;
        for (int i = threadIdx.x; i < BW * BH; i += blockDim.x) {
            const int j = i % BW, r = i / BW;
            float ss = 0.f;
            for (int vv = 0; vv < 2; ++vv)
                for (int uu = 0; uu < 2; ++uu) {
                    const float *hp = hc + ((r + vv) * CW + j + uu) * nbp;
                    for (int n = 0; n < nb; ++n) ss = fmaf(hp[n], hp[n], ss);
                }
            inv[i] = inv_block_norm(ss, a.eps);
        }
        __syncthreads();
    }

    const int tx = (int)threadIdx.x % a.tw, ty = (int)threadIdx.x / a.tw;
    const int wx = wx0 + tx, wy = wy0 + ty;
    if (ty >= a.th || wx >= v.win_x || wy >= v.win_y) return;
    float *sout = scores + v.score_off + ((int64_t)wy * v.win_x + wx) * a.k;

    for (int k = 0; k < a.k; ++k) {
        const float *T = tmpl + (int64_t)k * a.dim;
        double s = (double)bias[k];
        if (a.norm == 1) {
            if constexpr (NB > 0 && WCX > 0) {
                constexpr int NBX = WCX - 1;
                float gp[NBX], gc[NBX];
#pragma unroll
                for (int bx = 0; bx < NBX; ++bx) { gp[bx] = 0.f; gc[bx] = 0.f; }
                const int wcy = a.wcy;
                for (int q = 0; q < wcy; ++q) {
                    const bool has_prev = q >= 1, has_cur = q < wcy - 1;
#pragma unroll
                    for (int qx = 0; qx < WCX; ++qx) {
                        float h[NB];
                        load_cell<NB>(hc + ((ty + q) * CW + tx + qx) * nbp, h);
                        // block (q-1, qx-1): v=1,u=1; (q-1, qx): v=1,u=0;
                        // block (q, qx-1): v=0,u=1;   (q, qx):   v=0,u=0.
                        if (has_prev) {
                            if (qx >= 1)
                                gp[qx - 1] = dot_acc<NB>(T + (((q - 1) * NBX + qx - 1) * 4 + 3) * NB, h, gp[qx - 1]);
                            if (qx < NBX)
                                gp[qx] = dot_acc<NB>(T + (((q - 1) * NBX + qx) * 4 + 2) * NB, h, gp[qx]);
                        }
                        if (has_cur) {
                            if (qx >= 1)
                                gc[qx - 1] = dot_acc<NB>(T + ((q * NBX + qx - 1) * 4 + 1) * NB, h, gc[qx - 1]);
                            if (qx < NBX)
                                gc[qx] = dot_acc<NB>(T + ((q * NBX + qx) * 4 + 0) * NB, h, gc[qx]);
                        }
                    }
                    if (has_prev) {
                        const float *ip = inv + (ty + q - 1) * (CW - 1) + tx;
#pragma unroll
                        for (int bx = 0; bx < NBX; ++bx) s += (double)(gp[bx] * ip[bx]);
                    }
#pragma unroll
                    for (int bx = 0; bx < NBX; ++bx) { gp[bx] = gc[bx]; gc[bx] = 0.f; }
                }
            } else {
                // Generic bins / window width: the same sums, block by block.
                const int nbx = wcx - 1, nby = a.wcy - 1;
                for (int by = 0; by < nby; ++by)
                    for (int bx = 0; bx < nbx; ++bx) {
                        float g = 0.f;
                        for (int vv = 0; vv < 2; ++vv)
                            for (int uu = 0; uu < 2; ++uu) {
                                const float *hp = hc + ((ty + by + vv) * CW + tx + bx + uu) * nbp;
                                const float *w = T + ((by * nbx + bx) * 4 + vv * 2 + uu) * nb;
                                for (int n = 0; n < nb; ++n) g = fmaf(w[n], hp[n], g);
                            }
                        s += (double)(g * inv[(ty + by) * (CW - 1) + tx + bx]);
                    }
            }
        } else {
            for (int q = 0; q < a.wcy; ++q)
                for (int qx = 0; qx < wcx; ++qx) {
                    const float *hp = hc + ((ty + q) * CW + tx + qx) * nbp;
                    const float *w = T + (q * wcx + qx) * nb;
                    float g = 0.f;
                    for (int n = 0; n < nb; ++n) g = fmaf(w[n], hp[n], g);
                    s += (double)g;
                }
        }
        sout[k] = (float)s;
    }
}

// Optional output: every normalised 2x2 block, f = h / sqrt(|v|^2 + eps^2).
__global__ __launch_bounds__(256) void k_block_features(const Level *__restrict__ lv,
                                                        const int32_t *__restrict__ first,
                                                        int n_levels, int nb, float eps,
                                                        const uint8_t *__restrict__ ws,
                                                        float *__restrict__ out)
{
    const int g = (int)(blockIdx.x * 256 + threadIdx.x);
    if (g >= first[n_levels]) return;
    const int l = find_level(first, n_levels, g);
    const Level &v = lv[l];
    const int rel = g - first[l];
    const int bw = v.cells_x - 1;
    const int by = rel / bw, bx = rel % bw;
    const uint16_t *cache = reinterpret_cast<const uint16_t *>(ws + v.ws_cache);
    const int64_t cstride = (int64_t)v.cells_x * v.cells_y;
    float ss = 0.f;
    for (int vv = 0; vv < 2; ++vv)
        for (int uu = 0; uu < 2; ++uu)
            for (int n = 0; n < nb; ++n) {
                const float h = (float)cache[n * cstride + (int64_t)(by + vv) * v.cells_x + bx + uu];
                ss = fmaf(h, h, ss);
            }
    const float iv = inv_block_norm(ss, eps);
    float *o = out + v.block_off + (int64_t)rel * 4 * nb;
    for (int vv = 0; vv < 2; ++vv)
        for (int uu = 0; uu < 2; ++uu)
            for (int n = 0; n < nb; ++n) {
                const float h = (float)cache[n * cstride + (int64_t)(by + vv) * v.cells_x + bx + uu];
                o[(vv * 2 + uu) * nb + n] = h * iv;
            }
}

inline unsigned blocks_for(int64_t items, int per_block)
{
    return (unsigned)((items + per_block - 1) / per_block);
}

inline const int32_t *first_of(const PlanDev &p, int k)
{
    return p.first + (int64_t)k * (p.n_levels + 1);
}

}  // namespace

hipError_t launch_bin_map(const PlanDev &p, const uint8_t *lut, const uint8_t *img,
                          int64_t img_pitch, uint8_t *bins, hipStream_t stream)
{
    const int64_t waves = p.total[KB_BINMAP];
    if (waves == 0) return hipSuccess;
    const dim3 grid(blocks_for(waves, 4));
    if (p.channels == 1)
        hipLaunchKernelGGL(k_bin_map<1>, grid, dim3(256), 0, stream, p.levels,
                           first_of(p, KB_BINMAP), p.n_levels, p.mapx, p.mapy, img, img_pitch,
                           lut, bins);
    else
        hipLaunchKernelGGL(k_bin_map<3>, grid, dim3(256), 0, stream, p.levels,
                           first_of(p, KB_BINMAP), p.n_levels, p.mapx, p.mapy, img, img_pitch,
                           lut, bins);
    return hipGetLastError();
}

#define HOG_CHUNK_DISPATCH(KERNEL, GRID, STREAM, ...)                                           \
    switch (p.bin_chunk) {                                                                      \
    case 1: hipLaunchKernelGGL(KERNEL<1>, GRID, dim3(256), 0, STREAM, __VA_ARGS__); break;      \
    case 2: hipLaunchKernelGGL(KERNEL<2>, GRID, dim3(256), 0, STREAM, __VA_ARGS__); break;      \
    case 3: hipLaunchKernelGGL(KERNEL<3>, GRID, dim3(256), 0, STREAM, __VA_ARGS__); break;      \
    case 4: hipLaunchKernelGGL(KERNEL<4>, GRID, dim3(256), 0, STREAM, __VA_ARGS__); break;      \
    case 5: hipLaunchKernelGGL(KERNEL<5>, GRID, dim3(256), 0, STREAM, __VA_ARGS__); break;      \
    case 6: hipLaunchKernelGGL(KERNEL<6>, GRID, dim3(256), 0, STREAM, __VA_ARGS__); break;      \
    case 7: hipLaunchKernelGGL(KERNEL<7>, GRID, dim3(256), 0, STREAM, __VA_ARGS__); break;      \
    case 8: hipLaunchKernelGGL(KERNEL<8>, GRID, dim3(256), 0, STREAM, __VA_ARGS__); break;      \
    case 9: hipLaunchKernelGGL(KERNEL<9>, GRID, dim3(256), 0, STREAM, __VA_ARGS__); break;      \
    default: return hipErrorInvalidValue;                                                        \
    }

hipError_t launch_int_reduce(const PlanDev &p, const uint8_t *bins, uint8_t *ws, hipStream_t stream)
{
    const int64_t tiles = p.total[KB_ITILE];
    if (tiles == 0) return hipSuccess;
    const dim3 grid(blocks_for(tiles, 4), (unsigned)p.n_chunks);
    HOG_CHUNK_DISPATCH(k_int_reduce, grid, stream, p.levels, first_of(p, KB_ITILE), p.n_levels,
                       p.n_bins, bins, ws);
    return hipGetLastError();
}

hipError_t launch_int_scan_rows(const PlanDev &p, uint8_t *ws, hipStream_t stream)
{
    const int64_t n = p.total[KB_ESCAN];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_int_scan_rows, dim3(blocks_for(n, 256)), dim3(256), 0, stream, p.levels,
                       first_of(p, KB_ESCAN), p.n_levels, p.n_bins, ws);
    return hipGetLastError();
}

hipError_t launch_int_scan_cols(const PlanDev &p, uint8_t *ws, hipStream_t stream)
{
    const int64_t n = p.total[KB_TSCAN];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_int_scan_cols, dim3((unsigned)n), dim3(256), 0, stream, p.levels,
                       first_of(p, KB_TSCAN), p.n_levels, p.n_bins, ws);
    return hipGetLastError();
}

hipError_t launch_int_emit(const PlanDev &p, const uint8_t *bins, const uint8_t *ws, uint32_t *ii,
                           hipStream_t stream)
{
    const int64_t tiles = p.total[KB_ITILE];
    if (tiles == 0) return hipSuccess;
    const dim3 grid(blocks_for(tiles, 4), (unsigned)p.n_chunks);
    HOG_CHUNK_DISPATCH(k_int_emit, grid, stream, p.levels, first_of(p, KB_ITILE), p.n_levels,
                       p.n_bins, bins, ws, ii);
    return hipGetLastError();
}

hipError_t launch_cells(const PlanDev &p, const uint32_t *ii, uint8_t *ws, uint32_t *cell_hist,
                        hipStream_t stream)
{
    const int64_t n = p.total[KB_CELL];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cells, dim3(blocks_for(n, 256)), dim3(256), 0, stream, p.levels,
                       first_of(p, KB_CELL), p.n_levels, p.n_bins, p.cell, ii, ws, cell_hist);
    return hipGetLastError();
}

hipError_t launch_score(const PlanDev &p, const uint8_t *ws, const float *tmpl, const float *bias,
                        float *scores, hipStream_t stream)
{
    const int64_t n = p.total[KB_STILE];
    if (n == 0) return hipSuccess;
    ScoreArgs a;
    a.nb = p.n_bins;
    a.wcx = p.win_cells_x;
    a.wcy = p.win_cells_y;
    a.norm = p.norm;
    a.k = p.n_templates;
    a.dim = p.feat_dim;
    a.tw = p.st_tw;
    a.th = p.st_th;
    a.nbp = p.cell_stride;
    a.eps = p.eps;
    const dim3 grid((unsigned)n), block(256);
    const size_t lds = (size_t)p.st_lds_bytes;
    const int32_t *f = first_of(p, KB_STILE);
    const bool w8 = p.win_cells_x == 8 && p.norm == 1;
    if (w8 && p.n_bins == 8)
        hipLaunchKernelGGL((k_score<8, 8>), grid, block, lds, stream, p.levels, f, p.n_levels, a,
                           ws, tmpl, bias, scores);
    else if (w8 && p.n_bins == 9)
        hipLaunchKernelGGL((k_score<9, 8>), grid, block, lds, stream, p.levels, f, p.n_levels, a,
                           ws, tmpl, bias, scores);
    else if (w8 && p.n_bins == 18)
        hipLaunchKernelGGL((k_score<18, 8>), grid, block, lds, stream, p.levels, f, p.n_levels, a,
                           ws, tmpl, bias, scores);
    else
        hipLaunchKernelGGL((k_score<0, 0>), grid, block, lds, stream, p.levels, f, p.n_levels, a,
                           ws, tmpl, bias, scores);
    return hipGetLastError();
}

hipError_t launch_block_features(const PlanDev &p, const uint8_t *ws, float *block_feat,
                                 hipStream_t stream)
{
    const int64_t n = p.total[KB_BLOCK];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_block_features, dim3(blocks_for(n, 256)), dim3(256), 0, stream, p.levels,
                       first_of(p, KB_BLOCK), p.n_levels, p.n_bins, p.eps, ws, block_feat);
    return hipGetLastError();
}

}  // namespace hogk
