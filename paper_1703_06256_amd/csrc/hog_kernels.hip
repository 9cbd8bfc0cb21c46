// gfx950 kernels of the fast-HOG path (arXiv:1703.06256).
//
// Every kernel covers all pyramid levels of a plan in one launch: each
// level owns a contiguous range of the launch's waves, workgroups or
// threads (the plan's per-kernel prefix table `first`), and a wave finds
// its level by a binary search over that table.
//
//   k_bin_map         Eq. 1 + Sec. 2    gradients, channel choice, table lookup
//                                       (hard bins, or soft-vote entries)
//   k_int_reduce      Eq. 5 (pass 1)    per-tile row, column and total bin counts
//   k_int_scan        Eq. 5 (pass 2)    carries: row counts left of each tile, column
//                                       counts above it, counts above-left of it
//   k_int_emit        Eq. 4 + Eq. 5     one-hot in registers, write the planes
//                                       (uint32, or uint16 / uint8 mod 2^bits)
//   k_soft_reduce,    Eq. 5, soft votes per-tile row and column vote totals, their
//   k_soft_scan,                        prefixes, and the weighted planes written
//   k_soft_emit                         once (with the cell cache for 8-pixel cells)
//   k_cells           Eq. 6, Sec. 3.3   four-corner cell histograms, cached
//   k_score           Sec. 3.1, Sec. 4  window features and inner products (vector units)
//   k_score_prep,     Sec. 3.1, Sec. 4  the same on the matrix cores: one template per
//   k_score_strip                       wave over strips of windows (K < 16)
//   k_score_prep_wg*, Sec. 3.1, Sec. 4  windows x templates GEMM, 32 templates per
//   k_score_wgemm                       workgroup (K >= 16)
//   k_block_features  (optional output) normalised block vectors
#include "hog.h"
#include "hog_internal.h"

#define HOG_MAX_BINS_K 64

#include <algorithm>
#include <type_traits>

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

// base + byte_off, where base is wave-uniform and byte_off a 32-bit per-lane
// byte offset: lets loads and stores use the scalar-base addressing form.
template <class T>
__device__ __forceinline__ T *at_byte(T *base, uint32_t byte_off)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ const T *at_byte(const T *base, uint32_t byte_off)
{
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Raw buffer resource over [base, base + bytes): gfx9 descriptor word 3.
// Accesses outside the range read 0 and drop writes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}

// Cell histogram cache (uint16): 8 x 8-cell blocks, block (bx, by) of bin n
// at ((n * cby + by) * cbx + bx) * 64, cell (cx, cy) at (cy % 8) * 8 + cx % 8
// within its block. With 8-pixel cells a block is one integral tile.
__device__ __forceinline__ int64_t cache_index(const Level &v, int n, int cy, int cx)
{
    return (((int64_t)n * v.cby + (cy >> 3)) * v.cbx + (cx >> 3)) * 64 + ((cy & 7) << 3) + (cx & 7);
}

__device__ __forceinline__ float inv_block_norm(float ss, float eps)
{
    // v / sqrt(|v|^2 + eps^2): the sum of squares of integer counts is exact
    // in FP32 (at most 16 * cell^4 <= 2^24); sqrt and the reciprocal round.
    return 1.0f / sqrtf(ss + eps * eps);
}

// Lane i receives lane i-1's value (wave_shr:1) / lane i+1's (wave_shl:1);
// the lanes at the wave's ends keep their own value.
__device__ __forceinline__ uint32_t from_left_lane(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t from_right_lane(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x130, 0xF, 0xF, false);
}

// ---------------------------------------------------------------------------
// Eq. 1 + Sec. 2: bin map. The lookup table lives in LDS as its dy >= 0 half
// (kLutHalfBytes): entry (dx, |dy|) holds bin(dx, |dy|) in bits 0..5 and, in
// bit 6, f with bin(dx, -|dy|) = n - 1 - bin(dx, |dy|) + f (f = 1 exactly
// when the mirrored direction lies on a sector edge); 255 marks (0, 0).
// A persistent workgroup of 16 waves per CU loads the half table once, then
// each wave walks bin-map items: level columns x0-1 .. x0+62 (lane L is
// column x0-1+L) by kBinRows rows. Each lane reads one sample per row, the
// nearest-neighbour source pixel of its column (all channels in one dword);
// left and right neighbours come from the adjacent lanes, up and down from
// the rows above and below. All samples are loaded first, then every lookup
// is made, then lanes 1..62 store their bins.
// ---------------------------------------------------------------------------
//
// Soft votes (SOFT): the same walk; the lookup is the uint16 soft-table
// entry b0 | w1 << 8 (522 KB, read through L2; no LDS table), stored as two
// bytes per pixel.
//
// GLUT: the hard-vote lookup reads the full 511 x 511 table (261 KB) through
// the L1/L2 caches instead of the LDS half table (no staging and no LDS, so
// smaller workgroups, several per CU); the plan picks one
// (hog_tiles.lut_global).
// Occupancy: the soft RGB form, held to 6 waves per SIMD (at most 80 VGPRs,
// no spills), ran faster than at the 5 its default allocation gives (94.5
// against 95.6 us over the 1920 x 1080 pyramid's levels).
template <int C, bool SOFT, bool GLUT = false>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(SOFT && C == 3 ? 6 : 1))) void k_bin_map(const Level *__restrict__ lv,
                                                  const int32_t *__restrict__ first, int n_levels,
                                                  const int32_t *__restrict__ mapx,
                                                  const int32_t *__restrict__ mapy,
                                                  const uint8_t *__restrict__ img, int64_t call_pitch,
                                                  int nb,
                                                  const uint8_t *__restrict__ lut_half,
                                                  const uint16_t *__restrict__ soft,
                                                  uint8_t *__restrict__ bins)
{
    const uint8_t *lut = nullptr;
    // The table read through the caches (GLUT: the full 511 x 511 bytes,
    // passed as lut_half; SOFT: 511 x 511 uint16 entries) by buffer loads of
    // the entry's offset. Unused with the LDS half table.
    const __amdgpu_buffer_rsrc_t trsrc =
        SOFT ? buffer_rsrc(soft, 2 * kLutEntries) : buffer_rsrc(lut_half, kLutEntries);
    if constexpr (!SOFT && !GLUT) {
        __shared__ __attribute__((aligned(16))) uint8_t lut_lds[kLutHalfBytes];
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const u32x4 *src = reinterpret_cast<const u32x4 *>(lut_half);
        u32x4 *dst = reinterpret_cast<u32x4 *>(lut_lds);
        for (int i = threadIdx.x; i < kLutHalfBytes / 16; i += blockDim.x) dst[i] = src[i];
        __syncthreads();
        lut = lut_lds;
    }

    const int lane = threadIdx.x & 63;
    const int n_items = first[n_levels];
    const int waves_per_block = (int)(blockDim.x >> 6);
    // Wave w of workgroup b starts at item w * grid + b: each round of
    // grid x waves items spreads over every workgroup, so the last, partial
    // round adds at most one item to each wave of every CU rather than a
    // whole round to the first CUs.
    for (int item = wave_id_in_block() * (int)gridDim.x + (int)blockIdx.x; item < n_items;
         item += (int)gridDim.x * waves_per_block) {
        const int l = find_level(first, n_levels, item);
        const Level &v = lv[l];
        const int W = v.w, H = v.h;
        const int t = item - first[l];
        const int gx = t % v.bm_gx, gy = t / v.bm_gx;
        const int src_w = v.src_w;
        const int64_t pitch = v.src_pitch > 0 ? v.src_pitch : call_pitch;
        const int x = gx * kBinCols - 1 + lane;
        const bool col_ok = x >= 0 && x < W;
        const int32_t *my = mapy + v.mapy_off;
        const int y0 = gy * kBinRows;
        if (C == 3 && src_w < 2) {  // wave-uniform: a 1-pixel-wide image has no interior
            if (lane >= 1 && lane <= kBinCols && col_ok)
                for (int i = 0; i < kBinRows && y0 + i < H; ++i) {
                    if constexpr (SOFT)
                        *reinterpret_cast<uint16_t *>(bins + v.bins_off + (int64_t)(y0 + i) * v.bins_pitch + 2 * x) =
                            (uint16_t)kNoBin;
                    else
                        bins[v.bins_off + (int64_t)(y0 + i) * v.bins_pitch + x] = (uint8_t)kNoBin;
                }
            continue;
        }
        // Every lane and row loads from a clamped, valid position, so the
        // loads carry no condition and are all in flight at once. Samples
        // outside the level (clamped copies) reach only pixels off the
        // level's interior, which take no bin whatever they hold.
        const int sx = mapx[v.mapx_off + min(max(x, 0), W - 1)];
        // Byte offset of the sample in a source row; for RGB a 4-byte read that
        // stays inside the row (it starts one byte early at the last column).
        int64_t coff = sx;
        uint32_t shift = 0;
        if constexpr (C == 3) {
            const bool last = sx >= src_w - 1;
            coff = last ? 3 * (int64_t)sx - 1 : 3 * (int64_t)sx;
            shift = last ? 8u : 0u;
        }
        // The source image through one buffer descriptor (its byte extent,
        // below 2^32, is checked on the host): the lane's column offset in
        // the vector operand, the row's offset in the scalar one, so no
        // per-lane 64-bit address arithmetic.
        const __amdgpu_buffer_rsrc_t isrc =
            buffer_rsrc(img + v.src_off, (uint32_t)((int64_t)(v.src_h - 1) * pitch + (int64_t)src_w * C));
        const int coff32 = (int)(uint32_t)coff;

        uint32_t smp[kBinRows + 2];
#pragma unroll
        for (int i = 0; i < kBinRows + 2; ++i) {
            const int r = min(max(y0 - 1 + i, 0), H - 1);
            const int roff = (int)(uint32_t)((int64_t)my[r] * pitch);
            if constexpr (C == 1)
                smp[i] = __builtin_amdgcn_raw_buffer_load_b8(isrc, coff32, roff, 0);
            else
                smp[i] = __builtin_amdgcn_raw_buffer_load_b32(isrc, coff32, roff, 0);
        }
        if constexpr (C == 3) {
#pragma unroll
            for (int i = 0; i < kBinRows + 2; ++i) smp[i] = (smp[i] >> shift) & 0xFFFFFFu;
        }
        const bool col_interior = x >= 1 && x <= W - 2;
        typedef typename std::conditional<SOFT, uint16_t, uint8_t>::type bin_t;
        bin_t b[kBinRows];
#pragma unroll
        for (int i = 0; i < kBinRows; ++i) {
            const int y = y0 + i;
            const uint32_t up = smp[i], cur = smp[i + 1], down = smp[i + 2];
            const uint32_t left = from_left_lane(cur), right = from_right_lane(cur);
            // Channel 0 seeds the choice unconditionally (m = 0 only when
            // dx = dy = 0, the same as no choice at all).
            int bdx = (int)(right & 255u) - (int)(left & 255u);
            int bdy = (int)(down & 255u) - (int)(up & 255u);
            int best = bdx * bdx + bdy * bdy;
#pragma unroll
            for (int c = 1; c < C; ++c) {
                const int dx = (int)((right >> (8 * c)) & 255u) - (int)((left >> (8 * c)) & 255u);
                const int dy = (int)((down >> (8 * c)) & 255u) - (int)((up >> (8 * c)) & 255u);
                const int m = dx * dx + dy * dy;
                if (m > best) { best = m; bdx = dx; bdy = dy; }  // ties keep the lower channel
            }
            const bool ok = col_interior && y >= 1 && y <= H - 2 && best > 0;
            if constexpr (SOFT) {
                const uint16_t e = __builtin_amdgcn_raw_buffer_load_b16(
                    trsrc, (2 * ((bdy + 255) * 511 + (bdx + 255))) & -(int)ok, 0, 0);
                b[i] = ok ? e : (uint16_t)kNoBin;
            } else if constexpr (GLUT) {
                const uint8_t e = __builtin_amdgcn_raw_buffer_load_b8(trsrc, ((bdy + 255) * 511 + (bdx + 255)) & -(int)ok, 0, 0);
                b[i] = ok ? e : (uint8_t)kNoBin;
            } else {
                const int ady = bdy < 0 ? -bdy : bdy;
                // Index 0 for lanes with no bin, by a mask rather than a
                // select the compiler turns into a branch per row (whose
                // exec masks then spill).
                const uint32_t e = lut[(ady * 511 + (bdx + 255)) & -(int)ok];
                const uint32_t half_bin = e & 63u;
                const uint32_t bin = bdy < 0 ? (uint32_t)(nb - 1) - half_bin + (e >> 6) : half_bin;
                b[i] = ok ? (uint8_t)bin : (uint8_t)kNoBin;
            }
        }
        const bool writer = lane >= 1 && lane <= kBinCols && col_ok;
        const __amdgpu_buffer_rsrc_t bsrc = buffer_rsrc(bins + v.bins_off, (uint32_t)(v.bins_pitch * H));
        // Lanes that store nothing take an offset beyond the buffer, so their
        // stores are dropped without a branch; rows past the level are left
        // out by a scalar test, only in the last item of a column.
        const int xw = writer ? x * (int)sizeof(bin_t) : (int)0x80000000u;
        auto store = [&](int i) {
            if constexpr (SOFT)
                __builtin_amdgcn_raw_buffer_store_b16(b[i], bsrc, xw, (y0 + i) * (int)v.bins_pitch, 0);
            else
                __builtin_amdgcn_raw_buffer_store_b8(b[i], bsrc, xw, (y0 + i) * (int)v.bins_pitch, 0);
        };
        if (y0 + kBinRows <= H) {
#pragma unroll
            for (int i = 0; i < kBinRows; ++i) store(i);
        } else {
#pragma unroll
            for (int i = 0; i < kBinRows; ++i)
                if (y0 + i < H) store(i);  // wave-uniform
        }
    }
}

// Stage the kTile x kTile bins of tile (tx, ty) into this wave's LDS slice
// (row-major, kTile bytes per row): 4 x 16-byte loads per lane. Rows past
// the level's height read as 0 (outside the buffer range); columns past its
// width are masked by the caller.
__device__ __forceinline__ void stage_bin_tile(uint8_t *tb, __amdgpu_buffer_rsrc_t bsrc, int bpitch,
                                               int tx, int y0, int lane)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int k = lane + 64 * m;
        const int row = k >> 2, seg = k & 3;
        const u32x4 d = __builtin_amdgcn_raw_buffer_load_b128(bsrc, (y0 + row) * bpitch + tx * kTile + 16 * seg, 0, 0);
        *reinterpret_cast<u32x4 *>(tb + row * kTile + 16 * seg) = d;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Compiler-only ordering point for wave-private LDS traffic.
__device__ __forceinline__ void lds_order()
{
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// Inclusive prefix sum over the 64 lanes of a full wave, by DPP: shifts of
// 1, 2, 4 and 8 lanes inside each row of 16 (zero fill), then the last lane
// of row 0 (row 2) added to row 1 (row 3), then the last lane of row 1 added
// to rows 2 and 3. Every lane must be active.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// ---------------------------------------------------------------------------
// Integral images (Eq. 4 + Eq. 5) over pixel tiles of kTile x kTile: tile
// (tx, ty) holds pixels [64 tx, 64 tx + 64) x [64 ty, 64 ty + 64), lane L on
// pixel column 64 tx + L.
//
// Pass 1 (k_int_reduce): per tile, the count of each bin in each of its rows,
// in each of its columns, and in the whole tile.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_int_reduce(const Level *__restrict__ lv,
                                                   const int32_t *__restrict__ first, int n_levels,
                                                   int nb, const uint8_t *__restrict__ bins,
                                                   uint8_t *__restrict__ ws)
{
    // One wave per tile, every bin at once. LDS: the tile's bins (row stride
    // kRedStride bytes, 17 dwords, so lane-per-row reads hit distinct banks),
    // then per-lane histograms colh and rowh: each lane only ever adds to its
    // own slots. A count never exceeds 64, so four bins share a dword, one
    // byte each (bin n: dword n / 4, byte n % 4), which halves the LDS and
    // lets more tiles run at once.
    constexpr int kRedStride = 68;
    extern __shared__ __attribute__((aligned(16))) uint32_t red_smem[];
    const int tile = (int)blockIdx.x;
    const int lane = (int)threadIdx.x;
    if (tile >= first[n_levels]) return;
    const int l = find_level(first, n_levels, tile);
    const Level &v = lv[l];
    const int t = tile - first[l];
    const int tx = t % v.tiles_x, ty = t / v.tiles_x;
    uint8_t *tb = reinterpret_cast<uint8_t *>(red_smem);
    const int nw = (nb + 3) >> 2;  // dwords per lane and histogram
    // Each histogram has one more slot, never read: pixels with no bin, and
    // rows or columns outside the level, add there, so that every add is
    // unconditional (no branch around each atomic).
    uint32_t *colh = red_smem + kTile * kRedStride / 4;
    uint32_t *rowh = colh + (nw + 1) * 64;
    for (int n = 0; n < nw; ++n) {
        colh[n * 64 + lane] = 0u;
        rowh[n * 64 + lane] = 0u;
    }
    // Bins below nb: dword b / 4; no bin (255): the spare slot nw.
    auto slot = [nw](int b) { return min(b >> 2, nw) * 64; };
    auto one = [](int b) { return 1u << (8 * (b & 3)); };
    {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const __amdgpu_buffer_rsrc_t bsrc = buffer_rsrc(bins + v.bins_off, (uint32_t)(v.bins_pitch * v.h));
        const int bpitch = (int)v.bins_pitch;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int k = lane + 64 * m;
            const int row = k >> 2, seg = k & 3;
            const u32x4 d = __builtin_amdgcn_raw_buffer_load_b128(
                bsrc, (ty * kTile + row) * bpitch + tx * kTile + 16 * seg, 0, 0);
            uint32_t *dst = reinterpret_cast<uint32_t *>(tb + row * kRedStride + 16 * seg);
            dst[0] = d[0];
            dst[1] = d[1];
            dst[2] = d[2];
            dst[3] = d[3];
        }
    }
    // Byte 64 of row 0 is stride padding, never staged: kNoBin there serves
    // the pixels outside the level, read by address rather than through a
    // select on the loaded value (which the compiler turns into a branch).
    constexpr int kNoBinByte = kTile;
    if (lane == 0) tb[kNoBinByte] = (uint8_t)kNoBin;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int y0 = ty * kTile, nrows = min(kTile, v.h - y0);
    const int x = tx * kTile + lane;
    const bool xin = x < v.w;
    const int ncols = min(kTile, v.w - tx * kTile);
    // FULL: the whole tile lies inside the level (most tiles), so no pixel
    // needs a test.
    auto counts = [&](auto full_c) {
        constexpr bool FULL = decltype(full_c)::value;
        // Column counts: lane = column. Each batch of 16 bins is read before
        // its adds: the compiler keeps LDS reads and atomics in program
        // order, so a read after an add would wait for the add's round trip.
        for (int r0 = 0; r0 < (FULL ? kTile : nrows); r0 += 16) {
            int bb[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                if constexpr (FULL)
                    bb[i] = tb[(r0 + i) * kRedStride + lane];
                else
                    bb[i] = tb[xin & (r0 + i < nrows) ? (r0 + i) * kRedStride + lane : kNoBinByte];
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) atomicAdd(&colh[slot(bb[i]) + lane], one(bb[i]));
        }
        // Row counts: lane = row; its 64 bins are read first, 16 at a time.
        const uint32_t *rp = reinterpret_cast<const uint32_t *>(tb + lane * kRedStride);
        for (int k0 = 0; k0 < kTile / 4; k0 += 4) {
            uint32_t d[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) d[k] = rp[k0 + k];
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = 4 * (k0 + k) + e;
                    const int raw = (int)((d[k] >> (8 * e)) & 255u);
                    const int b = FULL ? raw : ((lane < nrows) & (c < ncols) ? raw : kNoBin);
                    atomicAdd(&rowh[slot(b) + lane], one(b));
                }
        }
    };
    if (nrows == kTile && ncols == kTile)
        counts(std::true_type{});
    else
        counts(std::false_type{});
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // rowtot [tx][n][hp], lane = row (rows below the level are not
    // written); coltot [ty][n][wp], lane = column (0 right of the level);
    // tiletot [ty][tx][n]. Each histogram dword (four bins) is read once,
    // and the stores go through buffer descriptors with the bin's offset in
    // the scalar operand; lanes with nothing to store take an offset past
    // the range.
    const uint32_t hp = kTile * v.tiles_y, wp = kTile * v.tiles_x;
    const __amdgpu_buffer_rsrc_t rts = buffer_rsrc(ws + v.ws_rowtot + (int64_t)tx * nb * hp + y0, (uint32_t)nb * hp);
    const __amdgpu_buffer_rsrc_t cts = buffer_rsrc(ws + v.ws_coltot + (int64_t)ty * nb * wp + tx * kTile, (uint32_t)nb * wp);
    const __amdgpu_buffer_rsrc_t tts =
        buffer_rsrc(ws + v.ws_tiletot + ((int64_t)ty * v.tiles_x + tx) * nb * 4, (uint32_t)nb * 4u);
    const int rvo = lane < nrows ? lane : (int)0x80000000u;
    for (int k = 0; k < nw; ++k) {
        const uint32_t rs = rowh[k * 64 + lane], cs = colh[k * 64 + lane];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (4 * k + e < nb) {  // wave-uniform
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(rs >> (8 * e)), rts, rvo, (4 * k + e) * (int)hp, 0);
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(cs >> (8 * e)), cts, lane, (4 * k + e) * (int)wp, 0);
            }
        // The four bins' tile totals: sums over the 64 columns of bytes 0
        // and 2, and of bytes 1 and 3, in 16-bit halves (at most 4096 each).
        const uint32_t lo = wave_incl_scan(cs & 0x00FF00FFu), hi = wave_incl_scan((cs >> 8) & 0x00FF00FFu);
        const uint32_t tl = (uint32_t)__builtin_amdgcn_readlane((int)lo, 63);
        const uint32_t th = (uint32_t)__builtin_amdgcn_readlane((int)hi, 63);
        const uint32_t tot = (((lane & 1) ? th : tl) >> (16 * (lane >> 1))) & 0xFFFFu;
        __builtin_amdgcn_raw_buffer_store_b32(tot, tts, (lane < 4) & (4 * k + lane < nb) ? 4 * (4 * k + lane) : (int)0x80000000u,
                                              0, 0);
    }
}

// ---------------------------------------------------------------------------
// Template weights for the matrix-core scorers (Sec. 4 inner product): their
// modes and, for the strip scorer, the prep of each template into B
// fragments (run by k_score_prep, or beside the carries by k_int_scan).
// ---------------------------------------------------------------------------
// Matrix-core scorer modes, per template (strips) or per tile of 32
// templates (window GEMM): fp16 hi + lo weights (the strips), the same with
// the lo halves scaled by 2^11 and the counts they multiply by 2^-11 (the
// window GEMM), or FP32 weights (either).
enum { kModeSplit = 0, kModeExact = 1, kModeWide = 2 };

struct StripArgs {
    int nb, nby, k, th, dim, lds_wave;
    int64_t tprep_off, tprep_stride;
    float eps;
};

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));

template <int NBP>
struct StripShape {
    static constexpr int K32 = (4 * NBP) / 32;         // 16x16x32 steps per block
    static constexpr int K16 = ((4 * NBP) % 32) / 16;  // 16x16x16 steps (0 or 1)
    static constexpr int S = K32 + K16;                // prepared fragments per (bx, hi|lo)
    static_assert(4 * NBP == 32 * K32 + 16 * K16, "bin padding must fill the steps");
};

// Feature k of a block (cell order w, u; NBP slots per cell) -> template
// element of block position (n, bx), or -1 for a padding slot / n >= nby.
__device__ __forceinline__ int strip_weight_index(int k, int nbp, int nb, int nby, int n, int bx)
{
    const int w = k / (2 * nbp), rem = k % (2 * nbp);
    const int u = rem / nbp, bin = rem % nbp;
    if (n >= nby || bin >= nb) return -1;
    return ((n * kStripMaxBX + bx) * 4 + w * 2 + u) * nb + bin;
}

// Template prep, one workgroup per template: the B fragments of every step
// and block column bx, in the layout the strip kernel loads: slots
// [bx][i][lane] of 16 bytes (i < NBP / 4), then the column scales [lane]
// (float), then the template's mode (int).
// kModeSplit: column n (block row offset) gets one power of two for all its
// bx, bringing its max |T| into [2^14, 2^15), and each scaled weight sv is
// split into fp16 hi = sv rounded and lo = (sv - hi) rounded; slot 2 j holds
// the hi and slot 2 j + 1 the lo halves of 16x16x32 step j, and the 16x16x16
// step (if any) is slot 2 K32, hi in its low and lo in its high 8 bytes.
// hi + lo holds sv to 2^-22 relative when |sv| >= 2^-3; below that lo is an
// fp16 subnormal and loses bits. So if any nonzero weight of the template
// scales below 2^-3 (its column also holds weights about 2^17 times larger),
// the template takes kModeExact instead: its FP32 weights unscaled, slot i
// holding the weights of bins 4 i .. 4 i + 3 of cell q = lane / 16 of the
// block (the 16x16x4 FP32 products' layout), and scale 1.
//
// The prep of template kk by the W waves of a workgroup, wave w taking the
// block columns bx = w, w + W, ... (k_score_prep: W = kStripMaxBX; the carry
// scan's prep workgroups: W = 8, the last wave idle; one column each). colmax,
// need_exact and wbuf (W x kStripPrepRows x 4 NBP floats) are the
// workgroup's LDS.
constexpr int kStripPrepRows = 16;  // block row offsets n a template may have (lane & 15)

template <int NBP, int W>
__device__ __forceinline__ void strip_prep(const StripArgs &a, const float *__restrict__ tmpl,
                                           uint8_t *__restrict__ ws, int kk, float (*colmax)[64],
                                           int *need_exact, float *wbuf)
{
    using Sh = StripShape<NBP>;
    constexpr int NI = NBP / 4;                          // 16-byte slots per (bx, lane)
    constexpr int BXW = (kStripMaxBX + W - 1) / W;       // block columns per wave
    constexpr int RS = 4 * NBP;                          // LDS floats per block row offset
    constexpr int NL = (RS + 63) / 64;                   // loads per block row offset
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63, w = wave_id_in_block();
    const int n = lane & 15, q = lane >> 4;
    const float *tk = tmpl + (int64_t)kk * a.dim;
    float *wb = wbuf + w * kStripPrepRows * RS;
    if (threadIdx.x == 0) *need_exact = 0;
    float vals[BXW][Sh::S][8];
    // The weights of block column bx are one run of 4 N_b consecutive
    // template elements per block row offset n (its four cells' bins):
    // loaded whole, 64 lanes at a time, every column of the wave at once,
    // then written to this wave's LDS rows one column at a time and gathered
    // into the fragment layout. (Gathered straight from the template, each
    // load would touch 64 cache lines.)
    const int run = 4 * a.nb;
    float t[BXW][kStripPrepRows][NL];
#pragma unroll
    for (int r = 0; r < BXW; ++r) {
        const int bx = w + W * r;
        if (bx < kStripMaxBX) {  // wave-uniform
#pragma unroll
            for (int m = 0; m < kStripPrepRows; ++m)
#pragma unroll
                for (int h = 0; h < NL; ++h) {
                    const int e = 64 * h + lane;
                    const bool ok = (m < a.nby) & (e < run);
                    t[r][m][h] = tk[ok ? (m * kStripMaxBX + bx) * run + e : 0];
                }
        }
    }
#pragma unroll
    for (int r = 0; r < BXW; ++r) {
        const int bx = w + W * r;
        float mx = 0.f;
        if (bx < kStripMaxBX) {  // wave-uniform
            lds_order();  // the previous column's gather reads come first
#pragma unroll
            for (int m = 0; m < kStripPrepRows; ++m)
#pragma unroll
                for (int h = 0; h < NL; ++h)
                    if (64 * h + lane < RS) wb[m * RS + 64 * h + lane] = t[r][m][h];
            lds_order();
        }
#pragma unroll
        for (int j = 0; j < Sh::S; ++j)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                float val = 0.f;
                if ((j < Sh::K32 || i < 4) && bx < kStripMaxBX) {  // compile-time; wave-uniform
                    const int k = j < Sh::K32 ? 32 * j + 8 * q + i : 32 * Sh::K32 + 4 * q + i;
                    // Feature k: cell c = 2 w + u of the block, bin slot b;
                    // padding slots and rows past the template weigh 0.
                    const int c = 2 * (k / (2 * NBP)) + (k % (2 * NBP)) / NBP, b = k % NBP;
                    const bool ok = (n < a.nby) & (b < a.nb);
                    const float wt = wb[n * RS + (ok ? c * a.nb + b : 0)];
                    val = ok ? wt : 0.f;
                }
                vals[r][j][i] = val;
                mx = fmaxf(mx, fabsf(val));
            }
        if (bx < kStripMaxBX) colmax[bx][lane] = mx;  // wave-uniform
    }
    __syncthreads();
    float mx = 0.f;
#pragma unroll
    for (int b = 0; b < kStripMaxBX; ++b)
#pragma unroll
        for (int g = 0; g < 4; ++g) mx = fmaxf(mx, colmax[b][16 * g + n]);
    int ex = 0;
    if (mx > 0.f) (void)frexpf(mx, &ex);  // mx = f 2^ex, f in [0.5, 1)
    const int e = mx > 0.f ? 15 - ex : 0;
    float svmin = INFINITY;  // smallest nonzero scaled weight
#pragma unroll
    for (int r = 0; r < BXW; ++r)
#pragma unroll
        for (int j = 0; j < Sh::S; ++j)
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (vals[r][j][i] != 0.f) svmin = fminf(svmin, fabsf(ldexpf(vals[r][j][i], e)));
    if (svmin < 0x1p-3f) *need_exact = 1;
    __syncthreads();
    const int mode = *need_exact ? kModeExact : kModeSplit;
    const bool exact = mode == kModeExact;
    uint8_t *tp = ws + a.tprep_off + (int64_t)kk * a.tprep_stride;
#pragma unroll
    for (int r = 0; r < BXW; ++r) {
        const int bx = w + W * r;
        if (bx >= kStripMaxBX) break;  // wave-uniform
        u32x4 *frag = reinterpret_cast<u32x4 *>(tp) + (int64_t)bx * NI * 64 + lane;
        if (exact) {
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                float4_t f;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int idx = strip_weight_index(q * NBP + 4 * i + c, NBP, a.nb, a.nby, n, bx);
                    const float wt = tk[idx >= 0 ? idx : 0];
                    f[c] = idx >= 0 ? wt : 0.f;
                }
                frag[(int64_t)i * 64] = __builtin_bit_cast(u32x4, f);
            }
        } else {
#pragma unroll
            for (int j = 0; j < Sh::S; ++j) {
                half8_t h, lo;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float sv = ldexpf(vals[r][j][i], e);
                    h[i] = (_Float16)sv;
                    lo[i] = (_Float16)(sv - (float)h[i]);
                }
                if (j < Sh::K32) {
                    frag[(int64_t)(2 * j) * 64] = __builtin_bit_cast(u32x4, h);
                    frag[(int64_t)(2 * j + 1) * 64] = __builtin_bit_cast(u32x4, lo);
                } else {  // the 16x16x16 step: four features per lane
                    frag[(int64_t)(2 * j) * 64] =
                        __builtin_bit_cast(u32x4, __builtin_shufflevector(h, lo, 0, 1, 2, 3, 8, 9, 10, 11));
                }
            }
        }
    }
    if (w == 0) {
        float *cs = reinterpret_cast<float *>(tp + (int64_t)kStripMaxBX * NI * 64 * 16);
        cs[lane] = exact ? 1.f : ldexpf(1.f, -e);
        if (lane == 0) reinterpret_cast<int *>(cs + 64)[0] = mode;
    }
}

// ---------------------------------------------------------------------------
// Pass 2 (k_int_scan), one launch with three kinds of work (block ranges):
//   rows:  E[tx][n][y]  = sum over t < tx of rowtot[t][n][y]   (thread per (n, y))
//   cols:  CS[ty][n][x] = sum over k < ty of coltot[k][n][x]   (thread per (n, x))
//   tiles: P[ty][tx][n] = sum over k < ty, t < tx of tiletot[k][t][n]
//          (wave per n; lanes over tx, a wave scan per tile row)
// From these the plane value just above a tile row is P + a prefix over the
// tile's columns of CS, and the row carry of a pixel row is E (k_int_emit).
struct ScanRanges {
    int prep_blocks;               // template prep workgroups first (one per template), if any
    int rows_blocks, cols_blocks;  // then blocks of the first two kinds; the rest are tiles
};


// Workgroups of eight waves: the template prep below then gives each wave
// one block column (kStripMaxBX = 7).
constexpr int kScanWaves = 8, kScanThreads = 64 * kScanWaves;

// NBP > 0: the launch also prepares the one-template strip scorer's weights
// (strip_prep, one wave per block column) in its first r.prep_blocks
// workgroups, beside the carries rather than as a launch of its own on the
// path (the two write disjoint parts of the workspace).
template <int NBP>
__global__ __launch_bounds__(kScanThreads) void k_int_scan(const Level *__restrict__ lv,
                                                  const int32_t *__restrict__ first_e,
                                                  const int32_t *__restrict__ first_c,
                                                  const int32_t *__restrict__ first_p, int n_levels,
                                                  int nb, ScanRanges r, uint8_t *__restrict__ ws,
                                                  StripArgs pa, const float *__restrict__ tmpl)
{
    int blk = (int)blockIdx.x;
    if constexpr (NBP > 0) {
        if (blk < r.prep_blocks) {
            __shared__ float colmax[kStripMaxBX][64];
            __shared__ int need_exact;
            __shared__ float wbuf[kScanWaves * kStripPrepRows * 4 * (NBP > 0 ? NBP : 1)];
            strip_prep<NBP, kScanWaves>(pa, tmpl, ws, blk, colmax, &need_exact, wbuf);
            return;
        }
        blk -= r.prep_blocks;
    }
    const int lane = threadIdx.x & 63;
    // Rows and columns: each thread carries four consecutive rows (columns)
    // of one bin: per tile one dword of four u8 counts in, four u16 carries
    // (8 bytes) out, kept as two pairs of 16-bit halves (a carry is at most
    // the level's width or height, below 2^15, so the halves never carry into
    // each other). Each (level, bin) holds a whole number of waves (its
    // threads are padded to a multiple of 64), so a wave's level, bin and tile
    // counts are uniform: found from its first thread, with the loads and
    // stores through buffer descriptors and the tile in the scalar offset.
    // Padding threads take offsets beyond the descriptors' ranges (their
    // loads read 0, their stores are dropped); rows past the level's height
    // get carries nobody reads.
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    auto walk4 = [](__amdgpu_buffer_rsrc_t src, __amdgpu_buffer_rsrc_t dst, int vs, int vd, uint32_t stride,
                    int count) {
        uint32_t lo = 0, hi = 0;  // carries of elements 0, 1 | 2, 3 in 16-bit halves
        auto step = [&](uint32_t c, int t) {
            __builtin_amdgcn_raw_buffer_store_b64(u32x2{lo, hi}, dst, vd, (int)(2u * (uint32_t)t * stride), 0);
            lo += (c & 0xFFu) | ((c << 8) & 0xFF0000u);
            hi += ((c >> 16) & 0xFFu) | ((c >> 8) & 0xFF0000u);
        };
        int t = 0;
        for (; t + 8 <= count; t += 8) {
            uint32_t c[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) c[i] = __builtin_amdgcn_raw_buffer_load_b32(src, vs, (int)((uint32_t)(t + i) * stride), 0);
#pragma unroll
            for (int i = 0; i < 8; ++i) step(c[i], t + i);
        }
        for (; t < count; ++t) step(__builtin_amdgcn_raw_buffer_load_b32(src, vs, (int)((uint32_t)t * stride), 0), t);
    };
    if (blk < r.rows_blocks) {
        const int g0 = __builtin_amdgcn_readfirstlane(blk * kScanThreads + (int)(threadIdx.x & ~63u));
        if (g0 >= first_e[n_levels]) return;
        const int l = find_level(first_e, n_levels, g0);
        const Level &v = lv[l];
        // Byte offsets as unsigned 32-bit values (a level's carries stay below 2^31 bytes).
        const uint32_t hp = kTile * v.tiles_y, stride = (uint32_t)nb * hp;
        const uint32_t q = 16u * (uint32_t)((v.tiles_y + 3) & ~3);  // threads per bin: hp / 4, whole waves
        const uint32_t rel0 = (uint32_t)(g0 - first_e[l]);
        const uint32_t n = rel0 / q;                           // wave-uniform
        const uint32_t y = 4u * (rel0 - n * q + (uint32_t)lane);  // first of the thread's rows
        const bool ok = y < hp;
        const __amdgpu_buffer_rsrc_t rts = buffer_rsrc(ws + v.ws_rowtot, (uint32_t)v.tiles_x * stride);
        const __amdgpu_buffer_rsrc_t es = buffer_rsrc(ws + v.ws_e, 2u * (uint32_t)v.tiles_x * stride);
        walk4(rts, es, ok ? (int)(n * hp + y) : (int)0x80000000u, ok ? (int)(2u * (n * hp + y)) : (int)0x80000000u,
              stride, v.tiles_x);
        return;
    }
    if (blk < r.rows_blocks + r.cols_blocks) {
        const int g0 = __builtin_amdgcn_readfirstlane((blk - r.rows_blocks) * kScanThreads + (int)(threadIdx.x & ~63u));
        if (g0 >= first_c[n_levels]) return;
        const int l = find_level(first_c, n_levels, g0);
        const Level &v = lv[l];
        const uint32_t wp = kTile * v.tiles_x, stride = (uint32_t)nb * wp;
        const uint32_t q = 16u * (uint32_t)((v.tiles_x + 3) & ~3);  // threads per bin: wp / 4, whole waves
        const uint32_t rel0 = (uint32_t)(g0 - first_c[l]);
        const uint32_t n = rel0 / q;
        const uint32_t x = 4u * (rel0 - n * q + (uint32_t)lane);
        const bool ok = x < wp;
        const __amdgpu_buffer_rsrc_t cts = buffer_rsrc(ws + v.ws_coltot, (uint32_t)v.tiles_y * stride);
        const __amdgpu_buffer_rsrc_t css = buffer_rsrc(ws + v.ws_cs, 2u * (uint32_t)v.tiles_y * stride);
        walk4(cts, css, ok ? (int)(n * wp + x) : (int)0x80000000u, ok ? (int)(2u * (n * wp + x)) : (int)0x80000000u,
              stride, v.tiles_y);
        return;
    }
    // Tiles: one wave per (level, n); lanes over tile columns in chunks of 64.
    const int g = (blk - r.rows_blocks - r.cols_blocks) * kScanWaves + wave_id_in_block();
    if (g >= first_p[n_levels]) return;
    const int l = find_level(first_p, n_levels, g);
    const Level &v = lv[l];
    const int n = g - first_p[l];
    // Tile totals in and prefixes out through buffer descriptors: lanes past
    // the level's tile columns take an offset beyond the array, so their
    // loads read 0 and their stores are dropped (no branch per lane).
    const uint32_t tbytes = (uint32_t)(v.tiles_x * v.tiles_y * nb) * 4u;
    const __amdgpu_buffer_rsrc_t tts = buffer_rsrc(ws + v.ws_tiletot, tbytes);
    const __amdgpu_buffer_rsrc_t ps = buffer_rsrc(ws + v.ws_p, tbytes);
    const int row_bytes = v.tiles_x * nb * 4;
    constexpr int kMaxChunks = 512 / 64;  // tiles_x <= 512 (width <= 32767)
    constexpr int kRows = 8;              // tile rows whose totals are loaded together
    uint32_t above[kMaxChunks];           // P of the current tile row, lane's columns
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c) above[c] = 0u;
    for (int ty0 = 0; ty0 < v.tiles_y; ty0 += kRows) {
        uint32_t carry[kRows];  // per row: its tiles left of the current chunk
#pragma unroll
        for (int i = 0; i < kRows; ++i) carry[i] = 0u;
#pragma unroll
        for (int c = 0; c < kMaxChunks; ++c) {
            if (64 * c < v.tiles_x) {  // wave-uniform
                const int tx = 64 * c + lane;
                const int vo = tx < v.tiles_x ? (tx * nb + n) * 4 : (int)0x80000000u;
                uint32_t t[kRows];
#pragma unroll
                for (int i = 0; i < kRows; ++i)
                    t[i] = ty0 + i < v.tiles_y  // wave-uniform
                               ? __builtin_amdgcn_raw_buffer_load_b32(tts, vo, (ty0 + i) * row_bytes, 0)
                               : 0u;
#pragma unroll
                for (int i = 0; i < kRows; ++i) {
                    if (ty0 + i < v.tiles_y) {  // wave-uniform
                        __builtin_amdgcn_raw_buffer_store_b32(above[c], ps, vo, (ty0 + i) * row_bytes, 0);
                        const uint32_t incl = wave_incl_scan(t[i]);
                        above[c] += carry[i] + incl - t[i];  // plus this row's tiles left of tx
                        carry[i] += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 3 (k_int_emit), Eq. 4 + Eq. 5 + Eq. 6. Each lane keeps, per bin of the
// wave's chunk, the running plane value of its column, seeded with the plane
// value just above the tile. Per pixel row: the one-hot image of Eq. 4 is a ballot per
// bin; its inclusive prefix along the tile row is a masked popcount (mbcnt);
// with the row carry E of the tiles on the left it gives the row prefix R,
// and ii(r, c) = ii(r-1, c) + R(r, c) is stored.
//
// Every 8th padded row is a row of cell corners: the lanes on every 8th
// padded column hold P(r, c); P(r, c-8) comes from the lane 8 to the left
// (or, for the tile's first cell, the plane column 64 tx: its value at row
// 64 ty plus the row carries E of the tile's rows so far, a wave scan of E
// read at each corner row), P(r-8, .) from the previous corner row. Their four-corner sum (Eq. 6) is the cell's
// histogram entry, cached here once per cell (uint16 [n][cy][cx]).
//
// The planes hold ii(x, y) at [y * pitch + x] (Eq. 5, one value per pixel),
// as PB-byte elements: the low 8 PB bits of the count (Sec. 4's 16-bit
// integral images, taken mod 2^(8 PB) so that four-corner sums of areas below
// 2^(8 PB) pixels stay exact). The running values in registers are full
// 32-bit counts either way, so the cell cache is the same for every PB.
//
// Occupancy: the uint16 writer with the cell cache waits mostly on
// instruction dependencies, so it is held to 8 waves per SIMD (at most 64
// VGPRs, no spills for any NBC), where the default allocation gives it 6.
// The uint32 writer (HBM-bound) and the uint8 writer ran slower so held.
// ---------------------------------------------------------------------------
template <int NBC, bool CELLS, int PB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PB == 2 && CELLS ? 8 : 1))) void k_int_emit(const Level *__restrict__ lv,
                                                  const int32_t *__restrict__ first, int n_levels,
                                                  int nb, int n_chunk,
                                                  const uint8_t *__restrict__ bins,
                                                  uint8_t *__restrict__ ws,
                                                  uint8_t *__restrict__ ii)
{
    static_assert(PB == 4 || PB == 2 || PB == 1, "plane element bytes");
    // Consecutive waves take the chunks of one tile.
    const int gw = (int)blockIdx.x * 4 + wave_id_in_block();
    const int lane = threadIdx.x & 63;
    const int tile = gw / n_chunk;
    if (tile >= first[n_levels]) return;
    const int l = find_level(first, n_levels, tile);
    const Level &v = lv[l];
    const int t = tile - first[l];
    const int tx = t % v.tiles_x, ty = t / v.tiles_x;
    // This wave's bins: b0 .. b0 + nbc - 1 (the last chunk may be short).
    const int b0 = (gw - tile * n_chunk) * NBC;
    const int nbc = min(NBC, nb - b0);
    const int W = v.w, H = v.h;
    const int x = tx * kTile + lane;
    const bool xin = x < W;
    const int y0 = ty * kTile, y1 = min(y0 + kTile, H);
    // Byte offset of this lane's column in a plane row. Lanes right of the
    // row pitch store at its last element: right of the level every lane
    // holds the value of column w - 1, so those duplicate stores write the
    // same value and every row store covers whole lines.
    const uint32_t colb = (uint32_t)min(x, (int)v.ii_pitch - 1) * (uint32_t)PB;

    // Carries (k_int_scan): the plane value at (x, 64 ty - 1) is P (pixels
    // above and left of the tile) plus the tile's columns' counts above it up
    // to x (a wave scan of CS); row y's count left of the tile is E (lane
    // y - y0 holds it). Right of the level CS is 0, so those lanes repeat the
    // value at column w - 1.
    const int64_t hp = (int64_t)kTile * v.tiles_y, wp = (int64_t)kTile * v.tiles_x;
    const uint16_t *Eb = reinterpret_cast<const uint16_t *>(ws + v.ws_e) + ((int64_t)tx * nb + b0) * hp;
    const uint16_t *CSb = reinterpret_cast<const uint16_t *>(ws + v.ws_cs) + ((int64_t)ty * nb + b0) * wp;
    const uint32_t *Pb = reinterpret_cast<const uint32_t *>(ws + v.ws_p) + ((int64_t)ty * v.tiles_x + tx) * nb + b0;
    const int er = y0 + lane;  // row whose carry this lane holds
    uint32_t run[NBC], top[NBC], ecar[NBC], lrun[NBC], ltop[NBC], cellacc[NBC];
#pragma unroll
    for (int j = 0; j < NBC; ++j) {
        const uint32_t pj = j < nbc ? Pb[j] : 0u;
        run[j] = pj + wave_incl_scan(j < nbc ? (uint32_t)CSb[(int64_t)j * wp + x] : 0u);
        top[j] = run[j];
        lrun[j] = pj;
        ltop[j] = pj;
        ecar[j] = (j < nbc && er < H) ? (uint32_t)Eb[(int64_t)j * hp + er] : 0u;
        cellacc[j] = 0u;
    }
    uint32_t ecum[NBC];  // lane r: P + the row carries of the tile's rows up to y0 + r
#pragma unroll
    for (int j = 0; j < NBC; ++j) ecum[j] = (CELLS && j < nbc) ? lrun[j] + wave_incl_scan(ecar[j]) : 0u;
    // All global loads of the tile happen here, before the first plane store:
    // on gfx9 one counter tracks loads and stores, so a load waited for later
    // would also wait for every store issued before it.
    __shared__ uint8_t tiles[4][kTile * kTile];
    uint8_t *tb = tiles[wave_id_in_block()];
    stage_bin_tile(tb, buffer_rsrc(bins + v.bins_off, (uint32_t)(v.bins_pitch * v.h)),
                   (int)v.bins_pitch, tx, y0, lane);

    // The chunk's nbc planes as one buffer; the plan keeps NBC * plane * PB < 2^31.
    const int planeb = (int)(v.ii_plane * PB), pitchb = (int)(v.ii_pitch * PB);
    const __amdgpu_buffer_rsrc_t isrc =
        buffer_rsrc(ii + (v.ii_off + (int64_t)b0 * v.ii_plane) * PB, (uint32_t)(nbc * planeb));
    auto store_row = [&](int j, int y, uint32_t val) {
        if constexpr (PB == 4)
            __builtin_amdgcn_raw_buffer_store_b32(val, isrc, (int)colb, j * planeb + y * pitchb, 0);
        else if constexpr (PB == 2)
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)val, isrc, (int)colb, j * planeb + y * pitchb, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)val, isrc, (int)colb, j * planeb + y * pitchb, 0);
    };

    // FULL: the chunk has all NBC bins (every chunk but possibly the last),
    // so the per-bin test is compiled out.
    auto do_row = [&](auto full_c, int bin, int y) {
        constexpr bool FULL = decltype(full_c)::value;
        const int rel = bin - b0;
        const int rr = y - y0;
#pragma unroll
        for (int j = 0; j < NBC; ++j) {
            if (!FULL && j >= nbc) break;  // wave-uniform
            const bool hit = rel == j;
            const uint64_t m = __ballot(hit);
            const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)ecar[j], rr);
            run[j] += e + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)m, hit ? 1u : 0u));
            store_row(j, y, run[j]);
        }
    };
    // Padded row r = y + 1 is a row of cell corners when r % 8 == 0. Lane
    // 8k + 7 computes the cell (k, q) of the tile (q = its cell row); the value
    // moves to lane 8q + k, so after the tile's 8 corner rows each lane holds
    // one cell of the tile's 8 x 8 block.
    auto do_corners = [&](auto full_c, int y) {
        constexpr bool FULL = decltype(full_c)::value;
        if constexpr (CELLS) {
            const int q = ((y + 1) >> 3) - 1 - 8 * ty;
            const int src = 8 * (lane & 7) + 7;
#pragma unroll
            for (int j = 0; j < NBC; ++j) {
                if (!FULL && j >= nbc) break;  // wave-uniform
                // The plane value left of the tile in row y: P plus the row
                // carries of the tile's rows up to y.
                lrun[j] = (uint32_t)__builtin_amdgcn_readlane((int)ecum[j], y - y0);
                const uint32_t rl = __shfl_up(run[j], 8u);
                const uint32_t tl = __shfl_up(top[j], 8u);
                const uint32_t left = (lane == 7) ? lrun[j] : rl;
                const uint32_t ltl = (lane == 7) ? ltop[j] : tl;
                const uint32_t h = run[j] - left - top[j] + ltl;
                const uint32_t moved = __shfl(h, src);
                cellacc[j] = ((lane >> 3) == q) ? moved : cellacc[j];
                top[j] = run[j];
                ltop[j] = lrun[j];
            }
        }
    };
    auto load_bin = [&](int y) -> int {
        const int raw = tb[(y - y0) * kTile + lane];
        return xin ? raw : kNoBin;
    };

    auto rows = [&](auto full_c) {
        int yb = y0;
        for (; yb + kRowBatch <= y1; yb += kRowBatch) {  // yb is a multiple of 16
            int bb[kRowBatch];
#pragma unroll
            for (int i = 0; i < kRowBatch; ++i) bb[i] = load_bin(yb + i);
#pragma unroll
            for (int i = 0; i < kRowBatch; ++i) {
                do_row(full_c, bb[i], yb + i);
                if ((i & 7) == 7) do_corners(full_c, yb + i);
            }
        }
        for (; yb < y1; ++yb) {
            do_row(full_c, load_bin(yb), yb);
            if (((yb + 1) & 7) == 0) do_corners(full_c, yb);
        }
    };
    if (nbc == NBC)
        rows(std::true_type{});
    else
        rows(std::false_type{});
    if constexpr (CELLS) {
        // One whole 128-byte line per bin: the tile's 8 x 8 cells.
        if (tx < v.cbx && ty < v.cby) {
            uint16_t *cache = reinterpret_cast<uint16_t *>(ws + v.ws_cache);
#pragma unroll
            for (int j = 0; j < NBC; ++j)
                if (j < nbc) cache[(((int64_t)(b0 + j) * v.cby + ty) * v.cbx + tx) * 64 + lane] = (uint16_t)cellacc[j];
        }
    }
}

// ---------------------------------------------------------------------------
// Eq. 6 + Sec. 3.3: the histogram of cell (cx, cy) is, on each bin's plane,
// P(r1, c1) + P(r0, c0) - P(r0, c1) - P(r1, c0) with (r0, c0) = cell * (cy, cx)
// and (r1, c1) = (r0, c0) + cell in padded coordinates. Computed once per
// cell and cached (uint16, [bin][cy][cx]) for every window that uses it.
// Narrow planes (T = uint16 / uint8) hold the counts mod 2^bits; the sum is
// taken mod 2^bits too and is exact, a cell having fewer than 2^bits pixels.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_cells(const Level *__restrict__ lv,
                                               const int32_t *__restrict__ first, int n_levels,
                                               int nb, int cell, const T *__restrict__ ii,
                                               uint8_t *__restrict__ ws,
                                               uint32_t *__restrict__ cell_hist)
{
    constexpr uint32_t kMask = sizeof(T) == 4 ? 0xffffffffu : (1u << (8 * sizeof(T))) - 1u;
    const int g = (int)(blockIdx.x * 256 + threadIdx.x);
    if (g >= first[n_levels]) return;
    const int l = find_level(first, n_levels, g);
    const Level &v = lv[l];
    const int rel = g - first[l];
    const int cy = rel / v.cells_x, cx = rel % v.cells_x;
    const T *P = ii + v.ii_off;
    // Corners: ii at the cell's last row/column and at the row/column just
    // before it; ii(-1, .) = ii(., -1) = 0.
    const int64_t y1 = (int64_t)(cy + 1) * cell - 1, x1 = (int64_t)(cx + 1) * cell - 1;
    const int64_t y0 = y1 - cell, x0 = x1 - cell;
    const int64_t r1 = y1 * v.ii_pitch, r0 = y0 * v.ii_pitch;
    uint16_t *cache = reinterpret_cast<uint16_t *>(ws + v.ws_cache);
    uint32_t *ch = cell_hist ? cell_hist + v.cell_off + (int64_t)rel * nb : nullptr;
    for (int n = 0; n < nb; ++n) {
        const T *p = P + (int64_t)n * v.ii_plane;
        const uint32_t a = p[r1 + x1];
        const uint32_t b = y0 >= 0 ? (uint32_t)p[r0 + x1] : 0u;
        const uint32_t c = x0 >= 0 ? (uint32_t)p[r1 + x0] : 0u;
        const uint32_t d = (y0 >= 0 && x0 >= 0) ? (uint32_t)p[r0 + x0] : 0u;
        const uint32_t h = (a - b - c + d) & kMask;
        cache[cache_index(v, n, cy, cx)] = (uint16_t)h;
        if (ch) ch[n] = h;
    }
}

// ---------------------------------------------------------------------------
// Soft votes (Sec. 2's two-bin split, quantised to 1/HOG_SOFT_QUANTUM):
// weighted integral images in the hard path's three passes over 64 x 64
// tiles, with vote weights in place of unit counts. A pixel with soft entry
// b0 | w1 << 8 gives Q - w1 to bin b0 and w1 to bin b0 + 1 mod nb (both to
// bin 0 when nb = 1).
//   1. k_soft_reduce: per tile, each bin's vote total in each of its rows,
//      into [n][tx][y] (row totals), and in each of its columns, into
//      [n][ty][x] (column totals);
//   2. k_soft_scan: the row totals become their exclusive prefix over tile
//      columns (the votes left of the tile in each row), the column totals
//      their exclusive prefix over tile rows (the votes above it in each
//      column);
//   3. k_soft_emit: per (tile, pair of bins), one wave seeds each column with
//      its plane value just above the tile -- the votes left of the tile in
//      the rows above, plus the prefix along the tile's columns of the votes
//      above -- then walks the tile's rows: each row's prefix inside the tile
//      is a wave scan of the votes, plus the votes left of the tile, and
//      ii(x, y) is written once. The two bins' votes share one scan as the
//      16-bit halves of a dword: a tile row holds at most 64 Q = 2048 votes
//      per bin, so the halves never carry into each other. With 8-pixel cells
//      the writer also caches every cell (Eq. 6) at each 8th row, as
//      k_int_emit does.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_soft_reduce(const Level *__restrict__ lv,
                                                    const int32_t *__restrict__ first, int n_levels,
                                                    int nb, const uint8_t *__restrict__ bins,
                                                    uint8_t *__restrict__ ws)
{
    // One wave per tile, every bin at once. LDS: the tile's soft entries
    // (row stride kStride bytes, 33 dwords, so lane-per-row reads hit
    // distinct banks), then per-lane histograms colh and rowh: each lane only
    // ever adds to its own slots. A total never exceeds 64 Q = 2048, so two
    // bins share a dword, 16 bits each (bin n: dword n / 2, half n % 2).
    constexpr uint32_t Q = HOG_SOFT_QUANTUM;
    constexpr int kStride = 2 * kTile + 4;
    extern __shared__ __attribute__((aligned(16))) uint32_t sred_smem[];
    const int tile = (int)blockIdx.x;
    const int lane = (int)threadIdx.x;
    if (tile >= first[n_levels]) return;
    const int l = find_level(first, n_levels, tile);
    const Level &v = lv[l];
    const int t = tile - first[l];
    const int tx = t % v.tiles_x, ty = t / v.tiles_x;
    uint8_t *tb = reinterpret_cast<uint8_t *>(sred_smem);
    const int nw = (nb + 1) >> 1;  // dwords per lane and histogram
    // One more slot per histogram, never read, takes the votes of entries
    // with no bin and of rows or columns outside the level, so every add is
    // unconditional.
    uint32_t *colh = sred_smem + kTile * kStride / 4;
    uint32_t *rowh = colh + (nw + 1) * 64;
    for (int k = 0; k < nw; ++k) {
        colh[k * 64 + lane] = 0u;
        rowh[k * 64 + lane] = 0u;
    }
    // Bins below nb: dword b / 2; no bin (255): the spare slot nw.
    auto slot = [nw](uint32_t b) { return min((int)(b >> 1), nw) * 64; };
    auto shift = [](uint32_t b) { return 16u * (b & 1u); };
    // Adds the votes of entry e to the histogram slots of lane ln (an entry
    // with no bin, b0 = 255, sends both to the spare slot).
    auto vote = [&](uint32_t *h, uint32_t e, int ln) {
        const uint32_t b0 = e & 255u, w1 = e >> 8;
        const uint32_t b1 = b0 + 1 == (uint32_t)nb ? 0u : b0 + 1;
        atomicAdd(&h[slot(b0) + ln], (Q - w1) << shift(b0));
        atomicAdd(&h[slot(b1) + ln], w1 << shift(b1));
    };
    {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        // Rows past the level's height read as 0 (outside the buffer range);
        // the tile's 128 bytes of a row lie inside the row pitch.
        const __amdgpu_buffer_rsrc_t bsrc = buffer_rsrc(bins + v.bins_off, (uint32_t)(v.bins_pitch * v.h));
        const int bpitch = (int)v.bins_pitch;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int k = lane + 64 * m;
            const int row = k >> 3, seg = k & 7;
            const u32x4 d = __builtin_amdgcn_raw_buffer_load_b128(
                bsrc, (ty * kTile + row) * bpitch + tx * 2 * kTile + 16 * seg, 0, 0);
            uint32_t *dst = reinterpret_cast<uint32_t *>(tb + row * kStride + 16 * seg);
            dst[0] = d[0];
            dst[1] = d[1];
            dst[2] = d[2];
            dst[3] = d[3];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int y0 = ty * kTile, nrows = min(kTile, v.h - y0);
    const int ncols = min(kTile, v.w - tx * kTile);
    // FULL: the whole tile lies inside the level (most tiles), so no entry
    // needs a test.
    auto totals = [&](auto full_c) {
        constexpr bool FULL = decltype(full_c)::value;
        // Column totals: lane = column; 16 rows read before their adds.
        const uint16_t *cp = reinterpret_cast<const uint16_t *>(tb) + lane;
        for (int r0 = 0; r0 < (FULL ? kTile : nrows); r0 += 16) {
            uint32_t e[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) e[j] = cp[(r0 + j) * (kStride / 2)];
#pragma unroll
            for (int j = 0; j < 16; ++j)
                vote(colh, FULL ? e[j] : ((lane < ncols) & (r0 + j < nrows) ? e[j] : (uint32_t)kNoBin), lane);
        }
        // Row totals: lane = row; two entries per dword.
        const uint32_t *rp = reinterpret_cast<const uint32_t *>(tb + lane * kStride);
        for (int k0 = 0; k0 < kTile / 2; k0 += 8) {
            uint32_t d[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) d[j] = rp[k0 + j];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int c = 2 * (k0 + j);
                const bool rin = lane < nrows;
                vote(rowh, FULL ? d[j] & 0xFFFFu : (rin & (c < ncols) ? d[j] & 0xFFFFu : (uint32_t)kNoBin), lane);
                vote(rowh, FULL ? d[j] >> 16 : (rin & (c + 1 < ncols) ? d[j] >> 16 : (uint32_t)kNoBin), lane);
            }
        }
    };
    if (nrows == kTile && ncols == kTile)
        totals(std::true_type{});
    else
        totals(std::false_type{});
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // Row totals [n][tx][hp] (lane = row), column totals [n][ty][wp] (lane =
    // column; 0 right of the level); each histogram dword (two bins) is read
    // once.
    const int64_t hp = (int64_t)kTile * v.tiles_y, wp = (int64_t)kTile * v.tiles_x;
    uint32_t *rowtot = reinterpret_cast<uint32_t *>(ws + v.ws_stot) + (int64_t)tx * hp + y0 + lane;
    uint32_t *coltot = reinterpret_cast<uint32_t *>(ws + v.ws_scol) + (int64_t)ty * wp + tx * kTile + lane;
    for (int k = 0; k < nw; ++k) {
        const uint32_t rs = rowh[k * 64 + lane], cs = colh[k * 64 + lane];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int n = 2 * k + e;
            if (n < nb) {  // wave-uniform
                if (lane < nrows) rowtot[(int64_t)n * v.tiles_x * hp] = (rs >> (16 * e)) & 0xFFFFu;
                coltot[(int64_t)n * v.tiles_y * wp] = (cs >> (16 * e)) & 0xFFFFu;
            }
        }
    }
}

// Pass 2: one thread per (bin, row) -- exclusive prefix of the row totals
// over tile columns -- then one per (bin, column) -- exclusive prefix of the
// column totals over tile rows.
__global__ __launch_bounds__(256) void k_soft_scan(const Level *__restrict__ lv,
                                                   const int32_t *__restrict__ first, int n_levels,
                                                   int nb, uint8_t *__restrict__ ws)
{
    // Row jobs are the tile-rounded rows hp per bin and column jobs the
    // columns wp per bin, both multiples of 64, so a wave's level, kind and
    // bin are uniform: found from its first item. Each (kind, bin) array goes
    // through one buffer descriptor (below 2^32 bytes), the lane's row or
    // column in the vector offset and the tile in the scalar one. Rows past
    // the level's height compute sums nobody reads.
    const int g0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 256 + (threadIdx.x & ~63u)));
    if (g0 >= first[n_levels]) return;
    const int lane = threadIdx.x & 63;
    const int l = find_level(first, n_levels, g0);
    const Level &v = lv[l];
    const uint32_t hp = kTile * v.tiles_y, wp = kTile * v.tiles_x;
    uint32_t rel0 = (uint32_t)(g0 - first[l]);
    const bool rows = rel0 < (uint32_t)nb * hp;
    if (!rows) rel0 -= (uint32_t)nb * hp;
    const uint32_t span = rows ? hp : wp;                  // items per bin
    const uint32_t n = rel0 / span;                        // the wave's bin
    const uint32_t count = rows ? v.tiles_x : v.tiles_y;   // tiles along the job
    const uint32_t plane = count * span * 4u;              // bytes per bin
    const __amdgpu_buffer_rsrc_t t = buffer_rsrc(ws + (rows ? v.ws_stot : v.ws_scol) + (int64_t)n * plane, plane);
    const int vo = (int)(4u * (rel0 - n * span + lane));
    const uint32_t step = 4u * span;
    uint32_t acc = 0;
    uint32_t k = 0;
    for (; k + 8 <= count; k += 8) {
        uint32_t c[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) c[i] = __builtin_amdgcn_raw_buffer_load_b32(t, vo, (int)((k + i) * step), 0);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            __builtin_amdgcn_raw_buffer_store_b32(acc, t, vo, (int)((k + i) * step), 0);
            acc += c[i];
        }
    }
    for (; k < count; ++k) {
        const uint32_t c = __builtin_amdgcn_raw_buffer_load_b32(t, vo, (int)(k * step), 0);
        __builtin_amdgcn_raw_buffer_store_b32(acc, t, vo, (int)(k * step), 0);
        acc += c;
    }
}

template <bool CELLS>
__global__ __launch_bounds__(256) void k_soft_emit(const Level *__restrict__ lv,
                                                   const int32_t *__restrict__ first, int n_levels,
                                                   int nb, const uint8_t *__restrict__ bins,
                                                   uint8_t *__restrict__ ws, uint32_t *__restrict__ ii)
{
    constexpr uint32_t Q = HOG_SOFT_QUANTUM;
    constexpr int kRows = 16;  // bin rows loaded ahead
    const int gw = (int)blockIdx.x * 4 + wave_id_in_block();
    if (gw >= first[n_levels]) return;  // whole wave: the scans below need every lane
    const int lane = threadIdx.x & 63;
    const int l = find_level(first, n_levels, gw);
    const Level &v = lv[l];
    const int pairs = (nb + 1) >> 1;
    const int rel = gw - first[l];
    const int tile = rel / pairs, n0 = 2 * (rel % pairs);
    const int tx = tile % v.tiles_x, ty = tile / v.tiles_x;
    const bool two = n0 + 1 < nb;  // wave-uniform: the pair's second bin exists
    // Bin n takes Q - w1 from pixels with b0 == n and w1 from those with
    // b0 == n - 1 (mod nb); a pixel without a bin (b0 = 255) matches neither.
    const uint32_t m0 = (uint32_t)n0, p0 = (uint32_t)(n0 == 0 ? nb - 1 : n0 - 1);
    const uint32_t m1 = (uint32_t)n0 + 1, p1 = (uint32_t)n0;
    const int x = tx * kTile + lane;
    const bool xin = x < v.w;
    const int y0 = ty * kTile, y1 = min(y0 + kTile, v.h);
    const int64_t hp = (int64_t)kTile * v.tiles_y, wp = (int64_t)kTile * v.tiles_x;
    // Votes left of the tile, per row, of both bins; votes above it, per column.
    const uint32_t *left0p = reinterpret_cast<const uint32_t *>(ws + v.ws_stot) + ((int64_t)n0 * v.tiles_x + tx) * hp;
    const uint32_t *left1p = left0p + v.tiles_x * hp;
    const uint32_t *above0p = reinterpret_cast<const uint32_t *>(ws + v.ws_scol) + ((int64_t)n0 * v.tiles_y + ty) * wp + x;
    const uint32_t *above1p = above0p + v.tiles_y * wp;
    // left*: the plane value at column 64 tx - 1 (the votes left of the tile
    // summed down the rows), here at row y0 - 1; four tile rows per step.
    uint32_t s0 = 0, s1 = 0;
    int yb = 0;
    for (; yb + 4 * kTile <= y0; yb += 4 * kTile) {
        uint32_t a[4], b[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = left0p[yb + k * kTile + lane];
            b[k] = two ? left1p[yb + k * kTile + lane] : 0u;
        }
        s0 += (a[0] + a[1]) + (a[2] + a[3]);
        s1 += (b[0] + b[1]) + (b[2] + b[3]);
    }
    for (; yb < y0; yb += kTile) {
        s0 += left0p[yb + lane];
        if (two) s1 += left1p[yb + lane];
    }
    const uint32_t left0 = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(s0), 63);
    const uint32_t left1 = (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(s1), 63);
    // ii(x, y0 - 1): the votes left of the tile above it, plus those above
    // the tile in its columns up to x.
    uint32_t acc0 = left0 + wave_incl_scan(above0p[0]);
    uint32_t acc1 = left1 + wave_incl_scan(two ? above1p[0] : 0u);
    // Cells: lanes 8c + 7 hold column x1 = 8 cx + 7 of cell cx; prev* is
    // ii(x1) - ii(x1 - 8) at the previous corner row (row y0 - 1 to start).
    uint16_t *cache = reinterpret_cast<uint16_t *>(ws + v.ws_cache);
    const int cx = x >> 3;
    const bool cell_lane = CELLS && (lane & 7) == 7 && cx < v.cells_x;
    auto corner_diff = [&](uint32_t a, uint32_t left) {
        const uint32_t w = __shfl_up(a, 8u);
        return a - (lane < 8 ? left : w);
    };
    uint32_t prev0 = 0, prev1 = 0;
    if (CELLS) {
        prev0 = corner_diff(acc0, left0);
        prev1 = corner_diff(acc1, left1);
    }
    // Lane i holds the votes left of the tile in row y0 + i; cum0 / cum1
    // their sums over the tile's rows up to y0 + i.
    const bool rin = y0 + lane < v.h;
    const uint32_t cv0 = rin ? left0p[y0 + lane] : 0u;
    const uint32_t cv1 = rin && two ? left1p[y0 + lane] : 0u;
    const uint32_t cum0 = wave_incl_scan(cv0), cum1 = wave_incl_scan(cv1);
    // Row y = y0 + i = 8 cy + 7, cy < cells_y. The plane value left of the
    // tile in that row is the votes above the tile's rows plus cum at i.
    auto corner = [&](auto two_c, int i) {
        constexpr bool TWO = decltype(two_c)::value;
        const int cy = (y0 + i) >> 3;
        const uint32_t l0 = left0 + (uint32_t)__builtin_amdgcn_readlane((int)cum0, i);
        const uint32_t l1 = left1 + (uint32_t)__builtin_amdgcn_readlane((int)cum1, i);
        const uint32_t d0 = corner_diff(acc0, l0), d1 = corner_diff(acc1, l1);
        if (cell_lane) {
            cache[cache_index(v, n0, cy, cx)] = (uint16_t)(d0 - prev0);
            if (TWO) cache[cache_index(v, n0 + 1, cy, cx)] = (uint16_t)(d1 - prev1);
        }
        prev0 = d0;
        prev1 = d1;
    };
    // The tile's soft entries (64 rows of 128 bytes) staged in LDS: with these
    // every global load happens before the first plane store (on gfx9 one
    // counter tracks loads and stores, so a load waited for between stores
    // would also wait for every store before it). Rows past the level's
    // height read as 0 and are never used; columns right of it are masked.
    __shared__ __attribute__((aligned(16))) uint8_t stiles[4][2 * kTile * kTile];
    uint8_t *tb = stiles[wave_id_in_block()];
    {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const __amdgpu_buffer_rsrc_t bsrc = buffer_rsrc(bins + v.bins_off, (uint32_t)(v.bins_pitch * v.h));
        const int bpitch = (int)v.bins_pitch;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int k = lane + 64 * m;
            const int r = k >> 3, seg = k & 7;
            const u32x4 d = __builtin_amdgcn_raw_buffer_load_b128(
                bsrc, (y0 + r) * bpitch + tx * 2 * kTile + 16 * seg, 0, 0);
            *reinterpret_cast<u32x4 *>(tb + r * 2 * kTile + 16 * seg) = d;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    const uint16_t *te = reinterpret_cast<const uint16_t *>(tb) + lane;
    // The pair's planes as one buffer (2 planes * 4 bytes < 2^31: the plan
    // keeps w * h * Q below 2^32). Lanes right of the row pitch store at its
    // last element: right of the level every lane holds the value of column
    // w - 1, so those duplicate stores write the same value.
    const int planeb = (int)(v.ii_plane * 4), pitchb = (int)(v.ii_pitch * 4);
    // (The size is made wave-uniform explicitly: a descriptor the compiler
    // takes for divergent costs a loop around every store.)
    const uint32_t isize = (uint32_t)__builtin_amdgcn_readfirstlane((two ? 2 : 1) * planeb);
    const __amdgpu_buffer_rsrc_t isrc = buffer_rsrc(ii + v.ii_off + (int64_t)n0 * v.ii_plane, isize);
    const int colb = min(x, (int)v.ii_pitch - 1) * 4;
    // TWO: the pair's second bin exists (every pair but possibly the last),
    // so its per-row tests are compiled out.
    auto row = [&](auto two_c, uint32_t e, int i) {
        constexpr bool TWO = decltype(two_c)::value;
        const int y = y0 + i;
        e = xin ? e : (uint32_t)kNoBin;
        const uint32_t b0 = e & 255u, w1 = e >> 8, qw = Q - w1;
        const uint32_t v0 = (b0 == m0 ? qw : 0u) + (b0 == p0 ? w1 : 0u);
        const uint32_t v1 = TWO ? (b0 == m1 ? qw : 0u) + (b0 == p1 ? w1 : 0u) : 0u;
        const uint32_t sc = wave_incl_scan(v0 | v1 << 16);
        const uint32_t c0 = (uint32_t)__builtin_amdgcn_readlane((int)cv0, i);
        const uint32_t c1 = (uint32_t)__builtin_amdgcn_readlane((int)cv1, i);
        acc0 += (sc & 0xFFFFu) + c0;
        acc1 += (sc >> 16) + c1;
        __builtin_amdgcn_raw_buffer_store_b32(acc0, isrc, colb, y * pitchb, 0);
        if (TWO) __builtin_amdgcn_raw_buffer_store_b32(acc1, isrc, colb, planeb + y * pitchb, 0);
        if (CELLS && (i & 7) == 7 && (y >> 3) < v.cells_y) corner(two_c, i);  // y0 is a multiple of 64
    };
    auto rows = [&](auto two_c) {
        int y = y0;
        for (; y + kRows <= y1; y += kRows) {  // y - y0 is a multiple of 16
#pragma unroll
            for (int i = 0; i < kRows; ++i) row(two_c, te[(y + i - y0) * kTile], y + i - y0);
        }
        for (; y < y1; ++y) row(two_c, te[(y - y0) * kTile], y - y0);
    };
    if (two)
        rows(std::true_type{});
    else
        rows(std::false_type{});
}

// Cell histograms cached by k_int_emit, exported as uint32 [cy][cx][n].
__global__ __launch_bounds__(256) void k_cache_export(const Level *__restrict__ lv,
                                                      const int32_t *__restrict__ first,
                                                      int n_levels, int nb,
                                                      const uint8_t *__restrict__ ws,
                                                      uint32_t *__restrict__ cell_hist)
{
    const int g = (int)(blockIdx.x * 256 + threadIdx.x);
    if (g >= first[n_levels]) return;
    const int l = find_level(first, n_levels, g);
    const Level &v = lv[l];
    const int rel = g - first[l];
    const int cy = rel / v.cells_x, cx = rel % v.cells_x;
    const uint16_t *cache = reinterpret_cast<const uint16_t *>(ws + v.ws_cache);
    uint32_t *ch = cell_hist + v.cell_off + (int64_t)rel * nb;
    for (int n = 0; n < nb; ++n) ch[n] = cache[cache_index(v, n, cy, cx)];
}

struct ScoreArgs {
    int nb, wcx, wcy, norm, k, dim, tw, th, nbp;
    float eps;
    float vscale;  // feature units per cached cell unit
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
    const int total = CH * CW * nb;
    for (int i = threadIdx.x; i < total; i += blockDim.x) {
        const int j = i % CW;
        const int rest = i / CW;
        const int r = rest % CH, n = rest / CH;
        const int cy = wy0 + r, cx = wx0 + j;
        float val = 0.f;
        if (cy < v.cells_y && cx < v.cells_x)
            val = (float)cache[cache_index(v, n, cy, cx)] * a.vscale;  // exact: a power of two
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

// ---------------------------------------------------------------------------
// Sec. 3.1 / Fig. 4 + Sec. 4 with raw features: a window's feature is its
// wcx x wcy cell histograms in row-major order, so its score is the bias
// plus one N_b-term inner product per cell. A workgroup takes a tile of
// tw x th = 64 windows, one per lane, and stages the cells they use into LDS
// as floats (up to kRawStage loads in flight per thread). Its R waves split
// the window's cell rows (wave r takes rows r, r + R, ...), so each lane walks
// about wcy / R rows instead of all of them, with the template weights of a
// row wave-uniform (scalar loads). As in k_score, each cell's N_b products
// form one FP32 partial and the partials are added in FP64: per wave, then
// across the waves in LDS.
// ---------------------------------------------------------------------------
constexpr int kRawStage = 8;

template <int NB, int WCX>
__global__ __launch_bounds__(1024) void k_score_raw(const Level *__restrict__ lv,
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
    const int nbp = NB > 0 ? NB : a.nbp;  // staged floats per cell
    const int wcx = WCX > 0 ? WCX : a.wcx;
    const int CW = a.tw + wcx - 1, CH = a.th + a.wcy - 1;
    const int nwaves = (int)(blockDim.x >> 6);
    float *hc = lds;
    double *red = reinterpret_cast<double *>(lds + ((CH * CW * nbp + 1) & ~1));  // [2][nwaves][64]

    // Stage the tile's cells (zero outside the level's cell grid): element
    // i = (n CH + r) CW + j, cell (wy0 + r, wx0 + j), bin n.
    const uint16_t *cache = reinterpret_cast<const uint16_t *>(ws + v.ws_cache);
    const int total = CH * CW * nb;
    for (int base = (int)threadIdx.x; base < total; base += kRawStage * (int)blockDim.x) {
        uint32_t val[kRawStage];
        int dst[kRawStage];
#pragma unroll
        for (int u = 0; u < kRawStage; ++u) {
            const int i = base + u * (int)blockDim.x;
            val[u] = 0u;
            dst[u] = -1;
            if (i < total) {
                const int j = i % CW, rest = i / CW;
                const int r = rest % CH, n = rest / CH;
                const int cy = wy0 + r, cx = wx0 + j;
                if (cy < v.cells_y && cx < v.cells_x) val[u] = cache[cache_index(v, n, cy, cx)];
                dst[u] = (r * CW + j) * nbp + n;
            }
        }
#pragma unroll
        for (int u = 0; u < kRawStage; ++u)
            if (dst[u] >= 0) hc[dst[u]] = (float)val[u] * a.vscale;  // exact: a power of two
    }
    __syncthreads();

    const int lane = (int)threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int tx = lane % a.tw, ty = lane / a.tw;
    const int wx = wx0 + tx, wy = wy0 + ty;
    const bool live = wx < v.win_x && wy < v.win_y;
    float *sout = scores + v.score_off + ((int64_t)wy * v.win_x + wx) * a.k;

    for (int k = 0; k < a.k; ++k) {
        const float *T = tmpl + (int64_t)k * a.dim;
        double s = 0.0;
        for (int q = w; q < a.wcy; q += nwaves) {
            const float *hrow = hc + ((ty + q) * CW + tx) * nbp;
            const float *trow = T + (int64_t)q * wcx * nb;
            if constexpr (NB > 0 && WCX > 0) {
#pragma unroll
                for (int qx = 0; qx < WCX; ++qx) {
                    float h[NB];
                    load_cell<NB>(hrow + qx * NB, h);
                    s += (double)dot_acc<NB>(trow + qx * NB, h, 0.f);
                }
            } else {
                for (int qx = 0; qx < wcx; ++qx) {
                    const float *hp = hrow + qx * nbp;
                    const float *wt = trow + qx * nb;
                    float g = 0.f;
                    for (int n = 0; n < nb; ++n) g = fmaf(wt[n], hp[n], g);
                    s += (double)g;
                }
            }
        }
        double *rk = red + (k & 1) * nwaves * 64;
        rk[w * 64 + lane] = s;
        __syncthreads();
        if (w == 0 && live) {
            double t = (double)bias[k];
            for (int r = 0; r < nwaves; ++r) t += rk[r * 64 + lane];
            sout[k] = (float)t;
        }
        // The next template writes the other half of red; the one after it
        // this half again, behind the barrier of the next iteration.
    }
}

// ---------------------------------------------------------------------------
// Sec. 3.1 / Fig. 4 + Sec. 4 on the matrix cores (L2 blocks of 2 x 2 cells).
//
// score(wx, wy) = bias + sum over block positions (by, bx) of
//     inv(B) * (T[by][bx] . v(B)),   B = (wy + by, wx + bx),
// with v(B) the block's 4 nb integer counts and inv(B) = 1/sqrt(|v|^2 + eps^2).
//
// One wave scores a strip of kStripW window columns (wx0 ..) over a range of
// window rows, walking the block rows Y. For block row Y and each bx, matrix
// instructions (16 x 16 outputs, fp16 inputs, FP32 accumulation) give
//     D_bx[m][n] = v(Y, wx0 + m + bx) . T[n][bx]      (m window column, n = by),
// the A rows being the row's blocks shifted by bx and B column n the weights
// at block position (n, bx). Then
//     acc32[m][n] = sum_bx inv(Y, wx0 + m + bx) * D_bx[m][n]       (FP32)
// is block row Y's share of window (wx0 + m, Y - n), added to that window's
// FP64 running sum, which lives in column n = Y - wy: after each block row
// every sum moves one column right (DPP row_shr:1), so a window enters at
// column 0 on its first block row and leaves column nby - 1 complete.
//
// The counts are exact in fp16. k_score_prep scales each weight column n
// by a power of two (its max |T| over all bx into [2^14, 2^15)) and splits it
// into fp16 hi + lo (each weight to 2^-22 relative); both products go into
// the block's FP32 accumulator. A template whose column weights span more
// than about 2^17 (where the lo halves would be fp16 subnormals) is scored in
// exact mode: the same walk with FP32 weights and FP32 16x16x4 products. A block's 4 NBP features are its cells (u, w) in the
// order w, u with NBP bin slots each (padding zero); the feature axis is
// covered by 16x16x32 steps, plus one 16x16x16 step when 4 NBP = 80.
// Cells sit in LDS as fp16 [cell][NBP] in a ring of four cell rows; each row
// is fetched from the blocked cache two block rows before it is needed.
// Waves are independent: no workgroup barrier. A wave's LDS operations are
// performed in issue order, so its own writes are visible to its later reads
// once the compiler keeps them in order (lds_order).
// ---------------------------------------------------------------------------
constexpr int kStripCells = kStripW + 8;    // cell columns staged per row

template <int V>
struct IntTag {
    static constexpr int value = V;
};
// Lane i of each 16-lane row takes lane i-1's value; lane 0 of a row takes 0.
__device__ __forceinline__ double shift_row_right(double x)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x111, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x111, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <int NBP>
__global__ __launch_bounds__(64 * kStripMaxBX) void k_score_prep(StripArgs a, const float *__restrict__ tmpl,
                                                                 uint8_t *__restrict__ ws)
{
    __shared__ float colmax[kStripMaxBX][64];
    __shared__ int need_exact;
    __shared__ float wbuf[kStripMaxBX * kStripPrepRows * 4 * NBP];
    strip_prep<NBP, kStripMaxBX>(a, tmpl, ws, (int)blockIdx.x, colmax, &need_exact, wbuf);
}

template <int NBP>
__global__ __launch_bounds__(256, 2) void k_score_strip(const Level *__restrict__ lv,
                                                     const int32_t *__restrict__ first, int n_levels,
                                                     StripArgs a, const uint8_t *__restrict__ ws,
                                                     const float *__restrict__ bias,
                                                     float *__restrict__ scores)
{
    using Sh = StripShape<NBP>;
    constexpr int ROWH = kStripCells * NBP;         // halves per staged cell row
    constexpr int NSEG = kStripCells / 8;           // 8-cell segments of the blocked cache
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];

    const int lane = threadIdx.x & 63, wave = wave_id_in_block();
    const int g = (int)blockIdx.x * 4 + wave;
    if (g >= first[n_levels]) return;
    const int l = find_level(first, n_levels, g);
    const Level &v = lv[l];
    int rel = g - first[l];
    const int sx = rel % v.st_x;
    rel /= v.st_x;
    const int sy = rel % v.st_y, kk = rel / v.st_y;
    const int wx0 = sx * kStripW, wy_lo = sy * a.th;
    const int wy_hi = min(wy_lo + a.th, v.win_y);
    const int y_last = wy_hi - 1 + a.nby - 1;  // last block row
    const int nb = a.nb;

    uint8_t *wl = smem + (size_t)wave * a.lds_wave;
    _Float16 *ring = reinterpret_cast<_Float16 *>(wl);
    float *invb = reinterpret_cast<float *>(wl + 4 * ROWH * 2);  // [2][32]: rows Y, Y + 1
    float *outb = invb + 64;
    {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        u32x4 *rz = reinterpret_cast<u32x4 *>(ring);
        for (int i = lane; i < 4 * ROWH / 8; i += 64) rz[i] = u32x4{0u, 0u, 0u, 0u};
    }

    // One 16-byte load per lane and row: lane t < nb * NSEG loads bin t / NSEG,
    // cells 8 (t % NSEG) .. + 7 of the strip (the plan keeps nb * NSEG <= 64).
    const uint16_t *cache = reinterpret_cast<const uint16_t *>(ws + v.ws_cache);
    const int f_bin = lane / NSEG, f_seg = lane - f_bin * NSEG;
    const bool f_on = lane < nb * NSEG && (wx0 >> 3) + f_seg < v.cbx;
    const uint16_t *f_base = cache + ((int64_t)f_bin * v.cby * v.cbx + (wx0 >> 3) + f_seg) * 64;
    const int64_t f_rowblk = (int64_t)v.cbx * 64;  // elements between 8-cell-row blocks
    auto fetch = [&](int cy) -> u16x8_t {
        u16x8_t val = {0, 0, 0, 0, 0, 0, 0, 0};
        if (f_on && cy < v.cells_y)
            val = *reinterpret_cast<const u16x8_t *>(f_base + (cy >> 3) * f_rowblk + (cy & 7) * 8);
        return val;
    };
    // Cells right of the level's last whole cell hold finite partial counts
    // (or 0 past the cache); they only reach windows that are not stored.
    auto store_row = [&](int slot, const u16x8_t &val) {
        _Float16 *rp = ring + slot * ROWH + f_bin + 8 * f_seg * NBP;
        if (lane < nb * NSEG) {
#pragma unroll
            for (int e = 0; e < 8; ++e) rp[e * NBP] = (_Float16)val[e];
        }
    };
    // Sum of squared counts of staged cell `lane` (exact in FP32). Lanes
    // past the staged cells repeat the last one (no branch); the blocks they
    // reach (22 and 23) are never read.
    auto row_sq = [&](int slot) -> float {
        float s = 0.f;
        const _Float16 *cp = ring + slot * ROWH + min(lane, kStripCells - 1) * NBP;
        typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int j = 0; j < NBP / 4; ++j) {
            const half4_t h = *reinterpret_cast<const half4_t *>(cp + 4 * j);
            const half2_t h0 = {h[0], h[1]}, h1 = {h[2], h[3]};
            s = __builtin_amdgcn_fdot2(h0, h0, s, false);
            s = __builtin_amdgcn_fdot2(h1, h1, s, false);
        }
        return s;
    };

    // The first four cell rows are in flight while the weights are loaded.
    u16x8_t pre0 = fetch(wy_lo), pre1 = fetch(wy_lo + 1);
    u16x8_t pre2 = fetch(wy_lo + 2), pre3 = fetch(wy_lo + 3);

    // Prepared B fragments (k_score_prep), column scales and mode.
    constexpr int NI = NBP / 4;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const uint8_t *tp = ws + a.tprep_off + (int64_t)kk * a.tprep_stride;
    const u32x4 *frag = reinterpret_cast<const u32x4 *>(tp) + lane;
    u32x4 braw[kStripMaxBX][NI];
#pragma unroll
    for (int bx = 0; bx < kStripMaxBX; ++bx)
#pragma unroll
        for (int i = 0; i < NI; ++i) braw[bx][i] = frag[(int64_t)(bx * NI + i) * 64];
    const float *csp = reinterpret_cast<const float *>(tp + (int64_t)kStripMaxBX * NI * 64 * 16);
    const float cs = csp[lane];
    const int mode = __builtin_amdgcn_readfirstlane(reinterpret_cast<const int *>(csp + 64)[0]);
    // Keep the fragments in registers for the whole strip: without this the
    // compiler may reload them from memory inside the row loop.
#pragma unroll
    for (int bx = 0; bx < kStripMaxBX; ++bx)
#pragma unroll
        for (int i = 0; i < NI; ++i) asm volatile("" : "+v"(braw[bx][i]));

    // A fragments: window column m = lane % 16; lane group q = lane / 16 takes
    // features k0 .. k0 + 7 (16x16x32) or k0 .. k0 + 3 (16x16x16) of each block:
    // cell row Y + k0 / 2NBP, offset k0 % 2NBP into the block's two cells.
    const int m = lane & 15, q = lane >> 4;
    int a_row[Sh::S], a_off[Sh::S];
#pragma unroll
    for (int j = 0; j < Sh::S; ++j) {
        const int k0 = j < Sh::K32 ? 32 * j + 8 * q : 32 * Sh::K32 + 4 * q;
        a_row[j] = k0 / (2 * NBP);
        a_off[j] = m * NBP + k0 % (2 * NBP);
    }
    auto load_a8 = [&](const _Float16 *p) -> half8_t {
        if constexpr ((NBP % 8) == 0) {
            return *reinterpret_cast<const half8_t *>(p);
        } else {  // 8-byte aligned
            const half4_t x = *reinterpret_cast<const half4_t *>(p), y = *reinterpret_cast<const half4_t *>(p + 4);
            return __builtin_shufflevector(x, y, 0, 1, 2, 3, 4, 5, 6, 7);
        }
    };

    // Norms of block row Y's blocks: block j = cells j, j + 1 of cell rows
    // Y, Y + 1 (sq0, sq1: each lane's cell), into invb[Y & 1].
    auto block_norms = [&](int Y, float sq0, float sq1) {
        const float t = sq0 + sq1;
        const float t1 = __builtin_bit_cast(float, from_right_lane(__builtin_bit_cast(uint32_t, t)));
        // Lanes 24 and up write the unused slots 24..31 (the same one from
        // lane 31 on): no branch.
        invb[(Y & 1) * 32 + min(lane, 31)] = inv_block_norm(t + t1, a.eps);
    };
    store_row(wy_lo & 3, pre0);
    store_row((wy_lo + 1) & 3, pre1);
    lds_order();
    float sq1 = row_sq((wy_lo + 1) & 3);
    block_norms(wy_lo, row_sq(wy_lo & 3), sq1);
    const double bk = (double)bias[kk];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};

    // Cell rows Y and Y + 1 are in the ring; rows Y + 2 and Y + 3 are in
    // flight in pre2 and pre3 (fetched two block rows ahead).
    // The row loop once per mode (a uniform branch outside it, so that each
    // loop gets its own register allocation).
    auto rows = [&](auto mtag) {
        constexpr int M = decltype(mtag)::value;
        for (int Y = wy_lo; Y <= y_last; ++Y) {
            const bool more = Y + 2 <= y_last + 1;
            lds_order();
            // iv[t] = inv of block 4 q + t of this row (t = r + bx <= 9).
            float iv[10];
            {
                const float *ib = invb + (Y & 1) * 32 + 4 * q;
                const float4_t f0 = *reinterpret_cast<const float4_t *>(ib);
                const float4_t f1 = *reinterpret_cast<const float4_t *>(ib + 4);
                const float2 f2 = *reinterpret_cast<const float2 *>(ib + 8);
                iv[0] = f0[0]; iv[1] = f0[1]; iv[2] = f0[2]; iv[3] = f0[3];
                iv[4] = f1[0]; iv[5] = f1[1]; iv[6] = f1[2]; iv[7] = f1[3];
                iv[8] = f2.x; iv[9] = f2.y;
            }
            // One FP32 accumulator per bx; the hi and lo products of a step are
            // issued bx-interleaved so consecutive instructions are independent.
            float4_t d[kStripMaxBX];
            auto zero_d = [&] {
#pragma unroll
                for (int bx = 0; bx < kStripMaxBX; ++bx) d[bx] = float4_t{0.f, 0.f, 0.f, 0.f};
            };
            // The fp16 products of every step, hi and lo halves.
            auto f16_products = [&] {
#pragma unroll
                for (int j = 0; j < Sh::K32; ++j) {
                    const _Float16 *ap = ring + ((Y + a_row[j]) & 3) * ROWH + a_off[j];
                    half8_t av[kStripMaxBX];
#pragma unroll
                    for (int bx = 0; bx < kStripMaxBX; ++bx) av[bx] = load_a8(ap + bx * NBP);
#pragma unroll
                    for (int bx = 0; bx < kStripMaxBX; ++bx)
                        d[bx] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                            av[bx], __builtin_bit_cast(half8_t, braw[bx][2 * j]), d[bx], 0, 0, 0);
#pragma unroll
                    for (int bx = 0; bx < kStripMaxBX; ++bx)
                        d[bx] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                            av[bx], __builtin_bit_cast(half8_t, braw[bx][2 * j + 1]), d[bx], 0, 0, 0);
                }
                if constexpr (Sh::K16 > 0) {
                    // The 16x16x16 products take the 16x16x32 products' results
                    // as their accumulator input. Left alone the compiler may
                    // issue one right behind the 16x16x32 product it reads, with
                    // no wait states, and that read has been seen to miss the
                    // chain's last two products (the last bx lost its second
                    // step). No matrix instruction crosses this barrier (LDS
                    // reads, vector and scalar ALU may: mask 0x106), so each
                    // bx's last 16x16x32 product is followed by those of later
                    // bx and the 16x16x16 ones of earlier bx before its own
                    // 16x16x16 product reads it (at least five other products).
                    __builtin_amdgcn_sched_barrier(0x106);
                    const _Float16 *ap = ring + ((Y + a_row[Sh::K32]) & 3) * ROWH + a_off[Sh::K32];
                    half4_t av[kStripMaxBX];
#pragma unroll
                    for (int bx = 0; bx < kStripMaxBX; ++bx) av[bx] = *reinterpret_cast<const half4_t *>(ap + bx * NBP);
#pragma unroll
                    for (int bx = 0; bx < kStripMaxBX; ++bx) {
                        const half8_t hl = __builtin_bit_cast(half8_t, braw[bx][2 * Sh::K32]);
                        d[bx] = __builtin_amdgcn_mfma_f32_16x16x16f16(
                            av[bx], __builtin_shufflevector(hl, hl, 0, 1, 2, 3), d[bx], 0, 0, 0);
                    }
#pragma unroll
                    for (int bx = 0; bx < kStripMaxBX; ++bx) {
                        const half8_t hl = __builtin_bit_cast(half8_t, braw[bx][2 * Sh::K32]);
                        d[bx] = __builtin_amdgcn_mfma_f32_16x16x16f16(
                            av[bx], __builtin_shufflevector(hl, hl, 4, 5, 6, 7), d[bx], 0, 0, 0);
                    }
                }
            };
            // acc32[r] (+)= sum_bx inv(Y, 4 q + r + bx) d[bx][r].
            float acc32[4] = {0.f, 0.f, 0.f, 0.f};
            auto fold = [&](float (&t)[4]) {
#pragma unroll
                for (int bx = 0; bx < kStripMaxBX; ++bx)
#pragma unroll
                    for (int r = 0; r < 4; ++r) t[r] = fmaf(d[bx][r], iv[r + bx], t[r]);
            };
            // The next rows' staging and norms do not depend on this row's
            // products (they write ring slot Y + 2 and invb[(Y + 1) & 1],
            // which this row does not read, its iv being loaded above), so
            // they run while the products are in the matrix pipe.
            auto next_rows = [&] {
                if (more) {
                    store_row((Y + 2) & 3, pre2);
                    lds_order();
                    // Next block row's norms, one row ahead of their use.
                    const float sq2 = row_sq((Y + 2) & 3);
                    block_norms(Y + 1, sq1, sq2);
                    sq1 = sq2;
                }
            };
            zero_d();
            if constexpr (M == kModeSplit) {
                f16_products();
                next_rows();
                fold(acc32);
            } else {
                // Exact mode: FP32 products, 4 features per step. Lane group q
                // takes cell q of each block -- cell row Y + q / 2, column
                // m + bx + q % 2 of the staged row -- bins 4 i .. 4 i + 3 at slot i.
                const _Float16 *cp = ring + ((Y + (q >> 1)) & 3) * ROWH + (m + (q & 1)) * NBP;
#pragma unroll
                for (int i = 0; i < NI; ++i) {
                    half4_t av[kStripMaxBX];
#pragma unroll
                    for (int bx = 0; bx < kStripMaxBX; ++bx) av[bx] = *reinterpret_cast<const half4_t *>(cp + bx * NBP + 4 * i);
#pragma unroll
                    for (int c = 0; c < 4; ++c)
#pragma unroll
                        for (int bx = 0; bx < kStripMaxBX; ++bx)
                            d[bx] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)av[bx][c],
                                                                        __uint_as_float(braw[bx][i][c]), d[bx], 0, 0, 0);
                }
                next_rows();
                fold(acc32);
            }
            const int wy_done = Y - (a.nby - 1);
            const bool done = m == a.nby - 1 && wy_done >= wy_lo && wy_done < wy_hi;
            float4_t o;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                acc[r] += (double)(acc32[r] * cs);
                o[r] = (float)(bk + acc[r]);
                acc[r] = shift_row_right(acc[r]);
            }
            if (done) *reinterpret_cast<float4_t *>(outb + (wy_done - wy_lo) * kStripW + 4 * q) = o;
            pre2 = pre3;
            if (Y + 4 <= y_last + 1) pre3 = fetch(Y + 4);
        }
    };
    if (mode == kModeExact)
        rows(IntTag<kModeExact>{});
    else
        rows(IntTag<kModeSplit>{});
    lds_order();
    const int n_out = (wy_hi - wy_lo) * kStripW;
    for (int i = lane; i < n_out; i += 64) {
        const int wx = wx0 + i % kStripW, wy = wy_lo + i / kStripW;
        if (wx < v.win_x) scores[v.score_off + ((int64_t)wy * v.win_x + wx) * a.k + kk] = outb[i];
    }
}

// ---------------------------------------------------------------------------
// Sec. 3.1 / Fig. 4 + Sec. 4 for many templates (K >= 16, in tiles of 32): a
// GEMM of windows x features by features x templates. For a window row wy
// and block position p = (by, bx), v_mfma_f32_32x32x16_f16 gives
//     D_p[k][m] = T_k[p] . v(B(m, p)),   B(m, p) = block (wy + by, wx0 + m + bx),
// with 32 templates on the M axis and 32 windows on the N axis, so each lane
// holds one window and the block's 1/sqrt(|v|^2 + eps^2) is one scale per
// lane: S[k][m] += inv(B(m, p)) * D_p[k][m] (FP32). The counts are exact in
// fp16; k_score_prep_wg scales each template by a power of two (its max |T|
// into [2^14, 2^15)) and splits it into fp16 hi + lo, lo stored times 2^11
// and multiplying the counts times 2^-11 (exact in fp16), so that each weight
// within about 2^28 of its template's largest keeps 2^-22 relative (an
// unscaled lo half would be an fp16 subnormal from about 2^17 down: with 32
// templates per tile that range is common). A tile holding a template
// that neither split carries to 2^-22 relative (a nonzero weight more than
// about 2^28 below the template's largest) is scored in exact mode: FP32
// weights and FP32 32x32x2 products on the same tiles.
//
// A workgroup covers one tile of windows for one tile of 32 templates, in
// one of two shapes (WgShape): kWgW window columns x kWgTH rows, where wave w
// owns rows w and w + 4, each as two 32-window halves; or, on levels at most
// kWgW / 2 windows wide, 32 columns x 2 kWgTH rows, where wave w owns rows
// w, w + 4, w + 8 and w + 12. Narrow levels would leave half of a wide tile
// empty. The workgroup walks by = 0 .. nby - 1: the tile's cell rows wy0 + by
// .. + TH sit in an LDS ring (one new row per by), so do the norms of the TH
// block rows in use (one new row per by), and the template fragments of the
// positions (by, 0 .. 6) are in LDS, fetched between the barriers that end the
// previous block row.
// ---------------------------------------------------------------------------
template <bool NARROW>
struct WgShape {
    static constexpr int W = NARROW ? kWgW / 2 : kWgW;     // window columns
    static constexpr int TH = NARROW ? 2 * kWgTH : kWgTH;  // window rows
    static constexpr int CELLS = W + 8;                    // cell columns staged per row
    static constexpr int SLOTS = TH + 1;                   // cell-row ring
};
// The LDS arrays hold either shape.
constexpr int kWgRingCells = WgShape<false>::SLOTS * WgShape<false>::CELLS > WgShape<true>::SLOTS * WgShape<true>::CELLS
                                 ? WgShape<false>::SLOTS * WgShape<false>::CELLS
                                 : WgShape<true>::SLOTS * WgShape<true>::CELLS;
constexpr int kWgInvCells = WgShape<false>::TH * WgShape<false>::CELLS > WgShape<true>::TH * WgShape<true>::CELLS
                                ? WgShape<false>::TH * WgShape<false>::CELLS
                                : WgShape<true>::TH * WgShape<true>::CELLS;

struct WgArgs {
    int nb, nby, k, dim;
    int64_t tprep_off, tprep_stride;
    float eps;
};

typedef float float16v_t __attribute__((ext_vector_type(16)));

// Per template: the power of two that brings its max |T| into [2^14, 2^15)
// -- scale 2^-e (float [32]) and exponent e (int [32]), stored after its
// tile's fragments -- and the template's mode (int [32] after those):
// kModeExact if some nonzero weight scales below 2^-14 (where hi is an fp16
// subnormal), else kModeWide. A tile with an exact template is scored in
// exact mode. One wave per template slot of every
// tile (0 past the last template), 8 loads in flight per lane.
__global__ __launch_bounds__(64) void k_score_prep_wg_scale(WgArgs a, const float *__restrict__ tmpl,
                                                            uint8_t *__restrict__ ws, int64_t frag_bytes)
{
    const int kk = (int)blockIdx.x, kt = kk >> 5, tk = kk & 31;
    const int lane = threadIdx.x;
    const float *t = tmpl + (int64_t)kk * a.dim;
    float mx = 0.f;
    if (kk < a.k) {
        int i = lane;
        for (; i + 7 * 64 < a.dim; i += 8 * 64) {
            float r[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) r[j] = t[i + 64 * j];
#pragma unroll
            for (int j = 0; j < 8; ++j) mx = fmaxf(mx, fabsf(r[j]));
        }
        for (; i < a.dim; i += 64) mx = fmaxf(mx, fabsf(t[i]));
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mx = fmaxf(mx, __shfl_xor(mx, d));
    int ex = 0;
    if (mx > 0.f) (void)frexpf(mx, &ex);  // mx = f 2^ex, f in [0.5, 1)
    const int e = mx > 0.f ? 15 - ex : 0;
    float svmin = INFINITY;  // smallest nonzero scaled weight
    if (kk < a.k)
        for (int i = lane; i < a.dim; i += 64) {
            const float w = t[i];
            if (w != 0.f) svmin = fminf(svmin, fabsf(ldexpf(w, e)));
        }
    const bool any_exact = __any(svmin < 0x1p-14f);
    uint8_t *tp = ws + a.tprep_off + (int64_t)kt * a.tprep_stride + frag_bytes;
    if (lane == 0) {
        reinterpret_cast<float *>(tp)[tk] = ldexpf(1.f, -e);
        reinterpret_cast<int *>(tp + 32 * 4)[tk] = e;
        reinterpret_cast<int *>(tp + 32 * 8)[tk] = any_exact ? kModeExact : kModeWide;
    }
}

// The A fragments of a tile, 16 bytes per thread, over as many workgroups as
// the tile has fragments / 256. Split mode: [p][s][hi|lo][lane] (lane:
// template kk0 + lane % 32, features 16 s + 8 (lane / 32) .. + 7 of the block
// at position p), the weights sv scaled by 2^e and split into fp16 hi = sv
// rounded and lo = (sv - hi) 2^11 rounded (the scorer multiplies lo by the
// counts times 2^-11, which is exact in fp16).
// Exact mode (a template of the tile flagged by k_score_prep_wg_scale): the
// FP32 weights [p][t][lane] for the 32x32x2 FP32 products, t < 2 NBP: lane
// (template kk0 + lane % 32, h = lane / 32) holds feature h 2 NBP + t of the
// block (cell row h, cell t / NBP, bin t % NBP). Both take 512 NBP bytes per
// block position.
template <int NBP>
__global__ __launch_bounds__(256) void k_score_prep_wg(WgArgs a, const float *__restrict__ tmpl,
                                                       uint8_t *__restrict__ ws)
{
    constexpr int KS = NBP / 4;  // 16-feature steps per block
    const int kt = (int)blockIdx.y, kk0 = 32 * kt;
    uint8_t *tp = ws + a.tprep_off + (int64_t)kt * a.tprep_stride;
    const int n_frag = a.nby * kStripMaxBX * KS * 2 * 64;
    const int f = (int)(blockIdx.x * 256 + threadIdx.x);
    if (f >= n_frag) return;
    const int *ex = reinterpret_cast<const int *>(tp + (int64_t)n_frag * 16 + 32 * 4);
    const int *tmode = ex + 32;
    bool exact = false;
    for (int i = 0; i < 32; ++i) exact |= tmode[i] == kModeExact;
    const int lane = f & 63, rest = f >> 6;
    const int pos = (rest >> 1) / KS;
    const int by = pos / kStripMaxBX, bx = pos % kStripMaxBX;
    const float *tpos = tmpl + (int64_t)(by * kStripMaxBX + bx) * 4 * a.nb;
    if (exact) {
        // Floats 4 fl .. 4 fl + 3 of position pos, fl = the thread's 16-byte
        // slot within it; float j sits at [t = j / 64][lane' = j % 64].
        const int fl = f - pos * KS * 2 * 64;
        float4_t out;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int j = 4 * fl + c, t = j >> 6, ln = j & 63;
            const int kk = kk0 + (ln & 31), h = ln >> 5;
            const int u = t / NBP, bin = t % NBP;
            out[c] = kk < a.k && bin < a.nb ? tpos[(int64_t)kk * a.dim + (h * 2 + u) * a.nb + bin] : 0.f;
        }
        *reinterpret_cast<float4_t *>(tp + (int64_t)f * 16) = out;
        return;
    }
    const int hl = rest & 1, s = (rest >> 1) % KS;
    const int kk = kk0 + (lane & 31), h = lane >> 5;
    const int e = ex[lane & 31];
    half8_t out;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int kf = 16 * s + 8 * h + i;
        const int w = kf / (2 * NBP), rem = kf % (2 * NBP);
        const int u = rem / NBP, bin = rem % NBP;
        float val = 0.f;
        if (kk < a.k && bin < a.nb) val = tpos[(int64_t)kk * a.dim + (w * 2 + u) * a.nb + bin];
        const float sv = ldexpf(val, e);
        const _Float16 hi = (_Float16)sv;
        out[i] = hl == 0 ? hi : (_Float16)((sv - (float)hi) * 2048.f);
    }
    *reinterpret_cast<half8_t *>(tp + (int64_t)f * 16) = out;
}

template <int NBP>
struct WgLds {
    static constexpr int NFRAG = kStripMaxBX * (NBP / 4) * 2;  // fragments per block row offset: [bx][s][hi|lo]
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 bst[1][NFRAG * 64];  // one block row offset's fragments (written between barriers)
    __attribute__((aligned(16))) _Float16 ring[kWgRingCells * NBP];
    float sqr[kWgRingCells];
    float invb[kWgInvCells];
};

template <int NBP, bool NARROW>
__device__ __forceinline__ void wgemm_tile(WgLds<NBP> &L, const Level &v, int rel, const WgArgs &a,
                                           const uint8_t *__restrict__ ws, const float *__restrict__ bias,
                                           float *__restrict__ scores)
{
    using Sh = WgShape<NARROW>;
    constexpr int KS = NBP / 4;                  // 16-feature steps per block
    constexpr int NFRAG = WgLds<NBP>::NFRAG;
    constexpr int CELLS = Sh::CELLS, SLOTS = Sh::SLOTS, TH = Sh::TH;
    constexpr int ROWH = CELLS * NBP;            // halves per staged cell row
    constexpr int NSEG = CELLS / 8;              // 8-cell segments of the blocked cache
    constexpr int PF = NFRAG * 64 / 256;         // 16-byte fragment loads per thread and by
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    auto &bst = L.bst;
    _Float16 (*ring)[ROWH] = reinterpret_cast<_Float16 (*)[ROWH]>(L.ring);
    float (*sqr)[CELLS] = reinterpret_cast<float (*)[CELLS]>(L.sqr);
    float (*invb)[CELLS] = reinterpret_cast<float (*)[CELLS]>(L.invb);

    const int tx = rel % v.st_x;
    rel /= v.st_x;
    const int ty = rel % v.st_y, kt = rel / v.st_y;
    const int wx0 = tx * Sh::W, wy0 = ty * TH, kk0 = 32 * kt;
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = lane & 31, h = lane >> 5;
    const int nb = a.nb, nby = a.nby;
    const uint8_t *tp = ws + a.tprep_off + (int64_t)kt * a.tprep_stride;
    const u32x4 *tfrag = reinterpret_cast<const u32x4 *>(tp);
    // The tile's mode: the strongest among its templates' (k_score_prep_wg_scale).
    const int tmode = reinterpret_cast<const int *>(tp + (int64_t)nby * NFRAG * 64 * 16 + 32 * 8)[lane & 31];
    const bool exact = __any(tmode == kModeExact);

    for (int i = tid; i < SLOTS * ROWH / 8; i += 256)
        reinterpret_cast<u32x4 *>(&ring[0][0])[i] = u32x4{0u, 0u, 0u, 0u};

    // Cell row cy: thread t < nb * NSEG loads bin t / NSEG of cells
    // 8 (t % NSEG) .. + 7 (0 outside the level's cache).
    const uint16_t *cache = reinterpret_cast<const uint16_t *>(ws + v.ws_cache);
    const int f_bin = tid / NSEG, f_seg = tid - f_bin * NSEG;
    const bool f_on = tid < nb * NSEG && (wx0 >> 3) + f_seg < v.cbx;
    auto fetch_row = [&](int cy) -> u16x8_t {
        u16x8_t val = {0, 0, 0, 0, 0, 0, 0, 0};
        if (f_on && cy < v.cells_y)
            val = *reinterpret_cast<const u16x8_t *>(
                cache + (((int64_t)f_bin * v.cby + (cy >> 3)) * v.cbx + (wx0 >> 3) + f_seg) * 64 + (cy & 7) * 8);
        return val;
    };
    auto store_row = [&](int cy, const u16x8_t &val) {
        if (tid < nb * NSEG) {
            _Float16 *rp = &ring[cy % SLOTS][8 * f_seg * NBP + f_bin];
#pragma unroll
            for (int e = 0; e < 8; ++e) rp[e * NBP] = (_Float16)val[e];
        }
    };
    auto row_sq = [&](int cy) {  // threads < CELLS
        if (tid < CELLS) {
            const _Float16 *cp = &ring[cy % SLOTS][tid * NBP];
            typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < NBP / 2; ++j) {
                const half2_t hv = {cp[2 * j], cp[2 * j + 1]};
                s = __builtin_amdgcn_fdot2(hv, hv, s, false);
            }
            sqr[cy % SLOTS][tid] = s;
        }
    };
    auto fetch_frags = [&](int by, u32x4 (&pf)[PF]) {
#pragma unroll
        for (int i = 0; i < PF; ++i) pf[i] = tfrag[(int64_t)by * NFRAG * 64 + tid + 256 * i];
    };
    auto store_frags = [&](const u32x4 (&pf)[PF]) {
#pragma unroll
        for (int i = 0; i < PF; ++i) bst[0][tid + 256 * i] = pf[i];
    };

    // Prologue: cell rows wy0 .. wy0 + TH and the fragments of by = 0; the
    // next row in flight. (Fragments are fetched between the barriers that
    // end each block row: holding them in registers across the walk would
    // cost the registers that let three workgroups share a CU.)
    {
        u32x4 pf[PF];
        fetch_frags(0, pf);
        u16x8_t rows[TH + 1];
#pragma unroll
        for (int i = 0; i <= TH; ++i) rows[i] = fetch_row(wy0 + i);
        __syncthreads();  // ring zeroed
#pragma unroll
        for (int i = 0; i <= TH; ++i) store_row(wy0 + i, rows[i]);
        store_frags(pf);
    }
    __syncthreads();
    for (int i = 0; i <= TH; ++i) row_sq(wy0 + i);
    u16x8_t cpre = fetch_row(wy0 + TH + 1);

    // Window rows of this wave: rho = wave, wave + 4; halves mu = 0, 1.
    float16v_t S[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) S[q][r] = 0.f;

    // The block-row walk once per mode (a uniform branch outside it, so that
    // each walk gets its own register allocation).
    auto walk = [&](auto mtag) {
        constexpr int M = decltype(mtag)::value;
        for (int by = 0; by < nby; ++by) {
            __syncthreads();  // rows and their sums of squares are in place
            // Norms of the block rows new to the tile's window rows: all TH at
            // by = 0, then one per by. Block row wy0 + Y sits in invb[Y % TH]
            // while it is in use (by <= Y < by + TH).
            const int r0 = by == 0 ? 0 : TH - 1;
            for (int i = tid; i < (TH - r0) * (CELLS - 1); i += 256) {
                const int rho = r0 + i / (CELLS - 1), c = i - (rho - r0) * (CELLS - 1);
                const int Y = by + rho;
                const int s0 = (wy0 + Y) % SLOTS, s1 = (wy0 + Y + 1) % SLOTS;
                invb[Y % TH][c] = inv_block_norm((sqr[s0][c] + sqr[s0][c + 1]) + (sqr[s1][c] + sqr[s1][c + 1]), a.eps);
            }
            __syncthreads();
            if constexpr (M == kModeExact) {
                // Exact mode: FP32 products, 2 features per step; at step t lane
                // (template or window n, h) takes feature h 2 NBP + t of the block:
                // cell row h, cell t / NBP, bin t % NBP.
                const float *af = reinterpret_cast<const float *>(bst[0]);
#pragma unroll 1
                for (int bx = 0; bx < kStripMaxBX; ++bx) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int rho = NARROW ? wave + 4 * q : wave + 4 * (q >> 1), mu = NARROW ? 0 : q & 1;
                        const float ivq = invb[(by + rho) % TH][32 * mu + n + bx];
                        const int wi = ((wy0 + by + rho + h) % SLOTS) * ROWH + (32 * mu + n + bx) * NBP;
                        float16v_t d;
#pragma unroll
                        for (int r = 0; r < 16; ++r) d[r] = 0.f;
#pragma unroll 2
                        for (int t = 0; t < 2 * NBP; ++t)
                            d = __builtin_amdgcn_mfma_f32_32x32x2f32(af[(bx * 2 * NBP + t) * 64 + lane],
                                                                    (float)L.ring[wi + t], d, 0, 0, 0);
#pragma unroll
                        for (int r = 0; r < 16; ++r) S[q][r] = fmaf(d[r], ivq, S[q][r]);
                    }
                }
            } else {
            const half8_t *bf = reinterpret_cast<const half8_t *>(bst[0]);
#pragma unroll 1
            for (int bx = 0; bx < kStripMaxBX; ++bx) {
                half8_t bh[KS], bl[KS];
#pragma unroll
                for (int s2 = 0; s2 < KS; ++s2) {
                    bh[s2] = bf[((bx * KS + s2) * 2 + 0) * 64 + lane];
                    bl[s2] = bf[((bx * KS + s2) * 2 + 1) * 64 + lane];
                }
                // The four window groups q in two rounds of two accumulators
                // each (registers for three workgroups per CU); per q the
                // products still go hi s2 = 0, 1, then lo, and S[q] takes its
                // terms in bx order.
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    half8_t wf[2][KS];
                    float iv[2];
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2) {
                        const int q = 2 * g + h2;
                        const int rho = NARROW ? wave + 4 * q : wave + 4 * (q >> 1), mu = NARROW ? 0 : q & 1;
#pragma unroll
                        for (int s2 = 0; s2 < KS; ++s2) {
                            const int kf = 16 * s2 + 8 * h;
                            const int w = kf / (2 * NBP);
                            wf[h2][s2] = *reinterpret_cast<const half8_t *>(
                                &ring[(wy0 + by + rho + w) % SLOTS][(32 * mu + n + bx) * NBP + kf % (2 * NBP)]);
                        }
                        iv[h2] = invb[(by + rho) % TH][32 * mu + n + bx];
                    }
                    float16v_t d[2];
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                        for (int r = 0; r < 16; ++r) d[h2][r] = 0.f;
#pragma unroll
                    for (int s2 = 0; s2 < KS; ++s2)
#pragma unroll
                        for (int h2 = 0; h2 < 2; ++h2)
                            d[h2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(bh[s2], wf[h2][s2], d[h2], 0, 0, 0);
#pragma unroll
                    for (int s2 = 0; s2 < KS; ++s2)
#pragma unroll
                        for (int h2 = 0; h2 < 2; ++h2)
                            d[h2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(bl[s2], wf[h2][s2] * (_Float16)0x1p-11f,
                                                                          d[h2], 0, 0, 0);
#pragma unroll
                    for (int h2 = 0; h2 < 2; ++h2)
#pragma unroll
                        for (int r = 0; r < 16; ++r) S[2 * g + h2][r] = fmaf(d[h2][r], iv[h2], S[2 * g + h2][r]);
                }
            }
            }
            __syncthreads();  // done with this by's ring slot, fragments and norms
            if (by + 1 < nby) {
                u32x4 pf[PF];
                fetch_frags(by + 1, pf);
                store_row(wy0 + by + TH + 1, cpre);
                store_frags(pf);
                __syncthreads();
                row_sq(wy0 + by + TH + 1);
                cpre = fetch_row(wy0 + by + TH + 2);
            }
        }
    };
    if (exact)
        walk(IntTag<kModeExact>{});
    else
        walk(IntTag<kModeWide>{});

    // scores[(wy * win_x + wx) * K + k] = bias_k + cs_k * S[k][window] (cs_k = 1
    // in exact mode).
    const float *cs = reinterpret_cast<const float *>(tp + (int64_t)nby * NFRAG * 64 * 16);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int rho = NARROW ? wave + 4 * q : wave + 4 * (q >> 1), mu = NARROW ? 0 : q & 1;
        const int wx = wx0 + 32 * mu + n, wy = wy0 + rho;
        if (wx < v.win_x && wy < v.win_y) {
            float *out = scores + v.score_off + ((int64_t)wy * v.win_x + wx) * a.k;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int kr = 8 * (r >> 2) + 4 * h + (r & 3);
                if (kk0 + kr < a.k)
                    out[kk0 + kr] = (float)((double)bias[kk0 + kr] + (double)((exact ? 1.f : cs[kr]) * S[q][r]));
            }
        }
    }
}

template <int NBP>
__global__ __launch_bounds__(256, NBP == 8 ? 3 : 1) void k_score_wgemm(const Level *__restrict__ lv,
                                                                      const int32_t *__restrict__ first,
                                                                      int n_levels, WgArgs a,
                                                                      const uint8_t *__restrict__ ws,
                                                                      const float *__restrict__ bias,
                                                                      float *__restrict__ scores)
{
    __shared__ WgLds<NBP> lds;
    const int wg = (int)blockIdx.x;
    if (wg >= first[n_levels]) return;  // whole workgroup
    const int l = find_level(first, n_levels, wg);
    const Level &v = lv[l];
    // The plan tiles a level the same way (wgemm_narrow).
    if (wgemm_narrow(v.win_x))
        wgemm_tile<NBP, true>(lds, v, wg - first[l], a, ws, bias, scores);
    else
        wgemm_tile<NBP, false>(lds, v, wg - first[l], a, ws, bias, scores);
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
    float ss = 0.f;
    for (int vv = 0; vv < 2; ++vv)
        for (int uu = 0; uu < 2; ++uu)
            for (int n = 0; n < nb; ++n) {
                const float h = (float)cache[cache_index(v, n, by + vv, bx + uu)];
                ss = fmaf(h, h, ss);
            }
    const float iv = inv_block_norm(ss, eps);
    float *o = out + v.block_off + (int64_t)rel * 4 * nb;
    for (int vv = 0; vv < 2; ++vv)
        for (int uu = 0; uu < 2; ++uu)
            for (int n = 0; n < nb; ++n) {
                const float h = (float)cache[cache_index(v, n, by + vv, bx + uu)];
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

// Workgroups of `block` threads (no dynamic LDS) of a persistent kernel that
// one CU holds at once, from the runtime's occupancy calculator (at least 1).
// A persistent grid larger than what is resident would leave its last
// workgroups to run as a second, thinly occupied round.
template <typename K>
int resident_blocks(K kernel, int block)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

// Persistent grid over `items` wave items: at most one item per wave, at
// most per_cu workgroups of `waves` waves per CU.
inline unsigned persistent_grid(const PlanDev &p, int64_t items, int64_t waves, int per_cu)
{
    return (unsigned)std::min<int64_t>((items + waves - 1) / waves, (int64_t)per_cu * p.n_cu);
}

}  // namespace

int bin_map_blocks_per_cu(bool soft, int channels)
{
    static const int l2_1 = resident_blocks(k_bin_map<1, false, true>, 256);
    static const int l2_3 = resident_blocks(k_bin_map<3, false, true>, 256);
    static const int soft_1 = resident_blocks(k_bin_map<1, true>, 256);
    static const int soft_3 = resident_blocks(k_bin_map<3, true>, 256);
    if (soft) return channels == 1 ? soft_1 : soft_3;
    return channels == 1 ? l2_1 : l2_3;
}

hipError_t launch_bin_map(const PlanDev &p, const uint8_t *lut_half, const uint8_t *lut_full,
                          const uint8_t *img, int64_t img_pitch, uint8_t *bins, hipStream_t stream)
{
    const int64_t items = p.total[KB_BINMAP];
    if (items == 0) return hipSuccess;
    const int64_t per_block = 16;  // waves of a 1024-thread workgroup
    if (p.lut_global) {  // no LDS table: 4-wave workgroups, as many per CU as its registers allow
        const int per_cu = bin_map_blocks_per_cu(false, p.channels);
        if (p.channels == 1) {
            hipLaunchKernelGGL((k_bin_map<1, false, true>), dim3(persistent_grid(p, items, 4, per_cu)), dim3(256), 0,
                               stream, p.levels, first_of(p, KB_BINMAP), p.n_levels, p.mapx, p.mapy, img,
                               img_pitch, p.n_bins, lut_full, nullptr, bins);
        } else {
            hipLaunchKernelGGL((k_bin_map<3, false, true>), dim3(persistent_grid(p, items, 4, per_cu)), dim3(256), 0,
                               stream, p.levels, first_of(p, KB_BINMAP), p.n_levels, p.mapx, p.mapy, img,
                               img_pitch, p.n_bins, lut_full, nullptr, bins);
        }
        return hipGetLastError();
    }
    const unsigned grid = (unsigned)std::min<int64_t>((items + per_block - 1) / per_block, p.n_cu);
    if (p.channels == 1)
        hipLaunchKernelGGL((k_bin_map<1, false>), dim3(grid), dim3(1024), 0, stream, p.levels,
                           first_of(p, KB_BINMAP), p.n_levels, p.mapx, p.mapy, img, img_pitch,
                           p.n_bins, lut_half, nullptr, bins);
    else
        hipLaunchKernelGGL((k_bin_map<3, false>), dim3(grid), dim3(1024), 0, stream, p.levels,
                           first_of(p, KB_BINMAP), p.n_levels, p.mapx, p.mapy, img, img_pitch,
                           p.n_bins, lut_half, nullptr, bins);
    return hipGetLastError();
}

hipError_t launch_bin_map_soft(const PlanDev &p, const uint16_t *soft_lut, const uint8_t *img,
                               int64_t img_pitch, uint8_t *bins, hipStream_t stream)
{
    const int64_t items = p.total[KB_BINMAP];
    if (items == 0) return hipSuccess;
    // No LDS table: 4-wave workgroups, as many per CU as its registers allow.
    const int per_cu = bin_map_blocks_per_cu(true, p.channels);
    if (p.channels == 1) {
        hipLaunchKernelGGL((k_bin_map<1, true>), dim3(persistent_grid(p, items, 4, per_cu)), dim3(256), 0, stream,
                           p.levels, first_of(p, KB_BINMAP), p.n_levels, p.mapx, p.mapy, img, img_pitch,
                           p.n_bins, nullptr, soft_lut, bins);
    } else {
        hipLaunchKernelGGL((k_bin_map<3, true>), dim3(persistent_grid(p, items, 4, per_cu)), dim3(256), 0, stream,
                           p.levels, first_of(p, KB_BINMAP), p.n_levels, p.mapx, p.mapy, img, img_pitch,
                           p.n_bins, nullptr, soft_lut, bins);
    }
    return hipGetLastError();
}

hipError_t launch_soft_integral(const PlanDev &p, const uint8_t *bins, uint8_t *ws, uint32_t *ii,
                                bool cells, hipStream_t stream)
{
    if (p.total[KB_SSEG] == 0) return hipSuccess;
    const size_t lds = (size_t)kTile * (2 * kTile + 4) + (size_t)((p.n_bins + 1) / 2 + 1) * 64 * 4 * 2;  // + spare slots
    hipLaunchKernelGGL(k_soft_reduce, dim3((unsigned)p.total[KB_SSEG]), dim3(64), lds, stream, p.levels,
                       first_of(p, KB_SSEG), p.n_levels, p.n_bins, bins, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_soft_scan, dim3(blocks_for(p.total[KB_SSCAN], 256)), dim3(256), 0, stream, p.levels,
                       first_of(p, KB_SSCAN), p.n_levels, p.n_bins, ws);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(blocks_for(p.total[KB_SEMIT], 4));
    if (cells)
        hipLaunchKernelGGL(k_soft_emit<true>, grid, dim3(256), 0, stream, p.levels, first_of(p, KB_SEMIT),
                           p.n_levels, p.n_bins, bins, ws, ii);
    else
        hipLaunchKernelGGL(k_soft_emit<false>, grid, dim3(256), 0, stream, p.levels, first_of(p, KB_SEMIT),
                           p.n_levels, p.n_bins, bins, ws, ii);
    return hipGetLastError();
}

hipError_t launch_int_reduce(const PlanDev &p, const uint8_t *bins, uint8_t *ws, hipStream_t stream)
{
    const int64_t tiles = p.total[KB_ITILE];
    if (tiles == 0) return hipSuccess;
    const size_t lds = (size_t)kTile * 68 + (size_t)((p.n_bins + 3) / 4 + 1) * 64 * 4 * 2;  // + spare slots
    hipLaunchKernelGGL(k_int_reduce, dim3((unsigned)tiles), dim3(64), lds, stream, p.levels,
                       first_of(p, KB_ITILE), p.n_levels, p.n_bins, bins, ws);
    return hipGetLastError();
}

static StripArgs strip_args(const PlanDev &p);

bool scan_runs_prep(const PlanDev &p) { return p.scorer == 1 && p.total[KB_STILE] > 0; }

hipError_t launch_int_scan(const PlanDev &p, uint8_t *ws, hipStream_t stream, const float *tmpl)
{
    ScanRanges r;
    // The strip scorer's template prep rides along when tmpl is given.
    const bool prep = tmpl && scan_runs_prep(p);
    const StripArgs pa = prep ? strip_args(p) : StripArgs{};
    r.prep_blocks = prep ? pa.k : 0;
    r.rows_blocks = (int)blocks_for(p.total[KB_ESCAN], kScanThreads);
    r.cols_blocks = (int)blocks_for(p.total[KB_CSCAN], kScanThreads);
    const int tile_blocks = (int)blocks_for(p.total[KB_PSCAN], kScanWaves);
    const int n = r.prep_blocks + r.rows_blocks + r.cols_blocks + tile_blocks;
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)n), block(kScanThreads);
    const int32_t *fe = first_of(p, KB_ESCAN), *fc = first_of(p, KB_CSCAN), *fp = first_of(p, KB_PSCAN);
    switch (prep ? p.mfma_ks : 0) {
    case 0: hipLaunchKernelGGL(k_int_scan<0>, grid, block, 0, stream, p.levels, fe, fc, fp, p.n_levels, p.n_bins, r, ws, pa, tmpl); break;
    case 8: hipLaunchKernelGGL(k_int_scan<8>, grid, block, 0, stream, p.levels, fe, fc, fp, p.n_levels, p.n_bins, r, ws, pa, tmpl); break;
    case 16: hipLaunchKernelGGL(k_int_scan<16>, grid, block, 0, stream, p.levels, fe, fc, fp, p.n_levels, p.n_bins, r, ws, pa, tmpl); break;
    case 20: hipLaunchKernelGGL(k_int_scan<20>, grid, block, 0, stream, p.levels, fe, fc, fp, p.n_levels, p.n_bins, r, ws, pa, tmpl); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// k_int_emit for chunks of NBC bins (the last one possibly shorter), with or
// without the fused cell cache, for PB-byte plane elements.
#define HOG_EMIT_CASE(NBC)                                                                          \
    case NBC:                                                                                       \
        if (cells)                                                                                  \
            hipLaunchKernelGGL((k_int_emit<NBC, true, PB>), grid, dim3(256), 0, stream, p.levels,   \
                               first_of(p, KB_ITILE), p.n_levels, p.n_bins, p.n_chunks, bins, ws,   \
                               ii);                                                                 \
        else                                                                                        \
            hipLaunchKernelGGL((k_int_emit<NBC, false, PB>), grid, dim3(256), 0, stream, p.levels,  \
                               first_of(p, KB_ITILE), p.n_levels, p.n_bins, p.n_chunks, bins, ws,   \
                               ii);                                                                 \
        break;

template <int PB>
static hipError_t launch_int_emit_pb(const PlanDev &p, const uint8_t *bins, uint8_t *ws, uint8_t *ii,
                                     hipStream_t stream)
{
    const bool cells = p.cell == 8;
    const dim3 grid(blocks_for(p.total[KB_ITILE] * p.n_chunks, 4));
    static_assert(kMaxBinChunk == 6, "one case per chunk size");
    switch (p.bin_chunk) {
        HOG_EMIT_CASE(1) HOG_EMIT_CASE(2) HOG_EMIT_CASE(3) HOG_EMIT_CASE(4) HOG_EMIT_CASE(5)
        HOG_EMIT_CASE(6)
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_int_emit(const PlanDev &p, const uint8_t *bins, uint8_t *ws, void *ii,
                           hipStream_t stream)
{
    if (p.total[KB_ITILE] == 0) return hipSuccess;
    uint8_t *iib = static_cast<uint8_t *>(ii);
    switch (p.plane_bytes) {
    case 4: return launch_int_emit_pb<4>(p, bins, ws, iib, stream);
    case 2: return launch_int_emit_pb<2>(p, bins, ws, iib, stream);
    case 1: return launch_int_emit_pb<1>(p, bins, ws, iib, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cells(const PlanDev &p, const void *ii, uint8_t *ws, uint32_t *cell_hist,
                        hipStream_t stream)
{
    const int64_t n = p.total[KB_CELL];
    if (n == 0) return hipSuccess;
    const dim3 grid(blocks_for(n, 256));
    const int32_t *f = first_of(p, KB_CELL);
    switch (p.plane_bytes) {
    case 4:
        hipLaunchKernelGGL(k_cells<uint32_t>, grid, dim3(256), 0, stream, p.levels, f, p.n_levels, p.n_bins, p.cell,
                           static_cast<const uint32_t *>(ii), ws, cell_hist);
        break;
    case 2:
        hipLaunchKernelGGL(k_cells<uint16_t>, grid, dim3(256), 0, stream, p.levels, f, p.n_levels, p.n_bins, p.cell,
                           static_cast<const uint16_t *>(ii), ws, cell_hist);
        break;
    case 1:
        hipLaunchKernelGGL(k_cells<uint8_t>, grid, dim3(256), 0, stream, p.levels, f, p.n_levels, p.n_bins, p.cell,
                           static_cast<const uint8_t *>(ii), ws, cell_hist);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cache_export(const PlanDev &p, const uint8_t *ws, uint32_t *cell_hist,
                               hipStream_t stream)
{
    const int64_t n = p.total[KB_CELL];
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cache_export, dim3(blocks_for(n, 256)), dim3(256), 0, stream, p.levels,
                       first_of(p, KB_CELL), p.n_levels, p.n_bins, ws, cell_hist);
    return hipGetLastError();
}

static WgArgs wg_args(const PlanDev &p)
{
    WgArgs m;
    m.nb = p.n_bins;
    m.nby = p.win_cells_y - 1;
    m.k = p.n_templates;
    m.dim = p.feat_dim;
    m.tprep_off = p.tprep_off;
    m.tprep_stride = p.tprep_stride;
    m.eps = p.eps_counts;  // the matrix-core scorers work on cell counts
    return m;
}

static StripArgs strip_args(const PlanDev &p)
{
    StripArgs m;
    m.nb = p.n_bins;
    m.nby = p.win_cells_y - 1;
    m.k = p.n_templates;
    m.th = p.st_th;
    m.dim = p.feat_dim;
    m.lds_wave = p.st_lds_bytes / 4;
    m.tprep_off = p.tprep_off;
    m.tprep_stride = p.tprep_stride;
    m.eps = p.eps_counts;  // the matrix-core scorers work on cell counts
    return m;
}

hipError_t launch_score_prep(const PlanDev &p, uint8_t *ws, const float *tmpl, hipStream_t stream)
{
    if (p.total[KB_STILE] == 0) return hipSuccess;
    if (p.scorer == 2) {
        const WgArgs m = wg_args(p);
        const unsigned ktiles = (unsigned)((m.k + 31) / 32);
        // Fragments per tile: [by][bx][step][hi|lo][lane].
        const int64_t n_frag = (int64_t)m.nby * kStripMaxBX * (p.mfma_ks / 4) * 2 * 64;
        const dim3 fgrid(blocks_for(n_frag, 256), ktiles);
        hipLaunchKernelGGL(k_score_prep_wg_scale, dim3(32 * ktiles), dim3(64), 0, stream, m, tmpl, ws, n_frag * 16);
        switch (p.mfma_ks) {
        case 8: hipLaunchKernelGGL(k_score_prep_wg<8>, fgrid, dim3(256), 0, stream, m, tmpl, ws); break;
        case 16: hipLaunchKernelGGL(k_score_prep_wg<16>, fgrid, dim3(256), 0, stream, m, tmpl, ws); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (p.scorer == 1) {
        const StripArgs m = strip_args(p);
        const dim3 pgrid((unsigned)m.k), pblock(64 * kStripMaxBX);
        switch (p.mfma_ks) {
        case 8: hipLaunchKernelGGL(k_score_prep<8>, pgrid, pblock, 0, stream, m, tmpl, ws); break;
        case 16: hipLaunchKernelGGL(k_score_prep<16>, pgrid, pblock, 0, stream, m, tmpl, ws); break;
        case 20: hipLaunchKernelGGL(k_score_prep<20>, pgrid, pblock, 0, stream, m, tmpl, ws); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    return hipSuccess;  // the vector scorer reads the templates as given
}

hipError_t launch_score(const PlanDev &p, const uint8_t *ws, const float *tmpl, const float *bias,
                        float *scores, hipStream_t stream, bool prep)
{
    const int64_t n = p.total[KB_STILE];
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)n), block(256);
    const int32_t *f = first_of(p, KB_STILE);
    if (prep) {
        // The prepared weights are rewritten in the workspace by every such call.
        hipError_t e = launch_score_prep(p, const_cast<uint8_t *>(ws), tmpl, stream);
        if (e != hipSuccess) return e;
    }
    if (p.scorer == 2) {
        const WgArgs m = wg_args(p);
        switch (p.mfma_ks) {
        case 8: hipLaunchKernelGGL(k_score_wgemm<8>, grid, block, 0, stream, p.levels, f, p.n_levels, m, ws, bias, scores); break;
        case 16: hipLaunchKernelGGL(k_score_wgemm<16>, grid, block, 0, stream, p.levels, f, p.n_levels, m, ws, bias, scores); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (p.scorer == 1) {
        const StripArgs m = strip_args(p);
        const dim3 sgrid(blocks_for(n, 4));
        const size_t lds = (size_t)p.st_lds_bytes;
        switch (p.mfma_ks) {
        case 8: hipLaunchKernelGGL(k_score_strip<8>, sgrid, block, lds, stream, p.levels, f, p.n_levels, m, ws, bias, scores); break;
        case 16: hipLaunchKernelGGL(k_score_strip<16>, sgrid, block, lds, stream, p.levels, f, p.n_levels, m, ws, bias, scores); break;
        case 20: hipLaunchKernelGGL(k_score_strip<20>, sgrid, block, lds, stream, p.levels, f, p.n_levels, m, ws, bias, scores); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
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
    a.vscale = p.vscale;
    const size_t lds = (size_t)p.st_lds_bytes;
    if (p.scorer == 3) {
        const dim3 rblock((unsigned)(64 * p.st_waves));
        if (p.win_cells_x == 8 && p.n_bins == 8)
            hipLaunchKernelGGL((k_score_raw<8, 8>), grid, rblock, lds, stream, p.levels, f, p.n_levels, a,
                               ws, tmpl, bias, scores);
        else if (p.win_cells_x == 8 && p.n_bins == 9)
            hipLaunchKernelGGL((k_score_raw<9, 8>), grid, rblock, lds, stream, p.levels, f, p.n_levels, a,
                               ws, tmpl, bias, scores);
        else if (p.win_cells_x == 8 && p.n_bins == 18)
            hipLaunchKernelGGL((k_score_raw<18, 8>), grid, rblock, lds, stream, p.levels, f, p.n_levels, a,
                               ws, tmpl, bias, scores);
        else
            hipLaunchKernelGGL((k_score_raw<0, 0>), grid, rblock, lds, stream, p.levels, f, p.n_levels, a,
                               ws, tmpl, bias, scores);
        return hipGetLastError();
    }
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
                       first_of(p, KB_BLOCK), p.n_levels, p.n_bins, p.eps_counts, ws, block_feat);
    return hipGetLastError();
}

}  // namespace hogk
