// Host half of libhog: argument checking, the lookup table (Sec. 2), level
// planning and buffer layout, launches, errors and kernel timing. Every
// public entry point is declared in include/hog.h.
#include "hog.h"
#include "hog_internal.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using hogk::Level;
using hogk::PlanDev;

namespace {

thread_local std::string g_last_error;

hog_status fail(hog_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

hog_status device_fail(hipError_t e, const char *what)
{
    return fail(HOG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// ---------------------------------------------------------------------------
// Kernel timing: HIP event pairs around each launch, on the launch stream.
// ---------------------------------------------------------------------------
struct PendingTiming {
    std::string name;
    hipEvent_t start, stop;
};
bool g_timing_on = false;
thread_local bool g_capturing = false;  // inside hog_graph_create: no timing events
thread_local bool g_no_alloc = false;   // inside hog_run_static: no timing events either
std::vector<PendingTiming> g_pending;
std::vector<hipEvent_t> g_event_pool;
std::map<std::string, std::pair<int64_t, double>> g_timing_totals;

hipError_t take_event(hipEvent_t *ev)
{
    if (!g_event_pool.empty()) {
        *ev = g_event_pool.back();
        g_event_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

template <class F>
hipError_t timed_launch(const char *name, hipStream_t stream, F &&launch)
{
    if (!g_timing_on || g_capturing || g_no_alloc) return launch();
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = take_event(&a);
    if (e == hipSuccess) e = take_event(&b);
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(a, stream)) != hipSuccess) return e;
    const hipError_t le = launch();
    if ((e = hipEventRecord(b, stream)) != hipSuccess) return e;
    g_pending.push_back({name, a, b});
    return le;
}

hipError_t drain_timing()
{
    hipError_t first_err = hipSuccess;
    for (auto &p : g_pending) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(p.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.start, p.stop);
        if (e != hipSuccess && first_err == hipSuccess) first_err = e;
        auto &tot = g_timing_totals[p.name];
        tot.first += 1;
        tot.second += ms;
        g_event_pool.push_back(p.start);
        g_event_pool.push_back(p.stop);
    }
    g_pending.clear();
    return first_err;
}

// ---------------------------------------------------------------------------
// Sec. 2: the bin of one integer gradient. Angle in [0, 2 pi) from +x towards
// +y, n half-open sectors of 2 pi / n. Integer gradients lie exactly on a
// multiple of pi/4 only along the axes and diagonals (Niven's theorem rules
// out any other rational slope at a rational multiple of pi); those are the
// only places a sector edge can be hit exactly, and there the sector is
// floor(m n / 8) for the direction m pi/4, computed in integers. Elsewhere
// the FP64 angle is far (> 1e-9 of a sector) from every edge.
// ---------------------------------------------------------------------------
// Unsigned orientation folds the angle into [0, pi): sectors of pi / n, and
// on the axes and diagonals floor((m mod 4) n / 4).
uint8_t lut_entry(int dx, int dy, int n, bool folded)
{
    if (dx == 0 && dy == 0) return HOG_NO_BIN;
    if (dx == 0 || dy == 0 || dx == dy || dx == -dy) {
        int m;
        if (dy == 0) m = dx > 0 ? 0 : 4;
        else if (dx == 0) m = dy > 0 ? 2 : 6;
        else if (dx > 0) m = dy > 0 ? 1 : 7;
        else m = dy > 0 ? 3 : 5;
        return folded ? (uint8_t)(((m % 4) * n) / 4) : (uint8_t)((m * n) / 8);
    }
    const double pi = 3.14159265358979323846264338327950;
    const double range = folded ? pi : 2.0 * pi;
    double a = std::atan2((double)dy, (double)dx);
    if (a < 0.0) a += 2.0 * pi;
    if (folded && a >= pi) a -= pi;
    int k = (int)std::floor(a * (double)n / range);
    if (k >= n) k = n - 1;
    return (uint8_t)k;
}

// Soft vote (Sec. 2's two-bin split, quantised): with a the angle in bin
// widths minus 1/2, b0 = floor(a) mod n and w1 = floor(frac(a) Q + 1/2)
// units go to b0 + 1. On the axes and diagonals a is the rational
// (m n - 4) / 8 (signed) or ((m mod 4) n - 2) / 4 (unsigned) and is taken in
// integers; elsewhere in FP64. Returns b0 | w1 << 8, or 255.
uint16_t soft_entry(int dx, int dy, int n, bool folded)
{
    constexpr int Q = HOG_SOFT_QUANTUM;
    if (dx == 0 && dy == 0) return HOG_NO_BIN;
    int b0, w1;
    if (dx == 0 || dy == 0 || dx == dy || dx == -dy) {
        int m;
        if (dy == 0) m = dx > 0 ? 0 : 4;
        else if (dx == 0) m = dy > 0 ? 2 : 6;
        else if (dx > 0) m = dy > 0 ? 1 : 7;
        else m = dy > 0 ? 3 : 5;
        const int den = folded ? 4 : 8;
        const int num = folded ? (m % 4) * n - 2 : m * n - 4;
        const int fl = (num >= 0 ? num : num - den + 1) / den;  // floor
        const int r = num - fl * den;                            // 0 .. den - 1
        b0 = ((fl % n) + n) % n;
        w1 = r * Q / den;
    } else {
        const double pi = 3.14159265358979323846264338327950;
        const double range = folded ? pi : 2.0 * pi;
        double t = std::atan2((double)dy, (double)dx);
        if (t < 0.0) t += folded ? pi : 2.0 * pi;
        const double a = t * (double)n / range - 0.5;
        const double fl = std::floor(a);
        w1 = (int)std::floor((a - fl) * Q + 0.5);
        b0 = (((int)fl % n) + n) % n;
    }
    return (uint16_t)(b0 | w1 << 8);
}

}  // namespace

// ---------------------------------------------------------------------------
struct hog_lut {
    int n_bins;
    int orientation;
    std::vector<uint8_t> host;
    uint8_t *dev;       // full table, 511 * 511 bytes
    uint8_t *dev_half;  // dy >= 0 half with mirror flags, as the kernels stage it in LDS
    uint16_t *dev_soft; // soft-vote table, 511 * 511 entries b0 | w1 << 8
};

// Streams and events of a grouped run (level groups on concurrent streams):
// group g > 0 runs on s[g - 1]; mid[g] is recorded when group g's planes
// start, join[g - 1] when group g's scores are done.
struct GroupStreams {
    hipStream_t s[HOG_MAX_LEVEL_GROUPS - 1];
    hipEvent_t mid[HOG_MAX_LEVEL_GROUPS];
    hipEvent_t join[HOG_MAX_LEVEL_GROUPS - 1];
};

struct hog_plan {
    hog_plan_desc desc;  // image 0's (shared fields are equal across images)
    bool batch;          // images packed in one buffer; hog_bin_map takes img_pitch 0
    int device;          // the device holding dev_mem
    std::vector<hog_image_info> images;
    std::vector<Level> levels;
    std::vector<hog_level_info> info;
    std::vector<int32_t> first;  // host copy of the per-kernel prefix tables
    size_t first_off;            // their offset in dev_mem
    size_t gfirst_off;           // offset in dev_mem of the level groups' prefix tables
    hog_plan_sizes sizes;
    PlanDev dev;
    void *dev_mem;
    // Level groups (hog_tiles.level_groups): views of dev over contiguous
    // level ranges, each with its own prefix tables; empty for one group.
    std::vector<PlanDev> groups;
    // The plan's own streams for grouped hog_run calls (created on first
    // use), and the lock that keeps one grouped enqueue at a time on them.
    bool have_gs = false;
    GroupStreams gs;
    std::mutex gs_mu;
};

namespace hogk {
void set_last_error(const char *msg) { g_last_error = msg ? msg : ""; }
}  // namespace hogk

extern "C" {

const char *hog_last_error(void) { return g_last_error.c_str(); }

hog_status hog_lut_fill_host_ex(int n_bins, int orientation, uint8_t *table)
{
    if (n_bins < 1 || n_bins > HOG_MAX_BINS)
        return fail(HOG_E_INVALID, "n_bins must be in [1, %d], got %d", HOG_MAX_BINS, n_bins);
    if (orientation != HOG_ORIENT_SIGNED && orientation != HOG_ORIENT_UNSIGNED)
        return fail(HOG_E_INVALID, "orientation must be HOG_ORIENT_SIGNED or HOG_ORIENT_UNSIGNED, got %d",
                    orientation);
    if (!table) return fail(HOG_E_INVALID, "table is NULL");
    const bool folded = orientation == HOG_ORIENT_UNSIGNED;
    for (int dy = -255; dy <= 255; ++dy)
        for (int dx = -255; dx <= 255; ++dx)
            table[(dy + 255) * HOG_LUT_SIDE + (dx + 255)] = lut_entry(dx, dy, n_bins, folded);
    return HOG_OK;
}

hog_status hog_lut_fill_soft_host(int n_bins, int orientation, uint16_t *table)
{
    if (n_bins < 1 || n_bins > HOG_MAX_BINS)
        return fail(HOG_E_INVALID, "n_bins must be in [1, %d], got %d", HOG_MAX_BINS, n_bins);
    if (orientation != HOG_ORIENT_SIGNED && orientation != HOG_ORIENT_UNSIGNED)
        return fail(HOG_E_INVALID, "orientation must be HOG_ORIENT_SIGNED or HOG_ORIENT_UNSIGNED, got %d",
                    orientation);
    if (!table) return fail(HOG_E_INVALID, "table is NULL");
    const bool folded = orientation == HOG_ORIENT_UNSIGNED;
    for (int dy = -255; dy <= 255; ++dy)
        for (int dx = -255; dx <= 255; ++dx)
            table[(dy + 255) * HOG_LUT_SIDE + (dx + 255)] = soft_entry(dx, dy, n_bins, folded);
    return HOG_OK;
}

hog_status hog_lut_fill_host(int n_bins, uint8_t *table)
{
    return hog_lut_fill_host_ex(n_bins, HOG_ORIENT_SIGNED, table);
}

hog_status hog_lut_build(int n_bins, hog_lut **out) { return hog_lut_build_ex(n_bins, HOG_ORIENT_SIGNED, out); }

int hog_lut_orientation(const hog_lut *lut) { return lut ? lut->orientation : -1; }

hog_status hog_lut_build_ex(int n_bins, int orientation, hog_lut **out)
{
    if (!out) return fail(HOG_E_INVALID, "out is NULL");
    *out = nullptr;
    hog_lut *lut = new (std::nothrow) hog_lut;
    if (!lut) return fail(HOG_E_NOMEM, "host allocation failed");
    lut->n_bins = n_bins;
    lut->orientation = orientation;
    lut->dev = nullptr;
    lut->dev_half = nullptr;
    lut->dev_soft = nullptr;
    try {
        lut->host.resize((size_t)HOG_LUT_SIDE * HOG_LUT_SIDE);
    } catch (...) {
        delete lut;
        return fail(HOG_E_NOMEM, "host allocation failed");
    }
    hog_status st = hog_lut_fill_host_ex(n_bins, orientation, lut->host.data());
    if (st != HOG_OK) {
        delete lut;
        return st;
    }
    // Half table: entry (dx, dy >= 0) = bin(dx, dy) | f << 6, where
    // bin(dx, -dy) = n - 1 - bin(dx, dy) + f. Mirroring dy maps the angle t to
    // 2 pi - t (unsigned: t mod pi to pi - t mod pi), so off the sector edges
    // the bin becomes n - 1 - bin and on an edge n - bin; f is read off the
    // full table and checked.
    std::vector<uint8_t> half((size_t)hogk::kLutHalfBytes, 0);
    for (int dy = 0; dy <= 255; ++dy)
        for (int dx = -255; dx <= 255; ++dx) {
            const uint8_t up = lut->host[(dy + 255) * HOG_LUT_SIDE + (dx + 255)];
            const uint8_t dn = lut->host[(-dy + 255) * HOG_LUT_SIDE + (dx + 255)];
            uint8_t e = up;
            if (up != HOG_NO_BIN && dy > 0) {
                const int f = (int)dn - (n_bins - 1 - (int)up);
                if (f != 0 && f != 1) {
                    delete lut;
                    return fail(HOG_E_INVALID, "lookup table is not mirror-symmetric at (%d,%d)", dx, dy);
                }
                e = (uint8_t)(up | (f << 6));
            }
            half[(size_t)dy * HOG_LUT_SIDE + (dx + 255)] = e;
        }
    std::vector<uint16_t> soft((size_t)HOG_LUT_SIDE * HOG_LUT_SIDE);
    (void)hog_lut_fill_soft_host(n_bins, orientation, soft.data());  // arguments checked above
    hipError_t e = hipMalloc((void **)&lut->dev, lut->host.size());
    if (e == hipSuccess) e = hipMalloc((void **)&lut->dev_half, half.size());
    if (e == hipSuccess) e = hipMalloc((void **)&lut->dev_soft, soft.size() * 2);
    if (e != hipSuccess) {
        hog_lut_free(lut);
        return device_fail(e, "hipMalloc(lut)");
    }
    e = hipMemcpy(lut->dev, lut->host.data(), lut->host.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(lut->dev_half, half.data(), half.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(lut->dev_soft, soft.data(), soft.size() * 2, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hog_lut_free(lut);
        return device_fail(e, "hipMemcpy(lut)");
    }
    *out = lut;
    return HOG_OK;
}

void hog_lut_free(hog_lut *lut)
{
    if (!lut) return;
    if (lut->dev) (void)hipFree(lut->dev);
    if (lut->dev_half) (void)hipFree(lut->dev_half);
    if (lut->dev_soft) (void)hipFree(lut->dev_soft);
    delete lut;
}

int hog_lut_bins(const hog_lut *lut) { return lut ? lut->n_bins : 0; }

const uint8_t *hog_lut_host(const hog_lut *lut) { return lut ? lut->host.data() : nullptr; }

hog_status hog_lut_read_device(const hog_lut *lut, int table, void *dst, int64_t bytes)
{
    if (!lut || !dst) return fail(HOG_E_INVALID, "lut or dst is NULL");
    const void *src = nullptr;
    int64_t size = 0;
    switch (table) {
    case HOG_LUT_DEVICE_FULL: src = lut->dev; size = (int64_t)HOG_LUT_SIDE * HOG_LUT_SIDE; break;
    case HOG_LUT_DEVICE_HALF: src = lut->dev_half; size = hogk::kLutHalfBytes; break;
    case HOG_LUT_DEVICE_SOFT: src = lut->dev_soft; size = (int64_t)HOG_LUT_SIDE * HOG_LUT_SIDE * 2; break;
    default: return fail(HOG_E_INVALID, "unknown table %d", table);
    }
    if (bytes != size) return fail(HOG_E_INVALID, "table %d has %lld bytes, not %lld", table, (long long)size,
                                   (long long)bytes);
    const hipError_t e = hipMemcpy(dst, src, (size_t)size, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_fail(e, "hipMemcpy(lut table)");
    return HOG_OK;
}

// ---------------------------------------------------------------------------
// Planning.
// ---------------------------------------------------------------------------
static hog_status check_desc(const hog_plan_desc *d)
{
    if (!d) return fail(HOG_E_INVALID, "desc is NULL");
    if (d->width < 1 || d->height < 1 || d->width > 32767 || d->height > 32767)
        return fail(HOG_E_INVALID, "image size %dx%d outside [1, 32767]", d->width, d->height);
    if (d->channels != 1 && d->channels != 3)
        return fail(HOG_E_INVALID, "channels must be 1 or 3, got %d", d->channels);
    if (d->n_bins < 1 || d->n_bins > HOG_MAX_BINS)
        return fail(HOG_E_INVALID, "n_bins must be in [1, %d], got %d", HOG_MAX_BINS, d->n_bins);
    if (d->max_levels < 0 || d->max_levels > 256)
        return fail(HOG_E_INVALID, "max_levels must be in [0, 256], got %d", d->max_levels);
    if (d->max_levels != 1 && !(d->scale > 1.0 && d->scale < 1e6))
        return fail(HOG_E_INVALID, "a pyramid needs scale > 1, got %g", d->scale);
    if (d->n_templates < 1 || d->n_templates > 4096)
        return fail(HOG_E_INVALID, "n_templates must be in [1, 4096], got %d", d->n_templates);
    const hog_scan_params &s = d->scan;
    if (s.cell < 1 || s.cell > 32) return fail(HOG_E_INVALID, "cell must be in [1, 32], got %d", s.cell);
    if (s.win_cells_x < 1 || s.win_cells_x > 64 || s.win_cells_y < 1 || s.win_cells_y > 64)
        return fail(HOG_E_INVALID, "window must be 1..64 cells per side");
    if (s.norm != HOG_NORM_RAW && s.norm != HOG_NORM_L2)
        return fail(HOG_E_INVALID, "norm must be HOG_NORM_RAW or HOG_NORM_L2");
    if (s.norm == HOG_NORM_L2) {
        if (s.block != 2) return fail(HOG_E_INVALID, "L2 blocks must be 2x2 cells");
        if (s.win_cells_x < 2 || s.win_cells_y < 2)
            return fail(HOG_E_INVALID, "an L2 window needs at least 2x2 cells");
        if (!(s.eps >= 0.f) || !std::isfinite(s.eps)) return fail(HOG_E_INVALID, "eps must be finite and >= 0");
    }
    const int pbits = d->plane_bits == 0 ? 32 : d->plane_bits;
    if (pbits != 32 && pbits != 16 && pbits != 8)
        return fail(HOG_E_INVALID, "plane_bits must be 32, 16 or 8 (0 = 32), got %d", d->plane_bits);
    if (d->votes != HOG_VOTES_HARD && d->votes != HOG_VOTES_SOFT)
        return fail(HOG_E_INVALID, "votes must be HOG_VOTES_HARD or HOG_VOTES_SOFT, got %d", d->votes);
    if (d->votes == HOG_VOTES_SOFT) {
        if (pbits != 32) return fail(HOG_E_INVALID, "soft votes need 32-bit planes");
        if ((int64_t)d->width * d->height * HOG_SOFT_QUANTUM >= ((int64_t)1 << 32))
            return fail(HOG_E_INVALID, "soft votes: width * height * %d must stay below 2^32", HOG_SOFT_QUANTUM);
    }
    // A cell's four-corner sum taken mod 2^bits is exact below 2^bits pixels.
    if ((int64_t)s.cell * s.cell >= ((int64_t)1 << pbits))
        return fail(HOG_E_INVALID, "%d-pixel cells hold up to %d pixels, too many for %d-bit planes", s.cell,
                    s.cell * s.cell, pbits);
    return HOG_OK;
}

static int plane_bytes_of(const hog_plan_desc &d) { return (d.plane_bits == 0 ? 32 : d.plane_bits) / 8; }

static bool same_scan(const hog_scan_params &a, const hog_scan_params &b)
{
    return a.cell == b.cell && a.win_cells_x == b.win_cells_x && a.win_cells_y == b.win_cells_y &&
           a.block == b.block && a.norm == b.norm && (a.eps == b.eps || a.norm == HOG_NORM_RAW);
}

// Builds a plan over n_img images (batch: packed input, per-level pitch).
static hog_status create_plan(const hog_plan_desc *descs, int n_img, bool batch, hog_plan **out)
{
    if (!out) return fail(HOG_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!descs) return fail(HOG_E_INVALID, "desc is NULL");
    if (n_img < 1 || n_img > 65536) return fail(HOG_E_INVALID, "n_images must be in [1, 65536], got %d", n_img);
    for (int i = 0; i < n_img; ++i) {
        hog_status st = check_desc(&descs[i]);
        if (st != HOG_OK) return st;
        const hog_plan_desc &a = descs[0], &b = descs[i];
        if (b.channels != a.channels || b.n_bins != a.n_bins || b.n_templates != a.n_templates ||
            !same_scan(a.scan, b.scan) || plane_bytes_of(a) != plane_bytes_of(b) || a.votes != b.votes)
            return fail(HOG_E_INVALID,
                        "image %d: channels, n_bins, n_templates, scan, plane_bits and votes must match image 0",
                        i);
    }
    const hog_plan_desc d0 = descs[0];
    const hog_scan_params &sp = d0.scan;
    const int nb = d0.n_bins, K = d0.n_templates;
    const int pb = plane_bytes_of(d0);  // bytes per plane element
    const bool soft = d0.votes == HOG_VOTES_SOFT;
    const int win_w = sp.cell * sp.win_cells_x, win_h = sp.cell * sp.win_cells_y;
    const int dim = sp.norm == HOG_NORM_RAW
                        ? sp.win_cells_x * sp.win_cells_y * nb
                        : (sp.win_cells_x - 1) * (sp.win_cells_y - 1) * 4 * nb;

    // Scorer. L2 blocks of 2 x 2 cells in windows 8 cells wide and at most 17 high, with
    // at most 20 bins go to the matrix-core scorer: one wave per strip of 16
    // window columns and kStripTH window rows (and per template). Otherwise
    // the vector scorer: tw x th windows per workgroup (<= 256 threads) with
    // the cells they use staged in LDS.
    const int nbp = (int)round_up(nb, 4);
    int best_tw = 0, best_th = 0, mfma_ks = 0, scorer = 0;
    int64_t best_lds = 0;
    const bool l2_8wide = sp.norm == HOG_NORM_L2 && sp.win_cells_x - 1 == hogk::kStripMaxBX &&
                          sp.win_cells_y - 1 <= 16;
    // The matrix-core scorers take cell values exactly in fp16 (integers up to
    // 2048): every hard-vote cell (at most 32 x 32 pixels), soft-vote cells
    // of up to 8 x 8 pixels.
    const bool fp16_exact = !soft || (int64_t)sp.cell * sp.cell * HOG_SOFT_QUANTUM <= 2048;
    if (l2_8wide && fp16_exact && nb <= 16 && K >= 16) {
        // Many templates: the window GEMM, one workgroup per 64 x 8 windows
        // and 32 templates.
        scorer = 2;
        mfma_ks = nb <= 8 ? 8 : 16;
        best_tw = hogk::kWgW;
        best_th = hogk::kWgTH;
    } else if (l2_8wide && fp16_exact && nb <= 20) {
        scorer = 1;
        mfma_ks = nb <= 8 ? 8 : nb <= 16 ? 16 : 20;  // bin slots per cell
        best_tw = hogk::kStripW;
        best_th = hogk::kStripTH;
        const int64_t rowh = (int64_t)(hogk::kStripW + 8) * mfma_ks;  // halves per staged cell row
        best_lds = 4 * round_up(4 * rowh * 2 + 64 * 4 + (int64_t)hogk::kStripW * best_th * 4, 16);
    }
    int raw_waves = 0;
    if (scorer == 0 && sp.norm == HOG_NORM_RAW) {
        // Raw features: 64 windows per workgroup (tw x th = 64, one per lane),
        // min(wcy, 8) waves splitting each window's cell rows; the shape
        // staging the fewest cells per tile that fits 64 KB of LDS. Eight
        // waves rather than one per cell row: one image's step is as fast,
        // and a batch's many tiles overlap more workgroups per CU.
        const int R = std::min(sp.win_cells_y, 8);
        int64_t best_cells = INT64_MAX;
        for (int tw = 64; tw >= 1; tw /= 2) {
            const int th = 64 / tw;
            const int64_t CW = tw + sp.win_cells_x - 1, CH = th + sp.win_cells_y - 1;
            const int64_t lds = round_up(CH * CW * nbp, 2) * 4 + 2 * (int64_t)R * 64 * 8;
            if (lds > 65536 || CH * CW >= best_cells) continue;
            best_cells = CH * CW;
            best_tw = tw;
            best_th = th;
            best_lds = lds;
        }
        if (best_tw > 0) {
            scorer = 3;
            raw_waves = R;
        }
    }
    if (scorer == 0) {
        double best_cost = 1e30;
        for (int tw = 1; tw <= 64; tw *= 2)
            for (int th = 1; tw * th <= 256; th *= 2) {
                const int64_t CW = tw + sp.win_cells_x - 1, CH = th + sp.win_cells_y - 1;
                const int64_t lds = CH * CW * nbp * 4 + (CH - 1) * (CW - 1) * 4;
                if (lds > 65536) continue;
                const double cost = (double)(CH * CW) / (tw * th) + (tw * th < 64 ? 4.0 : 0.0);
                if (cost < best_cost - 1e-9 || (std::fabs(cost - best_cost) <= 1e-9 && tw * th > best_tw * best_th)) {
                    best_cost = cost;
                    best_tw = tw;
                    best_th = th;
                    best_lds = lds;
                }
            }
        if (best_tw == 0)
            return fail(HOG_E_INVALID, "window of %dx%d cells with %d bins does not fit the scorer's LDS",
                        sp.win_cells_x, sp.win_cells_y, nb);
    }

    hog_plan *p = new (std::nothrow) hog_plan;
    if (!p) return fail(HOG_E_NOMEM, "host allocation failed");
    p->desc = d0;
    p->batch = batch;
    p->device = 0;
    p->dev_mem = nullptr;
    std::vector<int32_t> mapx, mapy;

    int64_t bins_off = 0, ii_off = 0, score_off = 0, cell_off = 0, block_off = 0, ws_off = 0;
    int64_t tot_px = 0, tot_win = 0, src_off = 0;
    const int n_chunks = (nb + hogk::kMaxBinChunk - 1) / hogk::kMaxBinChunk;
    const int chunk = (nb + n_chunks - 1) / n_chunks;
    int chunk_final = chunk;
    for (int img = 0; img < n_img; ++img) {
    const hog_plan_desc &d = descs[img];
    hog_image_info ii_info;
    std::memset(&ii_info, 0, sizeof ii_info);
    ii_info.first_level = (int32_t)p->levels.size();
    ii_info.width = d.width;
    ii_info.height = d.height;
    ii_info.img_offset = batch ? src_off : 0;
    ii_info.img_pitch = batch ? (int64_t)d.width * d.channels : 0;
    const int64_t img_px0 = tot_px, img_win0 = tot_win;
    // Levels (nearest-neighbour pyramid): s_0 = 1, s_l = s_{l-1} * scale.
    double s = 1.0;
    for (int l = 0;; ++l) {
        if (d.max_levels > 0 && l >= d.max_levels) break;
        if (l >= 256) break;
        const int lw = (int)std::floor((double)d.width / s);
        const int lh = (int)std::floor((double)d.height / s);
        if (l > 0 && (lw < win_w || lh < win_h || lw < 1 || lh < 1)) break;
        Level v;
        std::memset(&v, 0, sizeof v);
        hog_level_info info;
        std::memset(&info, 0, sizeof info);
        v.w = lw;
        v.h = lh;
        v.cells_x = lw / sp.cell;
        v.cells_y = lh / sp.cell;
        v.cbx = (v.cells_x + 7) / 8;
        v.cby = (v.cells_y + 7) / 8;
        v.win_x = v.cells_x - sp.win_cells_x + 1;
        v.win_y = v.cells_y - sp.win_cells_y + 1;
        if (v.win_x <= 0 || v.win_y <= 0) v.win_x = v.win_y = 0;
        v.tiles_x = (lw + hogk::kTile - 1) / hogk::kTile;
        v.tiles_y = (lh + hogk::kTile - 1) / hogk::kTile;
        v.bm_gx = (lw + hogk::kBinCols - 1) / hogk::kBinCols;
        v.bm_gy = (lh + hogk::kBinRows - 1) / hogk::kBinRows;
        const bool narrow = scorer == 2 && hogk::wgemm_narrow(v.win_x);  // as k_score_wgemm tiles it
        const int tw = narrow ? hogk::kWgW / 2 : best_tw, th = narrow ? 2 * hogk::kWgTH : best_th;
        v.st_x = v.win_x ? (v.win_x + tw - 1) / tw : 0;
        v.st_y = v.win_y ? (v.win_y + th - 1) / th : 0;
        v.src_w = d.width;
        v.src_h = d.height;
        v.src_off = ii_info.img_offset;
        v.src_pitch = ii_info.img_pitch;
        v.mapx_off = (int64_t)mapx.size();
        v.mapy_off = (int64_t)mapy.size();
        for (int x = 0; x < lw; ++x) {
            int64_t sx = (int64_t)std::floor((double)x * s);
            mapx.push_back((int32_t)std::min<int64_t>(sx, d.width - 1));
        }
        for (int y = 0; y < lh; ++y) {
            int64_t sy = (int64_t)std::floor((double)y * s);
            mapy.push_back((int32_t)std::min<int64_t>(sy, d.height - 1));
        }
        v.bins_pitch = soft ? round_up(2 * (int64_t)lw, 128) : round_up(lw, 64);
        v.bins_off = bins_off;
        bins_off = round_up(bins_off + v.bins_pitch * lh, 256);
        // Planes: ii(x, y) at [y * pitch + x]; rows are whole 128-byte lines
        // (pitch a multiple of 128 / element bytes), so every row store is
        // whole lines; levels start 256-byte aligned.
        v.ii_pitch = round_up(lw, 128 / pb);
        v.ii_plane = v.ii_pitch * lh;
        v.ii_off = round_up(ii_off, 256 / pb);
        ii_off = v.ii_off + v.ii_plane * nb;
        v.score_off = score_off;
        score_off += (int64_t)v.win_x * v.win_y * K;
        v.cell_off = cell_off;
        cell_off += (int64_t)v.cells_x * v.cells_y * nb;
        v.block_off = block_off;
        if (sp.norm == HOG_NORM_L2 && v.cells_x >= 2 && v.cells_y >= 2)
            block_off += (int64_t)(v.cells_x - 1) * (v.cells_y - 1) * 4 * nb;
        // workspace: integral carries (hp, wp = rows, columns rounded up to
        // whole tiles), then the cell cache
        {
            const int64_t hp = (int64_t)hogk::kTile * v.tiles_y, wp = (int64_t)hogk::kTile * v.tiles_x;
            const int64_t tiles = (int64_t)v.tiles_x * v.tiles_y;
            v.ws_rowtot = ws_off;
            ws_off = round_up(ws_off + (int64_t)v.tiles_x * nb * hp, 256);
            v.ws_coltot = ws_off;
            ws_off = round_up(ws_off + (int64_t)v.tiles_y * nb * wp, 256);
            v.ws_tiletot = ws_off;
            ws_off = round_up(ws_off + tiles * nb * 4, 256);
            v.ws_e = ws_off;
            ws_off = round_up(ws_off + (int64_t)v.tiles_x * nb * hp * 2, 256);
            v.ws_cs = ws_off;
            ws_off = round_up(ws_off + (int64_t)v.tiles_y * nb * wp * 2, 256);
            v.ws_p = ws_off;
            ws_off = round_up(ws_off + tiles * nb * 4, 256);
        }
        v.ws_cache = ws_off;
        ws_off = round_up(ws_off + (int64_t)nb * v.cby * v.cbx * 64 * 2, 256);
        v.ws_stot = 0;
        v.ws_scol = 0;
        if (soft) {  // tile vote totals per row and per column, uint32
            const int64_t hp = (int64_t)hogk::kTile * v.tiles_y, wp = (int64_t)hogk::kTile * v.tiles_x;
            v.ws_stot = ws_off;
            ws_off = round_up(ws_off + (int64_t)nb * v.tiles_x * hp * 4, 256);
            v.ws_scol = ws_off;
            ws_off = round_up(ws_off + (int64_t)nb * v.tiles_y * wp * 4, 256);
        }

        info.width = lw;
        info.height = lh;
        info.scale = s;
        info.bins_offset = v.bins_off;
        info.bins_pitch = v.bins_pitch;
        info.ii_offset = v.ii_off;
        info.ii_pitch = v.ii_pitch;
        info.ii_plane_stride = v.ii_plane;
        info.cells_x = v.cells_x;
        info.cells_y = v.cells_y;
        info.windows_x = v.win_x;
        info.windows_y = v.win_y;
        info.score_offset = v.score_off;
        info.cell_offset = v.cell_off;
        info.block_offset = v.block_off;
        p->levels.push_back(v);
        p->info.push_back(info);
        tot_px += (int64_t)lw * lh;
        tot_win += (int64_t)v.win_x * v.win_y;
        s = s * d.scale;
        if (d.max_levels == 1) break;
    }
    ii_info.n_levels = (int32_t)p->levels.size() - ii_info.first_level;
    ii_info.total_pixels = tot_px - img_px0;
    ii_info.total_windows = tot_win - img_win0;
    p->images.push_back(ii_info);
    src_off += (int64_t)d.width * d.height * d.channels;
    }
    const int L = (int)p->levels.size();
    // Prepared template fragments of the matrix-core scorer (rewritten by
    // every hog_scan_windows call).
    int64_t tprep_off = 0, tprep_stride = 0;
    if (scorer == 1) {
        tprep_stride = round_up(hogk::strip_prep_bytes(mfma_ks), 256);
        tprep_off = round_up(ws_off, 256);
        ws_off = tprep_off + tprep_stride * K;
    } else if (scorer == 2) {
        // per tile of 32 templates: fragments [by][bx][step][hi|lo][lane] of
        // 16 bytes, then 32 scales (float), then their exponents (int)
        const int64_t frags = (int64_t)(sp.win_cells_y - 1) * hogk::kStripMaxBX * (mfma_ks / 4) * 2 * 64;
        tprep_stride = round_up(frags * 16 + 32 * 12, 256);  // fragments, scales, exponents, flags
        tprep_off = round_up(ws_off, 256);
        ws_off = tprep_off + tprep_stride * ((K + 31) / 32);
    }
    // The integral kernels address a chunk of planes (and a level's bins)
    // through one buffer descriptor with 31-bit byte offsets.
    {
        int64_t max_plane = 0, max_bins = 0;
        for (const Level &v : p->levels) {
            max_plane = std::max(max_plane, v.ii_plane);
            max_bins = std::max(max_bins, v.bins_pitch * v.h);
        }
        const int64_t lim = ((int64_t)1 << 31) - 1;
        int c = chunk;
        while (c > 1 && (int64_t)c * max_plane * pb > lim) --c;
        if ((int64_t)c * max_plane * pb > lim || max_bins > lim) {
            delete p;
            return fail(HOG_E_INVALID, "image too large: one integral image exceeds 2 GiB");
        }
        chunk_final = c;
    }

    // Per-kernel prefix tables.
    std::vector<int32_t> first((size_t)hogk::KB_COUNT * (L + 1), 0);
    int64_t totals[hogk::KB_COUNT] = {0};
    for (int l = 0; l < L; ++l) {
        const Level &v = p->levels[l];
        int64_t items[hogk::KB_COUNT];
        items[hogk::KB_BINMAP] = (int64_t)v.bm_gx * v.bm_gy;
        items[hogk::KB_ITILE] = (int64_t)v.tiles_x * v.tiles_y;
        // Four rows (columns) per thread, padded to whole waves per bin: waves stay in one (level, bin).
        items[hogk::KB_CSCAN] = (int64_t)16 * round_up(v.tiles_x, 4) * nb;
        items[hogk::KB_ESCAN] = (int64_t)16 * round_up(v.tiles_y, 4) * nb;
        items[hogk::KB_PSCAN] = nb;
        items[hogk::KB_CELL] = (int64_t)v.cells_x * v.cells_y;
        items[hogk::KB_STILE] = (int64_t)v.st_x * v.st_y *
                                (scorer == 1 ? K : scorer == 2 ? (K + 31) / 32 : 1);
        items[hogk::KB_BLOCK] = (sp.norm == HOG_NORM_L2 && v.cells_x >= 2 && v.cells_y >= 2)
                                    ? (int64_t)(v.cells_x - 1) * (v.cells_y - 1)
                                    : 0;
        items[hogk::KB_SSEG] = soft ? (int64_t)v.tiles_x * v.tiles_y : 0;
        items[hogk::KB_SSCAN] = soft ? (int64_t)nb * hogk::kTile * v.tiles_y + (int64_t)nb * hogk::kTile * v.tiles_x : 0;
        items[hogk::KB_SEMIT] = soft ? (int64_t)v.tiles_x * v.tiles_y * ((nb + 1) / 2) : 0;
        for (int k = 0; k < hogk::KB_COUNT; ++k) {
            first[(size_t)k * (L + 1) + l] = (int32_t)totals[k];
            totals[k] += items[k];
        }
    }
    for (int k = 0; k < hogk::KB_COUNT; ++k) {
        if (totals[k] >= ((int64_t)1 << 30)) {
            delete p;
            return fail(HOG_E_INVALID, "image too large for one plan (kernel %d has %lld items)", k,
                        (long long)totals[k]);
        }
        first[(size_t)k * (L + 1) + L] = (int32_t)totals[k];
    }

    // Device tables: levels | first | mapx | mapy.
    const size_t lv_bytes = sizeof(Level) * L;
    const size_t first_bytes = sizeof(int32_t) * first.size();
    const size_t mx_bytes = sizeof(int32_t) * mapx.size();
    const size_t my_bytes = sizeof(int32_t) * mapy.size();
    const size_t o_first = round_up(lv_bytes, 256);
    // The level groups' prefix tables: at most L + HOG_MAX_LEVEL_GROUPS
    // entries per kernel over all groups.
    const size_t gfirst_bytes = sizeof(int32_t) * hogk::KB_COUNT * (L + HOG_MAX_LEVEL_GROUPS);
    const size_t o_gfirst = o_first + round_up(first_bytes, 256);
    const size_t o_mx = o_gfirst + round_up(gfirst_bytes, 256);
    const size_t o_my = o_mx + round_up(mx_bytes, 256);
    const size_t total_bytes = o_my + round_up(my_bytes, 256) + 256;
    std::vector<uint8_t> blob(total_bytes, 0);
    std::memcpy(blob.data(), p->levels.data(), lv_bytes);
    std::memcpy(blob.data() + o_first, first.data(), first_bytes);
    p->first = first;
    p->first_off = o_first;
    p->gfirst_off = o_gfirst;
    std::memcpy(blob.data() + o_mx, mapx.data(), mx_bytes);
    std::memcpy(blob.data() + o_my, mapy.data(), my_bytes);
    hipError_t e = hipMalloc(&p->dev_mem, total_bytes);
    if (e != hipSuccess) {
        delete p;
        return device_fail(e, "hipMalloc(plan tables)");
    }
    e = hipMemcpy(p->dev_mem, blob.data(), total_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->dev_mem);
        delete p;
        return device_fail(e, "hipMemcpy(plan tables)");
    }
    uint8_t *base = (uint8_t *)p->dev_mem;
    PlanDev &pd = p->dev;
    std::memset(&pd, 0, sizeof pd);
    pd.levels = (const Level *)base;
    pd.first = (const int32_t *)(base + o_first);
    pd.mapx = (const int32_t *)(base + o_mx);
    pd.mapy = (const int32_t *)(base + o_my);
    pd.n_levels = L;
    pd.n_bins = nb;
    pd.channels = d0.channels;
    pd.n_templates = K;
    pd.cell = sp.cell;
    pd.win_cells_x = sp.win_cells_x;
    pd.win_cells_y = sp.win_cells_y;
    pd.block = sp.block;
    pd.norm = sp.norm;
    pd.eps = sp.eps;
    pd.votes = d0.votes;
    pd.eps_counts = soft ? sp.eps * HOG_SOFT_QUANTUM : sp.eps;
    pd.vscale = soft ? 1.0f / HOG_SOFT_QUANTUM : 1.0f;
    pd.feat_dim = dim;
    pd.st_tw = best_tw;
    pd.st_th = best_th;
    pd.st_lds_bytes = (int32_t)best_lds;
    pd.mfma_ks = mfma_ks;
    pd.scorer = scorer;
    pd.st_waves = raw_waves;
    pd.cell_stride = nbp;
    pd.plane_bytes = pb;
    pd.bin_chunk = chunk_final;  // bins per wave; a last, smaller chunk takes the rest
    pd.lut_global = 0;           // the LDS half table until tiles say otherwise
    pd.n_chunks = (nb + chunk_final - 1) / chunk_final;
    for (int k = 0; k < hogk::KB_COUNT; ++k) pd.total[k] = totals[k];
    {
        int ncu = 0;
        if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess ||
            ncu < 1)
            ncu = 256;
        pd.n_cu = ncu;
        // The bin map's cache-read forms size their persistent grids from the
        // runtime's occupancy figures: asked here, so that no launch asks
        // first under stream capture.
        (void)hogk::bin_map_blocks_per_cu(false, pd.channels);
        (void)hogk::bin_map_blocks_per_cu(true, pd.channels);
        pd.tprep_off = tprep_off;
        pd.tprep_stride = tprep_stride;
    }

    hog_plan_sizes &z = p->sizes;
    std::memset(&z, 0, sizeof z);
    z.n_levels = L;
    z.bins_bytes = bins_off;
    z.ii_elems = ii_off;
    z.score_elems = score_off;
    z.cell_elems = cell_off;
    z.block_elems = block_off;
    z.workspace_bytes = ws_off;
    z.feature_dim = dim;
    z.total_pixels = tot_px;
    z.total_windows = tot_win;
    z.ii_elem_bytes = pb;
    *out = p;
    return HOG_OK;
}

extern "C" hog_status hog_plan_create(const hog_plan_desc *desc, hog_plan **out)
{
    return create_plan(desc, 1, false, out);
}

extern "C" hog_status hog_plan_create_batch(const hog_plan_desc *descs, int n_images, hog_plan **out)
{
    return create_plan(descs, n_images, true, out);
}

extern "C" int hog_plan_images(const hog_plan *plan) { return plan ? (int)plan->images.size() : 0; }

extern "C" hog_status hog_plan_get_image(const hog_plan *plan, int image, hog_image_info *out)
{
    if (!plan || !out) return fail(HOG_E_INVALID, "plan or out is NULL");
    if (image < 0 || image >= (int)plan->images.size())
        return fail(HOG_E_INVALID, "image %d outside [0, %d)", image, (int)plan->images.size());
    *out = plan->images[image];
    return HOG_OK;
}

static void destroy_group_streams(GroupStreams &g)
{
    for (int i = 0; i < HOG_MAX_LEVEL_GROUPS - 1; ++i) {
        if (g.s[i]) (void)hipStreamDestroy(g.s[i]);
        if (g.join[i]) (void)hipEventDestroy(g.join[i]);
    }
    for (int i = 0; i < HOG_MAX_LEVEL_GROUPS; ++i)
        if (g.mid[i]) (void)hipEventDestroy(g.mid[i]);
    std::memset(&g, 0, sizeof g);
}

// Streams (default priority, non-blocking) and timing-free events for a
// grouped run, created on the current device.
static hipError_t create_group_streams(GroupStreams &g)
{
    std::memset(&g, 0, sizeof g);
    hipError_t e = hipSuccess;
    for (int i = 0; i < HOG_MAX_LEVEL_GROUPS - 1 && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&g.s[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&g.join[i], hipEventDisableTiming);
    }
    for (int i = 0; i < HOG_MAX_LEVEL_GROUPS && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&g.mid[i], hipEventDisableTiming);
    if (e != hipSuccess) destroy_group_streams(g);
    return e;
}

extern "C" void hog_plan_destroy(hog_plan *plan)
{
    if (!plan) return;
    if (plan->have_gs) {
        int cur = 0;
        const bool got = hipGetDevice(&cur) == hipSuccess;
        if (got && cur != plan->device) (void)hipSetDevice(plan->device);
        destroy_group_streams(plan->gs);
        if (got && cur != plan->device) (void)hipSetDevice(cur);
    }
    if (plan->dev_mem) (void)hipFree(plan->dev_mem);
    delete plan;
}

extern "C" hog_status hog_plan_get_sizes(const hog_plan *plan, hog_plan_sizes *out)
{
    if (!plan || !out) return fail(HOG_E_INVALID, "plan or out is NULL");
    *out = plan->sizes;
    return HOG_OK;
}

extern "C" hog_status hog_plan_get_level(const hog_plan *plan, int level, hog_level_info *out)
{
    if (!plan || !out) return fail(HOG_E_INVALID, "plan or out is NULL");
    if (level < 0 || level >= (int)plan->info.size())
        return fail(HOG_E_INVALID, "level %d outside [0, %d)", level, (int)plan->info.size());
    *out = plan->info[level];
    return HOG_OK;
}

// ---------------------------------------------------------------------------
// The hot path.
// ---------------------------------------------------------------------------
// The bin map reads the source image through one buffer descriptor: its
// bytes, (height - 1) * pitch + width * channels, must fit 32 bits. (Packed
// batch images always do: 32767 x 32767 x 3 bytes is below 2^32.)
static bool image_extent_ok(const hog_plan *plan, int64_t img_pitch)
{
    const hog_plan_desc &d = plan->desc;
    return (int64_t)(d.height - 1) * img_pitch + (int64_t)d.width * d.channels <= (int64_t)0xFFFFFFFF;
}

extern "C" hog_status hog_bin_map(const hog_plan *plan, const hog_lut *lut, const uint8_t *img,
                                  int64_t img_pitch, uint8_t *bins, void *stream)
{
    if (!plan || !lut || !img || !bins) return fail(HOG_E_INVALID, "NULL argument");
    if (lut->n_bins != plan->desc.n_bins)
        return fail(HOG_E_INVALID, "lut has %d bins, plan has %d", lut->n_bins, plan->desc.n_bins);
    if (plan->batch) {
        if (img_pitch != 0) return fail(HOG_E_INVALID, "a batch plan takes img_pitch 0 (images are packed)");
    } else if (img_pitch < (int64_t)plan->desc.width * plan->desc.channels) {
        return fail(HOG_E_INVALID, "img_pitch %lld < width*channels", (long long)img_pitch);
    } else if (!image_extent_ok(plan, img_pitch)) {
        return fail(HOG_E_INVALID, "image of img_pitch %lld spans 4 GiB or more", (long long)img_pitch);
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = timed_launch("bin_map", s, [&] {
        return plan->dev.votes == HOG_VOTES_SOFT
                   ? hogk::launch_bin_map_soft(plan->dev, lut->dev_soft, img, img_pitch, bins, s)
                   : hogk::launch_bin_map(plan->dev, lut->dev_half, lut->dev, img, img_pitch, bins, s);
    });
    if (e != hipSuccess) return device_fail(e, "bin_map launch");
    return HOG_OK;
}

// hog_integral's passes. With prep_tmpl (hard votes, the one-template strip
// scorer), the carry scan also prepares that scorer's template weights.
static hog_status integral_impl(const hog_plan *plan, const uint8_t *bins, void *ii, void *workspace,
                                void *stream, const float *prep_tmpl)
{
    hipStream_t s = (hipStream_t)stream;
    uint8_t *ws = (uint8_t *)workspace;
    if (plan->dev.votes == HOG_VOTES_SOFT) {
        // Weighted planes; every cell cached, by the plane writer for 8-pixel
        // cells, else from the planes.
        const bool fused = plan->desc.scan.cell == 8;
        hipError_t e = timed_launch("integral_soft", s, [&] {
            return hogk::launch_soft_integral(plan->dev, bins, ws, (uint32_t *)ii, fused, s);
        });
        if (e != hipSuccess) return device_fail(e, "integral_soft launch");
        if (!fused) {
            e = timed_launch("cells", s, [&] { return hogk::launch_cells(plan->dev, ii, ws, nullptr, s); });
            if (e != hipSuccess) return device_fail(e, "cells launch");
        }
        return HOG_OK;
    }
    hipError_t e = timed_launch("integral_reduce", s, [&] {
        return hogk::launch_int_reduce(plan->dev, bins, ws, s);
    });
    if (e != hipSuccess) return device_fail(e, "integral_reduce launch");
    e = timed_launch("integral_scan", s, [&] {
        return hogk::launch_int_scan(plan->dev, ws, s, prep_tmpl);
    });
    if (e != hipSuccess) return device_fail(e, "integral_scan launch");
    e = timed_launch("integral_emit", s, [&] {
        return hogk::launch_int_emit(plan->dev, bins, ws, ii, s);
    });
    if (e != hipSuccess) return device_fail(e, "integral_emit launch");
    return HOG_OK;
}

extern "C" hog_status hog_integral(const hog_plan *plan, const uint8_t *bins, void *ii,
                                   void *workspace, void *stream)
{
    if (!plan || !bins || !ii || !workspace) return fail(HOG_E_INVALID, "NULL argument");
    return integral_impl(plan, bins, ii, workspace, stream, nullptr);
}

// hog_scan_windows; prep = false when the template weights were prepared on
// this workspace by the carry scan of the same call.
static hog_status scan_windows_impl(const hog_plan *plan, const void *ii, const float *tmpl,
                                    const float *bias, float *scores, uint32_t *cell_hist,
                                    float *block_feat, void *workspace, void *stream, bool prep)
{
    if (!plan || !workspace) return fail(HOG_E_INVALID, "NULL argument");
    const bool need_scores = plan->sizes.score_elems > 0;
    if (need_scores && (!tmpl || !bias || !scores))
        return fail(HOG_E_INVALID, "tmpl, bias and scores are required when the plan has windows");
    if (block_feat && plan->desc.scan.norm != HOG_NORM_L2)
        return fail(HOG_E_INVALID, "block_feat is only defined for HOG_NORM_L2");
    hipStream_t s = (hipStream_t)stream;
    uint8_t *ws = (uint8_t *)workspace;
    hipError_t e = hipSuccess;
    if (ii) {
        // Cell histograms from the given planes (four-corner sums).
        e = timed_launch("cells", s, [&] { return hogk::launch_cells(plan->dev, ii, ws, cell_hist, s); });
        if (e != hipSuccess) return device_fail(e, "cells launch");
    } else if (plan->desc.scan.cell != 8 && plan->dev.votes != HOG_VOTES_SOFT) {
        return fail(HOG_E_INVALID, "hog_integral caches cells only for 8-pixel cells; pass ii");
    } else if (cell_hist) {
        // Cell histograms cached by hog_integral in this workspace.
        e = timed_launch("cells", s, [&] { return hogk::launch_cache_export(plan->dev, ws, cell_hist, s); });
        if (e != hipSuccess) return device_fail(e, "cache export launch");
    }
    if (block_feat) {
        e = timed_launch("block_features", s, [&] {
            return hogk::launch_block_features(plan->dev, ws, block_feat, s);
        });
        if (e != hipSuccess) return device_fail(e, "block_features launch");
    }
    if (need_scores) {
        e = timed_launch("score", s, [&] {
            return hogk::launch_score(plan->dev, ws, tmpl, bias, scores, s, prep);
        });
        if (e != hipSuccess) return device_fail(e, "score launch");
    }
    return HOG_OK;
}

extern "C" hog_status hog_scan_windows(const hog_plan *plan, const void *ii, const float *tmpl,
                                       const float *bias, float *scores, uint32_t *cell_hist,
                                       float *block_feat, void *workspace, void *stream)
{
    return scan_windows_impl(plan, ii, tmpl, bias, scores, cell_hist, block_feat, workspace, stream, true);
}

// ---------------------------------------------------------------------------
// Tile shapes and their autotuner.
// ---------------------------------------------------------------------------

// Bins per integral wave: the cap c split evenly (chunks of ceil(nb / ceil(nb / c))).
static int chunk_for(int nb, int c) { return (nb + (nb + c - 1) / c - 1) / ((nb + c - 1) / c); }

// Level groups: up to G contiguous level ranges of about equal pixel counts
// (one level may make up a range on its own), each a view of the plan's
// tables whose prefix tables start at 0 for its first level. Fewer than two
// ranges leave the plan ungrouped.
static hog_status build_groups(hog_plan *p, int G)
{
    p->groups.clear();
    const int L = p->dev.n_levels;
    if (G < 2 || L < 2) return HOG_OK;
    int64_t tot = 0;
    for (const Level &v : p->levels) tot += (int64_t)v.w * v.h;
    std::vector<int> start(1, 0);
    int64_t acc = 0;
    for (int l = 0; l + 1 < L; ++l) {
        acc += (int64_t)p->levels[l].w * p->levels[l].h;
        const int64_t k = (int64_t)start.size();  // ranges begun so far
        if (k < G && acc * G >= tot * k) start.push_back(l + 1);
    }
    start.push_back(L);
    const int ng = (int)start.size() - 1;
    if (ng < 2) return HOG_OK;
    std::vector<int32_t> gf;
    std::vector<size_t> goff;
    for (int g = 0; g < ng; ++g) {
        goff.push_back(gf.size());
        for (int k = 0; k < hogk::KB_COUNT; ++k) {
            const int32_t *f = p->first.data() + (size_t)k * (L + 1);
            for (int l = start[g]; l <= start[g + 1]; ++l) gf.push_back(f[l] - f[start[g]]);
        }
    }
    // sum over ranges of KB_COUNT * (levels + 1) = KB_COUNT * (L + ng)
    if (gf.size() > (size_t)hogk::KB_COUNT * (L + HOG_MAX_LEVEL_GROUPS))
        return fail(HOG_E_INVALID, "level group tables overflow");
    int32_t *dgf = (int32_t *)((uint8_t *)p->dev_mem + p->gfirst_off);
    hipError_t e = hipMemcpy(dgf, gf.data(), sizeof(int32_t) * gf.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_fail(e, "hipMemcpy(level group tables)");
    for (int g = 0; g < ng; ++g) {
        PlanDev v = p->dev;
        v.levels = p->dev.levels + start[g];
        v.first = dgf + goff[g];
        v.n_levels = start[g + 1] - start[g];
        for (int k = 0; k < hogk::KB_COUNT; ++k) {
            const int32_t *f = p->first.data() + (size_t)k * (L + 1);
            v.total[k] = f[start[g + 1]] - f[start[g]];
        }
        p->groups.push_back(v);
    }
    return HOG_OK;
}

// Installs bins per integral wave, (strip scorer) window rows per strip and
// the level groups, updating the level table and the prefix tables on the
// device.
static hog_status apply_tiles(hog_plan *p, int chunk, int rows, int groups, int lut_global)
{
    if (groups == 0) groups = 1;
    if (lut_global != 0 && lut_global != 1) return fail(HOG_E_INVALID, "lut_global must be 0 or 1");
    if (groups < 1 || groups > HOG_MAX_LEVEL_GROUPS)
        return fail(HOG_E_INVALID, "level_groups must be in [0, %d]", HOG_MAX_LEVEL_GROUPS);
    PlanDev &pd = p->dev;
    const int L = pd.n_levels, K = pd.n_templates;
    int64_t max_plane = 0;
    for (const Level &v : p->levels) max_plane = std::max(max_plane, v.ii_plane);
    if (chunk < 1 || chunk > hogk::kMaxBinChunk || (int64_t)chunk * max_plane * p->dev.plane_bytes > ((int64_t)1 << 31) - 1)
        return fail(HOG_E_INVALID, "bins per integral wave must be in [1, %d] and fit 2 GiB", hogk::kMaxBinChunk);
    pd.bin_chunk = chunk;
    pd.n_chunks = (pd.n_bins + chunk - 1) / chunk;
    pd.lut_global = lut_global;
    if (pd.scorer == 1 && rows != pd.st_th) {
        if (rows < 1 || rows > 64) return fail(HOG_E_INVALID, "window rows per strip must be in [1, 64]");
        pd.st_th = rows;
        const int64_t rowh = (int64_t)(hogk::kStripW + 8) * pd.mfma_ks;
        pd.st_lds_bytes = (int32_t)(4 * round_up(4 * rowh * 2 + 64 * 4 + (int64_t)hogk::kStripW * rows * 4, 16));
        int64_t tot = 0;
        int32_t *f = p->first.data() + (size_t)hogk::KB_STILE * (L + 1);
        for (int l = 0; l < L; ++l) {
            Level &v = p->levels[l];
            v.st_y = v.win_y ? (v.win_y + rows - 1) / rows : 0;
            f[l] = (int32_t)tot;
            tot += (int64_t)v.st_x * v.st_y * K;
        }
        f[L] = (int32_t)tot;
        pd.total[hogk::KB_STILE] = tot;
        hipError_t e = hipMemcpy(p->dev_mem, p->levels.data(), sizeof(Level) * L, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy((uint8_t *)p->dev_mem + p->first_off, p->first.data(), sizeof(int32_t) * p->first.size(),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) return device_fail(e, "hipMemcpy(plan tables)");
    }
    return build_groups(p, groups);
}

static int level_groups_of(const hog_plan *p) { return p->groups.empty() ? 1 : (int)p->groups.size(); }

extern "C" hog_status hog_plan_get_tiles(const hog_plan *plan, hog_tiles *out)
{
    if (!plan || !out) return fail(HOG_E_INVALID, "plan or out is NULL");
    out->bin_chunk = plan->dev.bin_chunk;
    out->score_rows = plan->dev.scorer == 1 ? plan->dev.st_th : 0;
    out->level_groups = level_groups_of(plan);
    out->lut_global = plan->dev.lut_global;
    return HOG_OK;
}

extern "C" hog_status hog_plan_set_tiles(hog_plan *plan, const hog_tiles *tiles)
{
    if (!plan || !tiles) return fail(HOG_E_INVALID, "plan or tiles is NULL");
    return apply_tiles(plan, tiles->bin_chunk, plan->dev.scorer == 1 ? tiles->score_rows : plan->dev.st_th,
                       tiles->level_groups, tiles->lut_global);
}

static hog_status check_run_args(const hog_plan *plan, const hog_lut *lut, const uint8_t *img,
                                 int64_t img_pitch, uint8_t *bins, void *ii, const float *tmpl,
                                 const float *bias, float *scores, void *workspace);
static hog_status run_plan(const hog_plan *plan, const hog_lut *lut, const uint8_t *img, int64_t img_pitch,
                           uint8_t *bins, void *ii, const float *tmpl, const float *bias, float *scores,
                           void *workspace, void *stream);

// Autotune cache: earlier hog_plan_autotune results, keyed by device,
// library build and plan shape, kept in memory and appended to a text file
// ("hogtune <key> <bin_chunk> <score_rows> <level_groups> <lut_global>").
namespace {
std::mutex g_tune_mu;
std::string g_tune_path;
std::map<uint64_t, std::array<int32_t, 4>> g_tune;
int64_t g_tune_hits = 0, g_tune_misses = 0;

uint64_t fnv1a(uint64_t h, const void *p, size_t n)
{
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

// The device (architecture, compute units), this build of the library, and
// what the tiles' timing depends on in the plan: every level's size and the
// shared parameters.
uint64_t tune_key(const hog_plan *p)
{
    uint64_t h = 1469598103934665603ull;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
        h = fnv1a(h, prop.gcnArchName, strnlen(prop.gcnArchName, sizeof prop.gcnArchName));
        h = fnv1a(h, &prop.multiProcessorCount, sizeof prop.multiProcessorCount);
    }
    static const char build[] = __DATE__ " " __TIME__;
    h = fnv1a(h, build, sizeof build);
    const hog_plan_desc &d = p->desc;
    const int32_t f[] = {d.channels, d.n_bins, d.n_templates, d.scan.cell, d.scan.win_cells_x,
                         d.scan.win_cells_y, d.scan.block, d.scan.norm, d.plane_bits, d.votes,
                         (int32_t)p->batch, (int32_t)p->levels.size()};
    h = fnv1a(h, f, sizeof f);
    uint32_t eps_bits;
    std::memcpy(&eps_bits, &d.scan.eps, sizeof eps_bits);
    h = fnv1a(h, &eps_bits, sizeof eps_bits);
    for (const Level &v : p->levels) {
        h = fnv1a(h, &v.w, sizeof v.w);
        h = fnv1a(h, &v.h, sizeof v.h);
    }
    return h;
}
}  // namespace

extern "C" hog_status hog_tune_cache_open(const char *path)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_hits = g_tune_misses = 0;
    g_tune_path = path ? path : "";
    if (!path) return HOG_OK;
    if (!*path) return fail(HOG_E_INVALID, "empty cache path");
    FILE *fp = std::fopen(path, "r");
    if (!fp) return HOG_OK;  // created at the first result
    char line[256];
    while (std::fgets(line, sizeof line, fp)) {
        unsigned long long key = 0;
        int t[4];
        char tail = 0;
        if (std::sscanf(line, "hogtune %llx %d %d %d %d %c", &key, &t[0], &t[1], &t[2], &t[3], &tail) == 5)
            g_tune[(uint64_t)key] = {t[0], t[1], t[2], t[3]};
    }
    std::fclose(fp);
    return HOG_OK;
}

extern "C" hog_status hog_tune_cache_stats(int64_t *hits, int64_t *misses, int64_t *entries)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (hits) *hits = g_tune_hits;
    if (misses) *misses = g_tune_misses;
    if (entries) *entries = (int64_t)g_tune.size();
    return HOG_OK;
}

extern "C" hog_status hog_plan_autotune(hog_plan *plan, const hog_lut *lut, const uint8_t *img,
                                        int64_t img_pitch, uint8_t *bins, void *ii, const float *tmpl,
                                        const float *bias, float *scores, void *workspace, void *stream,
                                        int reps, hog_tiles *chosen)
{
    hog_status st = check_run_args(plan, lut, img, img_pitch, bins, ii, tmpl, bias, scores, workspace);
    if (st != HOG_OK) return st;
    if (reps < 1 || reps > 1000) return fail(HOG_E_INVALID, "reps must be in [1, 1000]");
    hipStream_t s = (hipStream_t)stream;
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        cached = !g_tune_path.empty();
    }
    uint64_t key = 0;
    if (cached) {
        key = tune_key(plan);
        std::array<int32_t, 4> t{};
        bool found = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(key);
            if (it != g_tune.end()) {
                found = true;
                t = it->second;
            }
        }
        // A stored result is installed as it is (one hog_run leaves the
        // buffers as the tuned call would); one the plan rejects is re-tuned.
        if (found && apply_tiles(plan, t[0], t[1], t[2], t[3]) == HOG_OK) {
            st = run_plan(plan, lut, img, img_pitch, bins, ii, tmpl, bias, scores, workspace, stream);
            if (st != HOG_OK) return st;
            hipError_t he = hipStreamSynchronize(s);
            if (he != hipSuccess) return device_fail(he, "hipStreamSynchronize");
            {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                ++g_tune_hits;
            }
            return chosen ? hog_plan_get_tiles(plan, chosen) : HOG_OK;
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return device_fail(e, "hipEventCreate");
    }
    // Per-run time of reps whole runs back to back (the way a caller runs
    // the path step after step), the best of three such rounds, after one
    // untimed run, with these tiles: the best round is steadier than one
    // long average, and back-to-back runs rank level groups, which overlap
    // work across streams, as a stream of steps sees them.
    int best_lut = plan->dev.lut_global;
    auto time_with = [&](int chunk, int rows, int groups, float *ms) -> hog_status {
        hog_status r = apply_tiles(plan, chunk, rows, groups, best_lut);
        if (r != HOG_OK) return r;
        r = run_plan(plan, lut, img, img_pitch, bins, ii, tmpl, bias, scores, workspace, stream);
        if (r != HOG_OK) return r;
        float best_ms = 1e30f;
        for (int round = 0; round < 3; ++round) {
            hipError_t he = hipEventRecord(e0, s);
            for (int i = 0; i < reps && r == HOG_OK; ++i)
                r = run_plan(plan, lut, img, img_pitch, bins, ii, tmpl, bias, scores, workspace, stream);
            if (r != HOG_OK) return r;
            float total = 0.f;
            if (he == hipSuccess) he = hipEventRecord(e1, s);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            if (he == hipSuccess) he = hipEventElapsedTime(&total, e0, e1);
            if (he != hipSuccess) return device_fail(he, "autotune timing");
            best_ms = std::min(best_ms, total / (float)reps);
        }
        *ms = best_ms;
        return HOG_OK;
    };
    const int nb = plan->dev.n_bins;
    int best_chunk = plan->dev.bin_chunk, best_rows = plan->dev.st_th, best_groups = 1;
    float best = 1e30f;
    // Bins per integral wave, then window rows per strip (strip scorer), both
    // with the levels in one group; then the number of level groups.
    int64_t max_plane = 0;
    for (const Level &v : plan->levels) max_plane = std::max(max_plane, v.ii_plane);
    for (int c = 2; c <= hogk::kMaxBinChunk && st == HOG_OK; ++c) {
        const int chunk = chunk_for(nb, c);
        if (chunk != c || (int64_t)chunk * max_plane * plan->dev.plane_bytes > ((int64_t)1 << 31) - 1) continue;
        float ms = 0.f;
        st = time_with(chunk, best_rows, 1, &ms);
        if (st == HOG_OK && ms < best) {
            best = ms;
            best_chunk = chunk;
        }
    }
    if (st == HOG_OK && plan->dev.scorer == 1) {
        // Small heights suit small images (more, shorter waves); 20 puts the
        // 1920 x 1080 pyramid's strips at one wave per SIMD (991 strips).
        const int cand[] = {4, 6, 8, 12, 16, 20, 24, 32};
        for (int rows : cand) {
            float ms = 0.f;
            st = time_with(best_chunk, rows, 1, &ms);
            if (st != HOG_OK) break;
            if (ms < best) {
                best = ms;
                best_rows = rows;
            }
        }
    }
    if (st == HOG_OK && plan->dev.votes == HOG_VOTES_HARD) {
        const int cur = best_lut;
        best_lut = 1 - cur;
        float ms = 0.f;
        st = time_with(best_chunk, best_rows, 1, &ms);
        if (st == HOG_OK && ms < best)
            best = ms;
        else
            best_lut = cur;
    }
    for (int g = 2; g <= HOG_MAX_LEVEL_GROUPS && st == HOG_OK && g <= plan->dev.n_levels; ++g) {
        float ms = 0.f;
        st = time_with(best_chunk, best_rows, g, &ms);
        if (st == HOG_OK && ms < best) {
            best = ms;
            best_groups = g;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != HOG_OK) return st;
    st = apply_tiles(plan, best_chunk, best_rows, best_groups, best_lut);
    if (st == HOG_OK && cached) {
        const std::array<int32_t, 4> t = {plan->dev.bin_chunk, plan->dev.st_th, best_groups, best_lut};
        std::lock_guard<std::mutex> lk(g_tune_mu);
        ++g_tune_misses;
        if (!g_tune_path.empty()) {
            g_tune[key] = t;
            // A file that cannot be written keeps the result in memory only.
            if (FILE *fp = std::fopen(g_tune_path.c_str(), "a")) {
                std::fprintf(fp, "hogtune %016llx %d %d %d %d\n", (unsigned long long)key, t[0], t[1], t[2], t[3]);
                std::fclose(fp);
            }
        }
    }
    if (st == HOG_OK && chosen) st = hog_plan_get_tiles(plan, chosen);
    return st;
}

// ---------------------------------------------------------------------------
// The whole path in one call, and captured into a HIP graph.
// ---------------------------------------------------------------------------
static hog_status check_run_args(const hog_plan *plan, const hog_lut *lut, const uint8_t *img,
                                 int64_t img_pitch, uint8_t *bins, void *ii, const float *tmpl,
                                 const float *bias, float *scores, void *workspace)
{
    if (!plan || !lut || !img || !bins || !ii || !workspace) return fail(HOG_E_INVALID, "NULL argument");
    if (plan->sizes.score_elems > 0 && (!tmpl || !bias || !scores))
        return fail(HOG_E_INVALID, "tmpl, bias and scores are required when the plan has windows");
    if (lut->n_bins != plan->desc.n_bins)
        return fail(HOG_E_INVALID, "lut has %d bins, plan has %d", lut->n_bins, plan->desc.n_bins);
    if (plan->batch ? img_pitch != 0 : img_pitch < (int64_t)plan->desc.width * plan->desc.channels)
        return fail(HOG_E_INVALID, "bad img_pitch %lld", (long long)img_pitch);
    if (!plan->batch && !image_extent_ok(plan, img_pitch))
        return fail(HOG_E_INVALID, "image of img_pitch %lld spans 4 GiB or more", (long long)img_pitch);
    return HOG_OK;
}

static hog_status run_path(const hog_plan *plan, const hog_lut *lut, const uint8_t *img, int64_t img_pitch,
                           uint8_t *bins, void *ii, const float *tmpl, const float *bias, float *scores,
                           void *workspace, void *stream)
{
    hog_status st = hog_bin_map(plan, lut, img, img_pitch, bins, stream);
    if (st != HOG_OK) return st;
    // The one-template strip scorer's template prep runs inside the carry
    // scan's launch instead of as a launch of its own before the scores.
    const bool soft = plan->dev.votes == HOG_VOTES_SOFT;
    const bool fuse_prep = !soft && plan->sizes.score_elems > 0 && hogk::scan_runs_prep(plan->dev);
    st = integral_impl(plan, bins, ii, workspace, stream, fuse_prep ? tmpl : nullptr);
    if (st != HOG_OK) return st;
    // The integral caches 8-pixel cells (every cell size with soft votes).
    const bool from_planes = plan->desc.scan.cell != 8 && !soft;
    return scan_windows_impl(plan, from_planes ? ii : nullptr, tmpl, bias, scores, nullptr, nullptr,
                             workspace, stream, !fuse_prep);
}

// The path with level groups. The matrix-core scorer's template weights are
// prepared once, on the caller's stream. Group 0 then runs on that stream and
// group g > 0 on gs.s[g - 1], which waits until group g - 1 has its carries
// and starts writing planes: one group's bin map, reduce and scan run while
// the previous group's plane writer holds HBM. Every group's end is joined
// back into the caller's stream, so the call is ordered on it like run_path.
static hog_status run_groups(const hog_plan *plan, const GroupStreams &gs, const hog_lut *lut,
                             const uint8_t *img, int64_t img_pitch, uint8_t *bins, void *ii,
                             const float *tmpl, const float *bias, float *scores, void *workspace,
                             void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    uint8_t *ws = (uint8_t *)workspace;
    const bool soft = plan->dev.votes == HOG_VOTES_SOFT;
    const bool need_scores = plan->sizes.score_elems > 0;
    const bool from_planes = plan->desc.scan.cell != 8 && !soft;
    const char *what = "score_prep launch";
    hipError_t e = hipSuccess;
    if (need_scores)
        e = timed_launch("score_prep", s, [&] { return hogk::launch_score_prep(plan->dev, ws, tmpl, s); });
    const int ng = (int)plan->groups.size();
    int forked = 0;  // groups g > 0 whose stream has joined this call's work
    for (int g = 0; g < ng && e == hipSuccess; ++g) {
        const PlanDev &v = plan->groups[g];
        hipStream_t sg = g == 0 ? s : gs.s[g - 1];
        if (g > 0) {
            what = "hipStreamWaitEvent";
            e = hipStreamWaitEvent(sg, gs.mid[g - 1], 0);
            if (e != hipSuccess) break;
            forked = g;
        }
        what = "bin_map launch";
        e = timed_launch("bin_map", sg, [&] {
            return soft ? hogk::launch_bin_map_soft(v, lut->dev_soft, img, img_pitch, bins, sg)
                        : hogk::launch_bin_map(v, lut->dev_half, lut->dev, img, img_pitch, bins, sg);
        });
        if (e != hipSuccess) break;
        if (soft) {
            what = "hipEventRecord";
            e = hipEventRecord(gs.mid[g], sg);
            if (e != hipSuccess) break;
            what = "integral_soft launch";
            const bool fused = plan->desc.scan.cell == 8;
            e = timed_launch("integral_soft", sg, [&] {
                return hogk::launch_soft_integral(v, bins, ws, (uint32_t *)ii, fused, sg);
            });
            if (e != hipSuccess) break;
            if (!fused) {
                what = "cells launch";
                e = timed_launch("cells", sg, [&] { return hogk::launch_cells(v, ii, ws, nullptr, sg); });
            }
        } else {
            what = "integral_reduce launch";
            e = timed_launch("integral_reduce", sg, [&] { return hogk::launch_int_reduce(v, bins, ws, sg); });
            if (e != hipSuccess) break;
            what = "integral_scan launch";
            e = timed_launch("integral_scan", sg, [&] { return hogk::launch_int_scan(v, ws, sg); });
            if (e != hipSuccess) break;
            what = "hipEventRecord";
            e = hipEventRecord(gs.mid[g], sg);
            if (e != hipSuccess) break;
            what = "integral_emit launch";
            e = timed_launch("integral_emit", sg, [&] { return hogk::launch_int_emit(v, bins, ws, ii, sg); });
            if (e == hipSuccess && from_planes) {
                what = "cells launch";
                e = timed_launch("cells", sg, [&] { return hogk::launch_cells(v, ii, ws, nullptr, sg); });
            }
        }
        if (e != hipSuccess) break;
        if (need_scores) {
            what = "score launch";
            e = timed_launch("score", sg, [&] { return hogk::launch_score(v, ws, tmpl, bias, scores, sg, false); });
        }
    }
    // Join every forked stream back, also after a failure.
    for (int g = 1; g <= forked; ++g) {
        hipError_t je = hipEventRecord(gs.join[g - 1], gs.s[g - 1]);
        if (je == hipSuccess) je = hipStreamWaitEvent(s, gs.join[g - 1], 0);
        if (je != hipSuccess && e == hipSuccess) {
            e = je;
            what = "joining level-group streams";
        }
    }
    return e == hipSuccess ? HOG_OK : device_fail(e, what);
}

// run_path, or run_groups on the plan's own streams (created on first use,
// on the plan's device) under the plan's lock.
static hog_status run_plan(const hog_plan *plan, const hog_lut *lut, const uint8_t *img, int64_t img_pitch,
                           uint8_t *bins, void *ii, const float *tmpl, const float *bias, float *scores,
                           void *workspace, void *stream)
{
    if (plan->groups.empty())
        return run_path(plan, lut, img, img_pitch, bins, ii, tmpl, bias, scores, workspace, stream);
    hog_plan *mp = const_cast<hog_plan *>(plan);
    std::lock_guard<std::mutex> lock(mp->gs_mu);
    if (!mp->have_gs) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != mp->device) e = hipSetDevice(mp->device);
        if (e == hipSuccess) e = create_group_streams(mp->gs);
        if (cur != mp->device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return device_fail(e, "creating level-group streams");
        mp->have_gs = true;
    }
    return run_groups(plan, mp->gs, lut, img, img_pitch, bins, ii, tmpl, bias, scores, workspace, stream);
}

extern "C" hog_status hog_run(const hog_plan *plan, const hog_lut *lut, const uint8_t *img, int64_t img_pitch,
                              uint8_t *bins, void *ii, const float *tmpl, const float *bias,
                              float *scores, void *workspace, void *stream)
{
    hog_status st = check_run_args(plan, lut, img, img_pitch, bins, ii, tmpl, bias, scores, workspace);
    if (st != HOG_OK) return st;
    return run_plan(plan, lut, img, img_pitch, bins, ii, tmpl, bias, scores, workspace, stream);
}

// The workspace of hog_run_static: one static device array per GPU (each
// device that loads the library holds its own copy). Host code never uses
// the symbol itself, only the address hipGetSymbolAddress gives for the
// current device, looked up once per device and kept.
static __device__ __align__(256) uint8_t scratch[HOG_STATIC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_ptr;

static hog_status static_scratch(int device, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return HOG_OK;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return device_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                    "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = ptr;
    *out = ptr;
    return HOG_OK;
}

extern "C" hog_status hog_run_static(const hog_plan *plan, const hog_lut *lut, const uint8_t *img,
                                     int64_t img_pitch, uint8_t *bins, void *ii, const float *tmpl,
                                     const float *bias, float *scores, void *stream)
{
    uint8_t placeholder = 0;  // the workspace is checked below, not passed in
    hog_status st = check_run_args(plan, lut, img, img_pitch, bins, ii, tmpl, bias, scores, &placeholder);
    if (st != HOG_OK) return st;
    if (plan->sizes.workspace_bytes > HOG_STATIC_SCRATCH_BYTES)
        return fail(HOG_E_INVALID, "the plan needs %lld workspace bytes; the static scratch holds %lld",
                    (long long)plan->sizes.workspace_bytes, (long long)HOG_STATIC_SCRATCH_BYTES);
    int cur = 0;
    const hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    if (cur != plan->device)
        return fail(HOG_E_INVALID, "the plan is on device %d, the current device is %d", plan->device, cur);
    void *ws = nullptr;
    st = static_scratch(cur, &ws);
    if (st != HOG_OK) return st;
    g_no_alloc = true;
    st = run_path(plan, lut, img, img_pitch, bins, ii, tmpl, bias, scores, ws, stream);
    g_no_alloc = false;
    return st;
}

struct hog_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" hog_status hog_graph_create(const hog_plan *plan, const hog_lut *lut, const uint8_t *img,
                                       int64_t img_pitch, uint8_t *bins, void *ii, const float *tmpl,
                                       const float *bias, float *scores, void *workspace, hog_graph **out)
{
    if (!out) return fail(HOG_E_INVALID, "out is NULL");
    *out = nullptr;
    hog_status st = check_run_args(plan, lut, img, img_pitch, bins, ii, tmpl, bias, scores, workspace);
    if (st != HOG_OK) return st;
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return device_fail(e, "hipStreamCreate (capture)");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return device_fail(e, "hipStreamBeginCapture");
    }
    // Level groups are captured on streams of this capture's own: their fork
    // and join events become the graph's edges.
    GroupStreams gs;
    std::memset(&gs, 0, sizeof gs);
    if (!plan->groups.empty()) {
        e = create_group_streams(gs);
        if (e != hipSuccess) {
            hipGraph_t dead = nullptr;
            (void)hipStreamEndCapture(cs, &dead);
            if (dead) (void)hipGraphDestroy(dead);
            (void)hipStreamDestroy(cs);
            return device_fail(e, "creating level-group streams");
        }
    }
    g_capturing = true;
    st = plan->groups.empty()
             ? run_path(plan, lut, img, img_pitch, bins, ii, tmpl, bias, scores, workspace, cs)
             : run_groups(plan, gs, lut, img, img_pitch, bins, ii, tmpl, bias, scores, workspace, cs);
    g_capturing = false;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (!plan->groups.empty()) destroy_group_streams(gs);
    (void)hipStreamDestroy(cs);
    if (st != HOG_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return st != HOG_OK ? st : device_fail(e, "hipStreamEndCapture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return device_fail(e, "hipGraphInstantiate");
    }
    hog_graph *g = new (std::nothrow) hog_graph;
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return fail(HOG_E_NOMEM, "host allocation failed");
    }
    g->graph = graph;
    g->exec = exec;
    *out = g;
    return HOG_OK;
}

extern "C" hog_status hog_graph_launch(hog_graph *g, void *stream)
{
    if (!g) return fail(HOG_E_INVALID, "graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return device_fail(e, "hipGraphLaunch");
    return HOG_OK;
}

extern "C" void hog_graph_destroy(hog_graph *g)
{
    if (!g) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
}

// ---------------------------------------------------------------------------
extern "C" hog_status hog_timing_enable(int on)
{
    g_timing_on = on != 0;
    return HOG_OK;
}

extern "C" hog_status hog_timing_reset(void)
{
    hipError_t e = drain_timing();
    g_timing_totals.clear();
    if (e != hipSuccess) return device_fail(e, "timing events");
    return HOG_OK;
}

extern "C" hog_status hog_timing_get(const char *kernel, int64_t *launches, double *total_ms)
{
    if (!kernel || !launches || !total_ms) return fail(HOG_E_INVALID, "NULL argument");
    hipError_t e = drain_timing();
    if (e != hipSuccess) return device_fail(e, "timing events");
    auto it = g_timing_totals.find(kernel);
    if (it == g_timing_totals.end()) {
        *launches = 0;
        *total_ms = 0.0;
    } else {
        *launches = it->second.first;
        *total_ms = it->second.second;
    }
    return HOG_OK;
}

}  // extern "C"
