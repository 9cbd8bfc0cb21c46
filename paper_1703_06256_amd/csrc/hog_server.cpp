// Request serving with continuous batching (hog_server_*, hog_submit,
// hog_poll): the scan of Sec. 4 applied to a stream of images.
//
// hog_submit copies a host image into the server and returns a ticket. A
// worker thread admits pending requests, oldest first, into a batch while
// in-flight slots and device memory allow; admission is by the device
// footprint of the batch's buffers (bins, integral images, workspace,
// scores), carved from one arena allocated at creation. The batch is packed
// into pinned host memory, copied in, run through hog_run on a batch plan
// (one launch per kernel for all its images), and its scores copied back,
// all on one of several non-blocking streams; requests that arrive while
// batches are on the device form the next batch on another stream, so their
// work overlaps. Batch plans are cached by composition; the lookup table and
// the templates stay resident. hog_poll returns a finished request's scores
// and its latency (submit to ready, host clock).
#include "hog.h"
#include "hog_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <utility>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

hog_status srv_fail(hog_status st, const char *fmt, ...)
{
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    hogk::set_last_error(msg);
    return st;
}

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

struct Request {
    uint64_t ticket = 0;
    int w = 0, h = 0;
    std::vector<uint8_t> img;  // host copy, rows of w * channels bytes
    int64_t footprint = 0;     // device bytes of the image alone
    Clock::time_point t_submit;
    bool ready = false;
    hog_status status = HOG_OK;
    std::vector<float> scores;
    int nwx = 0, nwy = 0;
    double latency = 0.0;
};
using ReqPtr = std::shared_ptr<Request>;

// First-fit allocator over [0, size) of the device arena.
class Arena {
  public:
    void reset(int64_t size)
    {
        free_.clear();
        if (size > 0) free_[0] = size;
    }
    bool alloc(int64_t bytes, int64_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const int64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest > 0) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(int64_t off, int64_t bytes)
    {
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<int64_t, int64_t> free_;  // offset -> bytes
};

struct Layout {  // a batch plan's buffers inside one arena region
    int64_t bins, ii, scores, ws, img, total;
};

Layout layout_of(const hog_plan_sizes &z, int64_t img_bytes)
{
    Layout L;
    int64_t o = 0;
    L.bins = o;
    o = align256(o + z.bins_bytes);
    L.ii = o;
    o = align256(o + z.ii_elems * 4);
    L.scores = o;
    o = align256(o + std::max<int64_t>(z.score_elems, 1) * 4);
    L.ws = o;
    o = align256(o + z.workspace_bytes);
    L.img = o;
    o = align256(o + img_bytes);
    L.total = o;
    return L;
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint8_t *pin_in = nullptr;  // packed images (pinned)
    size_t in_cap = 0;
    float *pin_out = nullptr;  // scores (pinned)
    size_t out_cap = 0;
    bool busy = false;
    std::vector<ReqPtr> reqs;
    hog_plan *plan = nullptr;
    int64_t off = 0, bytes = 0;
};

}  // namespace

struct hog_server {
    hog_server_config cfg;
    int device = 0;
    hog_lut *lut = nullptr;
    float *d_tmpl = nullptr, *d_bias = nullptr;
    uint8_t *arena_base = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    std::map<std::vector<std::pair<int, int>>, hog_plan *> plans;  // by batch composition
    std::mutex mu;                                                 // guards the fields below
    std::condition_variable cv;
    std::deque<ReqPtr> pending;
    std::map<uint64_t, ReqPtr> live;  // submitted and not yet returned by hog_poll
    int in_flight = 0;                // requests on the device
    uint64_t next_ticket = 1;
    bool stop = false;
    std::mutex plan_mu;  // guards plans
    std::thread worker;
};

namespace {

hog_plan_desc desc_for(const hog_server_config &c, int w, int h)
{
    hog_plan_desc d;
    std::memset(&d, 0, sizeof d);
    d.width = w;
    d.height = h;
    d.channels = c.channels;
    d.n_bins = c.n_bins;
    d.max_levels = c.max_levels;
    d.scale = c.scale;
    d.n_templates = c.n_templates;
    d.scan = c.scan;
    return d;
}

// Cached batch plan for the given sizes (in order); nullptr on failure.
hog_plan *plan_for(hog_server *s, const std::vector<std::pair<int, int>> &key)
{
    std::lock_guard<std::mutex> lk(s->plan_mu);
    (void)hipSetDevice(s->device);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) return it->second;
    std::vector<hog_plan_desc> descs;
    for (auto &wh : key) descs.push_back(desc_for(s->cfg, wh.first, wh.second));
    hog_plan *p = nullptr;
    if (hog_plan_create_batch(descs.data(), (int)descs.size(), &p) != HOG_OK) return nullptr;
    s->plans[key] = p;
    return p;
}

int64_t batch_bytes(hog_plan *p, int64_t img_bytes)
{
    hog_plan_sizes z;
    hog_plan_get_sizes(p, &z);
    return layout_of(z, img_bytes).total;
}

// Finished batch in slot i: scores to the requests, memory back to the arena.
void finish(hog_server *s, Slot &sl, hipError_t err)
{
    hog_plan_sizes z;
    hog_plan_get_sizes(sl.plan, &z);
    const int K = s->cfg.n_templates;
    const auto now = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        Request &r = *sl.reqs[i];
        if (err != hipSuccess) {
            r.status = HOG_E_DEVICE;
        } else {
            hog_image_info im;
            hog_plan_get_image(sl.plan, (int)i, &im);
            hog_level_info first, last;
            hog_plan_get_level(sl.plan, im.first_level, &first);
            hog_plan_get_level(sl.plan, im.first_level + im.n_levels - 1, &last);
            const int64_t a = first.score_offset;
            const int64_t b = last.score_offset + (int64_t)last.windows_x * last.windows_y * K;
            r.scores.assign(sl.pin_out + a, sl.pin_out + b);
            r.nwx = first.windows_x;
            r.nwy = first.windows_y;
        }
        r.latency = std::chrono::duration<double>(now - r.t_submit).count();
        r.ready = true;
    }
    s->arena.release(sl.off, sl.bytes);
    s->in_flight -= (int)sl.reqs.size();
    sl.reqs.clear();
    sl.busy = false;
    s->cv.notify_all();
}

// Launches one batch into a free slot if requests and memory allow.
bool admit(hog_server *s, Slot &sl)
{
    std::vector<ReqPtr> take;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const int room = std::min(s->cfg.max_batch, s->cfg.max_slots - s->in_flight);
        for (auto it = s->pending.begin(); it != s->pending.end() && (int)take.size() < room; ++it)
            take.push_back(*it);
    }
    if (take.empty()) return false;
    // Largest batch (oldest first) whose buffers fit the arena now.
    while (!take.empty()) {
        std::vector<ReqPtr> order(take);
        std::stable_sort(order.begin(), order.end(), [](const ReqPtr &a, const ReqPtr &b) {
            return std::make_pair(a->w, a->h) < std::make_pair(b->w, b->h);
        });
        std::vector<std::pair<int, int>> key;
        int64_t img_bytes = 0;
        for (auto &r : order) {
            key.emplace_back(r->w, r->h);
            img_bytes += (int64_t)r->img.size();
        }
        hog_plan *p = plan_for(s, key);
        if (!p) {  // cannot plan this batch: fail its oldest request
            std::lock_guard<std::mutex> lk(s->mu);
            ReqPtr r = take.front();
            r->status = HOG_E_INVALID;
            r->ready = true;
            s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
            return true;
        }
        const int64_t bytes = batch_bytes(p, img_bytes);
        hog_plan_sizes z;
        hog_plan_get_sizes(p, &z);
        int64_t off = 0;
        bool ok;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            ok = (size_t)img_bytes <= sl.in_cap && (size_t)z.score_elems <= sl.out_cap &&
                 s->arena.alloc(bytes, &off);
            if (ok) {
                for (auto &r : take) s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
                s->in_flight += (int)take.size();
            }
        }
        if (!ok) {
            take.pop_back();
            continue;
        }
        // Pack, copy in, run, copy the scores out.
        const Layout L = layout_of(z, img_bytes);
        for (int i = 0; i < (int)order.size(); ++i) {
            hog_image_info im;
            hog_plan_get_image(p, i, &im);
            std::memcpy(sl.pin_in + im.img_offset, order[i]->img.data(), order[i]->img.size());
        }
        uint8_t *base = s->arena_base + off;
        hipError_t e = hipMemcpyAsync(base + L.img, sl.pin_in, (size_t)img_bytes, hipMemcpyHostToDevice, sl.stream);
        hog_status st = HOG_OK;
        if (e == hipSuccess)
            st = hog_run(p, s->lut, base + L.img, 0, base + L.bins, (uint32_t *)(base + L.ii), s->d_tmpl,
                         s->d_bias, (float *)(base + L.scores), base + L.ws, sl.stream);
        if (e == hipSuccess && st == HOG_OK && z.score_elems > 0)
            e = hipMemcpyAsync(sl.pin_out, base + L.scores, (size_t)z.score_elems * 4, hipMemcpyDeviceToHost,
                               sl.stream);
        if (e == hipSuccess && st == HOG_OK) e = hipEventRecord(sl.done, sl.stream);
        sl.reqs = order;
        sl.plan = p;
        sl.off = off;
        sl.bytes = bytes;
        sl.busy = true;
        if (e != hipSuccess || st != HOG_OK) finish(s, sl, e != hipSuccess ? e : hipErrorLaunchFailure);
        return true;
    }
    return false;
}

void worker_main(hog_server *s)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        bool progress = false;
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            finish(s, sl, q);
            progress = true;
        }
        for (Slot &sl : s->slots)
            if (!sl.busy && admit(s, sl)) progress = true;
        std::unique_lock<std::mutex> lk(s->mu);
        bool any_busy = false;
        for (Slot &sl : s->slots) any_busy = any_busy || sl.busy;
        if (s->stop && !any_busy) break;
        if (!progress) {
            if (any_busy)
                s->cv.wait_for(lk, std::chrono::microseconds(20));
            else
                s->cv.wait_for(lk, std::chrono::milliseconds(5),
                               [&] { return s->stop || !s->pending.empty(); });
        }
    }
}

}  // namespace

extern "C" hog_status hog_server_create(const hog_server_config *cfg, const float *tmpl_host,
                                        const float *bias_host, hog_server **out)
{
    if (!out) return srv_fail(HOG_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!cfg || !tmpl_host || !bias_host) return srv_fail(HOG_E_INVALID, "NULL argument");
    const hog_server_config c = *cfg;
    if (c.max_slots < 1 || c.max_slots > 4096 || c.max_batch < 1 || c.max_batch > c.max_slots ||
        c.streams < 1 || c.streams > 8)
        return srv_fail(HOG_E_INVALID, "need 1 <= max_batch <= max_slots <= 4096 and 1 <= streams <= 8");
    if (c.max_width < 1 || c.max_height < 1 || c.max_width > 32767 || c.max_height > 32767)
        return srv_fail(HOG_E_INVALID, "max_width / max_height outside [1, 32767]");
    if (c.memory_budget < 1) return srv_fail(HOG_E_INVALID, "memory_budget must be positive");
    if (c.max_queue < 1) return srv_fail(HOG_E_INVALID, "max_queue must be positive");
    // Validate the description through a plan of the largest image.
    hog_plan_desc d = desc_for(c, c.max_width, c.max_height);
    hog_plan *probe = nullptr;
    if (hog_plan_create(&d, &probe) != HOG_OK) {
        const std::string why = hog_last_error();
        return srv_fail(HOG_E_INVALID, "configuration rejected: %s", why.c_str());
    }
    hog_plan_sizes z;
    hog_plan_get_sizes(probe, &z);
    hog_plan_destroy(probe);

    hog_server *s = new (std::nothrow) hog_server;
    if (!s) return srv_fail(HOG_E_NOMEM, "host allocation failed");
    s->cfg = c;
    hipError_t e = hipGetDevice(&s->device);
    auto cleanup = [&](hog_status st, const char *what) {
        hog_server_destroy(s);
        return srv_fail(st, "%s", what);
    };
    if (e != hipSuccess) return cleanup(HOG_E_DEVICE, "hipGetDevice");
    if (hog_lut_build(c.n_bins, &s->lut) != HOG_OK) return cleanup(HOG_E_DEVICE, "lookup table");
    const size_t tb = (size_t)c.n_templates * z.feature_dim * 4, bb = (size_t)c.n_templates * 4;
    if (hipMalloc(&s->d_tmpl, tb) != hipSuccess || hipMalloc(&s->d_bias, bb) != hipSuccess)
        return cleanup(HOG_E_NOMEM, "templates");
    if (hipMemcpy(s->d_tmpl, tmpl_host, tb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_bias, bias_host, bb, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(HOG_E_DEVICE, "template upload");
    if (hipMalloc(&s->arena_base, (size_t)c.memory_budget) != hipSuccess)
        return cleanup(HOG_E_NOMEM, "arena of memory_budget bytes");
    s->arena.reset(c.memory_budget);
    const size_t in_cap = (size_t)c.max_batch * c.max_width * c.max_height * c.channels;
    s->slots.resize(c.streams);
    for (Slot &sl : s->slots) {
        sl.in_cap = in_cap;
        sl.out_cap = (size_t)c.max_batch * (size_t)std::max<int64_t>(z.score_elems, 1);
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&sl.pin_in, in_cap, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&sl.pin_out, sl.out_cap * 4, hipHostMallocDefault) != hipSuccess)
            return cleanup(HOG_E_NOMEM, "stream slot");
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return HOG_OK;
}

extern "C" void hog_server_destroy(hog_server *s)
{
    if (!s) return;
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
            s->pending.clear();  // queued, never started
        }
        s->cv.notify_all();
        s->worker.join();
    }
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.pin_in) (void)hipHostFree(sl.pin_in);
        if (sl.pin_out) (void)hipHostFree(sl.pin_out);
    }
    for (auto &kv : s->plans) hog_plan_destroy(kv.second);
    if (s->arena_base) (void)hipFree(s->arena_base);
    if (s->d_tmpl) (void)hipFree(s->d_tmpl);
    if (s->d_bias) (void)hipFree(s->d_bias);
    if (s->lut) hog_lut_free(s->lut);
    delete s;
}

extern "C" hog_status hog_submit(hog_server *s, const uint8_t *host_img, int w, int h, uint64_t *ticket)
{
    if (!s || !host_img || !ticket) return srv_fail(HOG_E_INVALID, "NULL argument");
    if (w < 1 || h < 1 || w > s->cfg.max_width || h > s->cfg.max_height)
        return srv_fail(HOG_E_INVALID, "image %dx%d outside [1, %d] x [1, %d]", w, h, s->cfg.max_width,
                        s->cfg.max_height);
    // Footprint of the image alone: it must fit the arena by itself.
    int64_t fp;
    {
        std::vector<std::pair<int, int>> key{{w, h}};
        hog_plan *p = plan_for(s, key);
        if (!p) {
            const std::string why = hog_last_error();
            return srv_fail(HOG_E_INVALID, "cannot plan a %dx%d image: %s", w, h, why.c_str());
        }
        fp = batch_bytes(p, (int64_t)w * h * s->cfg.channels);
    }
    if (fp > s->cfg.memory_budget)
        return srv_fail(HOG_E_INVALID, "a %dx%d image needs %lld bytes, over the memory budget", w, h,
                        (long long)fp);
    auto r = std::make_shared<Request>();
    r->w = w;
    r->h = h;
    r->img.assign(host_img, host_img + (size_t)w * h * s->cfg.channels);
    r->footprint = fp;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int)s->pending.size() >= s->cfg.max_queue) return srv_fail(HOG_E_BUSY, "queue full");
        r->ticket = s->next_ticket++;
        s->pending.push_back(r);
        s->live[r->ticket] = r;
    }
    s->cv.notify_all();
    *ticket = r->ticket;
    return HOG_OK;
}

extern "C" hog_status hog_poll(hog_server *s, uint64_t ticket, float *scores, size_t cap, int *nwx, int *nwy,
                               double *latency_s)
{
    if (!s) return srv_fail(HOG_E_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    if (it == s->live.end()) return srv_fail(HOG_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
    Request &r = *it->second;
    if (!r.ready) return HOG_E_NOT_READY;
    if (r.status != HOG_OK) {
        const hog_status st = r.status;
        s->live.erase(it);
        return srv_fail(st, "request failed on the device");
    }
    if (r.scores.size() > cap || (!scores && !r.scores.empty()))
        return srv_fail(HOG_E_INVALID, "scores needs %zu floats", r.scores.size());
    if (!r.scores.empty()) std::memcpy(scores, r.scores.data(), r.scores.size() * 4);
    if (nwx) *nwx = r.nwx;
    if (nwy) *nwy = r.nwy;
    if (latency_s) *latency_s = r.latency;
    s->live.erase(it);
    return HOG_OK;
}
