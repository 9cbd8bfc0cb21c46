// Request serving with continuous batching (hog_server_*, hog_submit,
// hog_poll): the scan of Sec. 4 applied to a stream of images.
//
// hog_submit copies a host image into the server's pinned host arena and
// returns a ticket. A worker thread forms batches: the oldest waiting
// request and the waiting requests of the same image size behind it, as many
// as in-flight slots and device memory allow. Admission is by the device
// footprint of the batch's buffers (bins, integral images, workspace,
// scores), carved from one arena allocated at creation. The batch's images
// are copied in from pinned memory, run through hog_run on a batch plan (one
// launch per kernel for all its images), and its scores copied back, all on
// one of several non-blocking streams; requests that arrive while batches
// are on the device form the next batch on another stream. Batches of one
// size keep the plan cache to (sizes seen) x max_batch entries, each built
// once (building one allocates and copies its tables synchronously, too slow
// to do per batch). The lookup table and the templates stay resident.
// hog_wait_any reports finished tickets as they complete; hog_poll returns a
// finished request's scores and its latency (submit to ready, host clock).
#include "hog.h"
#include "hog_internal.h"
#include "copy_pool.h"

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
    int64_t img_off = 0, img_bytes = 0;  // the image in the pinned host arena
    int64_t footprint = 0;               // device bytes of the image alone
    Clock::time_point t_submit;
    bool ready = false;
    hog_status status = HOG_OK;
    int64_t out_off = -1, n_scores = 0;  // the scores in the pinned output arena
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
    o = align256(o + z.ii_elems * z.ii_elem_bytes);
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
    bool busy = false;
    std::vector<ReqPtr> reqs;
    hog_plan *plan = nullptr;  // pinned in the plan cache while the batch runs
    std::vector<std::pair<int, int>> plan_key;
    int64_t off = 0, bytes = 0;
};

// A cached batch plan: pinned (pins > 0) while a caller or a running batch
// uses it; unpinned plans are evicted least recently used first.
struct CachedPlan {
    hog_plan *plan = nullptr;
    uint64_t last_use = 0;
    int pins = 0;
};

}  // namespace

struct hog_server {
    hog_server_config cfg;
    int device = 0;
    hog_lut *lut = nullptr;
    float *d_tmpl = nullptr, *d_bias = nullptr;
    uint8_t *arena_base = nullptr;
    Arena arena;
    uint8_t *host_base = nullptr;  // pinned host arena for queued images
    Arena host_arena;
    uint8_t *out_base = nullptr;   // pinned arena for finished requests' scores
    Arena out_arena;
    hogk::CopyPool copies;
    std::vector<Slot> slots;
    std::map<std::vector<std::pair<int, int>>, CachedPlan> plans;  // by batch composition
    size_t plan_cap = 0;     // cached plans kept: 4 max_batch + 16
    uint64_t plan_clock = 0;
    std::mutex mu;                                                 // guards the fields below
    std::condition_variable cv;       // wakes the worker
    std::condition_variable done_cv;  // wakes hog_wait_any
    std::deque<ReqPtr> pending;
    std::deque<uint64_t> done_q;      // finished, not yet reported by hog_wait_any
    std::map<uint64_t, ReqPtr> live;  // submitted and not yet returned by hog_poll
    int in_flight = 0;                // requests on the device
    uint64_t events = 0;              // bumped by every change that may let the worker admit
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
    d.votes = c.votes;
    d.plane_bits = c.plane_bits;
    return d;
}

// The cached batch plan for the given sizes (in order), pinned for the caller
// (release it with plan_release); nullptr on failure. A new plan's tables go
// to the server's device; the calling thread's current device is left as it
// was. Beyond plan_cap cached plans, unpinned ones are destroyed least
// recently used first, so that a stream of ever new image sizes does not
// hold plan tables without bound.
hog_plan *plan_for(hog_server *s, const std::vector<std::pair<int, int>> &key)
{
    std::lock_guard<std::mutex> lk(s->plan_mu);
    auto it = s->plans.find(key);
    if (it != s->plans.end()) {
        it->second.last_use = ++s->plan_clock;
        ++it->second.pins;
        return it->second.plan;
    }
    std::vector<hog_plan_desc> descs;
    for (auto &wh : key) descs.push_back(desc_for(s->cfg, wh.first, wh.second));
    int prev = -1;
    const bool switched = hipGetDevice(&prev) == hipSuccess && prev != s->device &&
                          hipSetDevice(s->device) == hipSuccess;
    hog_plan *p = nullptr;
    const hog_status st = hog_plan_create_batch(descs.data(), (int)descs.size(), &p);
    if (switched) (void)hipSetDevice(prev);
    if (st != HOG_OK) return nullptr;
    CachedPlan &cp = s->plans[key];
    cp.plan = p;
    cp.last_use = ++s->plan_clock;
    cp.pins = 1;
    while (s->plans.size() > s->plan_cap) {
        auto victim = s->plans.end();
        for (auto jt = s->plans.begin(); jt != s->plans.end(); ++jt)
            if (jt->second.pins == 0 && (victim == s->plans.end() || jt->second.last_use < victim->second.last_use))
                victim = jt;
        if (victim == s->plans.end()) break;  // every cached plan is in use
        hog_plan_destroy(victim->second.plan);
        s->plans.erase(victim);
    }
    return p;
}

void plan_release(hog_server *s, const std::vector<std::pair<int, int>> &key)
{
    std::lock_guard<std::mutex> lk(s->plan_mu);
    auto it = s->plans.find(key);
    if (it != s->plans.end() && it->second.pins > 0) --it->second.pins;
}

int64_t batch_bytes(hog_plan *p, int64_t img_bytes)
{
    hog_plan_sizes z;
    hog_plan_get_sizes(p, &z);
    return layout_of(z, img_bytes).total;
}

// Finished batch: its requests become ready (their scores are already in
// their output regions), its device memory goes back to the arena. Copies
// nothing.
void finish(hog_server *s, Slot &sl, hipError_t err)
{
    const auto now = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &rp : sl.reqs) {
        Request &r = *rp;
        if (err != hipSuccess) {
            r.status = HOG_E_DEVICE;
            if (r.out_off >= 0) s->out_arena.release(r.out_off, align256(r.n_scores * 4));
            r.out_off = -1;
        }
        r.latency = std::chrono::duration<double>(now - r.t_submit).count();
        r.ready = true;
        s->host_arena.release(r.img_off, align256(r.img_bytes));
        s->done_q.push_back(r.ticket);
    }
    s->done_cv.notify_all();
    s->arena.release(sl.off, sl.bytes);
    s->in_flight -= (int)sl.reqs.size();
    sl.reqs.clear();
    sl.busy = false;
    ++s->events;
    if (sl.plan) plan_release(s, sl.plan_key);
    sl.plan = nullptr;
}

// Launches one batch into a free slot if requests and memory allow: the
// oldest waiting request and those of its size behind it, in arrival order.
bool admit(hog_server *s, Slot &sl)
{
    std::vector<ReqPtr> take;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const int room = std::min(s->cfg.max_batch, s->cfg.max_slots - s->in_flight);
        if (room > 0 && !s->pending.empty()) {
            const int w = s->pending.front()->w, h = s->pending.front()->h;
            for (auto it = s->pending.begin(); it != s->pending.end() && (int)take.size() < room; ++it)
                if ((*it)->w == w && (*it)->h == h) take.push_back(*it);
        }
    }
    if (take.empty()) return false;
    // Largest batch (oldest first) whose buffers fit the arena now.
    while (!take.empty()) {
        const std::vector<ReqPtr> &order = take;
        std::vector<std::pair<int, int>> key;
        int64_t img_bytes = 0;
        for (auto &r : order) {
            key.emplace_back(r->w, r->h);
            img_bytes += r->img_bytes;
        }
        hog_plan *p = plan_for(s, key);
        if (!p && take.size() > 1) {  // cannot plan this batch (e.g. out of memory): try a smaller one
            take.pop_back();
            continue;
        }
        if (!p) {  // cannot plan even this request alone: fail it
            std::lock_guard<std::mutex> lk(s->mu);
            ReqPtr r = take.front();
            r->status = HOG_E_INVALID;
            r->ready = true;
            s->host_arena.release(r->img_off, align256(r->img_bytes));
            s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
            s->done_q.push_back(r->ticket);
            s->done_cv.notify_all();
            return true;
        }
        const int64_t bytes = batch_bytes(p, img_bytes);
        hog_plan_sizes z;
        hog_plan_get_sizes(p, &z);
        // Each request's scores: [a, b) of the batch's score buffer.
        const int K = s->cfg.n_templates;
        std::vector<int64_t> sc_a(order.size()), sc_n(order.size());
        for (size_t i = 0; i < order.size(); ++i) {
            hog_image_info im;
            hog_plan_get_image(p, (int)i, &im);
            hog_level_info first, last;
            hog_plan_get_level(p, im.first_level, &first);
            hog_plan_get_level(p, im.first_level + im.n_levels - 1, &last);
            sc_a[i] = first.score_offset;
            sc_n[i] = last.score_offset + (int64_t)last.windows_x * last.windows_y * K - sc_a[i];
            order[i]->nwx = first.windows_x;
            order[i]->nwy = first.windows_y;
            order[i]->n_scores = sc_n[i];
        }
        int64_t off = 0;
        bool ok;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            ok = s->arena.alloc(bytes, &off);
            size_t i = 0;
            for (; ok && i < order.size(); ++i)
                if (sc_n[i] > 0 && !s->out_arena.alloc(align256(sc_n[i] * 4), &order[i]->out_off)) ok = false;
            if (!ok) {  // undo
                for (size_t j = 0; j + 1 < i; ++j)
                    if (sc_n[j] > 0) s->out_arena.release(order[j]->out_off, align256(sc_n[j] * 4));
                if (i > 0) s->arena.release(off, bytes);
                for (auto &r : order) r->out_off = -1;
            } else {
                for (auto &r : take) s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
                s->in_flight += (int)take.size();
            }
        }
        if (!ok) {
            plan_release(s, key);
            take.pop_back();
            continue;
        }
        // Copy the images in (packed as the batch plan reads them), run, copy
        // the scores out.
        const Layout L = layout_of(z, img_bytes);
        uint8_t *base = s->arena_base + off;
        hipError_t e = hipSuccess;
        for (int i = 0; i < (int)order.size() && e == hipSuccess; ++i) {
            hog_image_info im;
            hog_plan_get_image(p, i, &im);
            e = hipMemcpyAsync(base + L.img + im.img_offset, s->host_base + order[i]->img_off,
                               (size_t)order[i]->img_bytes, hipMemcpyHostToDevice, sl.stream);
        }
        hog_status st = HOG_OK;
        if (e == hipSuccess)
            st = hog_run(p, s->lut, base + L.img, 0, base + L.bins, base + L.ii, s->d_tmpl,
                         s->d_bias, (float *)(base + L.scores), base + L.ws, sl.stream);
        for (size_t i = 0; i < order.size() && e == hipSuccess && st == HOG_OK; ++i)
            if (sc_n[i] > 0)
                e = hipMemcpyAsync(s->out_base + order[i]->out_off, base + L.scores + sc_a[i] * 4,
                                   (size_t)sc_n[i] * 4, hipMemcpyDeviceToHost, sl.stream);
        if (e == hipSuccess && st == HOG_OK) e = hipEventRecord(sl.done, sl.stream);
        sl.reqs = order;
        sl.plan = p;
        sl.plan_key = key;
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
        uint64_t seen;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            seen = s->events;
        }
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
            // Batches on the device: poll their events again soon. Otherwise
            // sleep until a submission, a poll that frees output space, or
            // stop (events counts them, so none is missed).
            if (any_busy)
                s->cv.wait_for(lk, std::chrono::microseconds(20));
            else
                s->cv.wait_for(lk, std::chrono::milliseconds(50),
                               [&] { return s->stop || s->events != seen; });
        }
    }
}

// Callers that only poll never drain the completion queue: drop the tickets
// hog_poll has taken once they outnumber the live ones (caller holds mu).
void forget_done(hog_server *s)
{
    if (s->done_q.size() <= 2 * s->live.size() + 64) return;
    std::deque<uint64_t> keep;
    for (uint64_t t : s->done_q)
        if (s->live.count(t)) keep.push_back(t);
    s->done_q.swap(keep);
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
    if (c.copy_threads < 0 || c.copy_threads > 32) return srv_fail(HOG_E_INVALID, "copy_threads outside [0, 32]");
    if (c.orientation != HOG_ORIENT_SIGNED && c.orientation != HOG_ORIENT_UNSIGNED)
        return srv_fail(HOG_E_INVALID, "orientation must be HOG_ORIENT_SIGNED or HOG_ORIENT_UNSIGNED");
    const int64_t max_img = (int64_t)c.max_width * c.max_height * c.channels;
    if (c.host_budget < max_img) return srv_fail(HOG_E_INVALID, "host_budget must hold the largest image");
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
    s->plan_cap = 4 * (size_t)c.max_batch + 16;
    hipError_t e = hipGetDevice(&s->device);
    auto cleanup = [&](hog_status st, const char *what) {
        hog_server_destroy(s);
        return srv_fail(st, "%s", what);
    };
    if (e != hipSuccess) return cleanup(HOG_E_DEVICE, "hipGetDevice");
    if (hog_lut_build_ex(c.n_bins, c.orientation, &s->lut) != HOG_OK) return cleanup(HOG_E_DEVICE, "lookup table");
    const size_t tb = (size_t)c.n_templates * z.feature_dim * 4, bb = (size_t)c.n_templates * 4;
    if (hipMalloc(&s->d_tmpl, tb) != hipSuccess || hipMalloc(&s->d_bias, bb) != hipSuccess)
        return cleanup(HOG_E_NOMEM, "templates");
    if (hipMemcpy(s->d_tmpl, tmpl_host, tb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_bias, bias_host, bb, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(HOG_E_DEVICE, "template upload");
    if (hipMalloc(&s->arena_base, (size_t)c.memory_budget) != hipSuccess)
        return cleanup(HOG_E_NOMEM, "arena of memory_budget bytes");
    s->arena.reset(c.memory_budget);
    if (hipHostMalloc((void **)&s->host_base, (size_t)c.host_budget, hipHostMallocDefault) != hipSuccess)
        return cleanup(HOG_E_NOMEM, "pinned host arena of host_budget bytes");
    s->host_arena.reset(c.host_budget);
    // Scores of the requests on the device and of finished ones not yet
    // polled: twice max_slots requests of the largest image.
    const int64_t out_bytes = 2 * (int64_t)c.max_slots * align256(std::max<int64_t>(z.score_elems, 1) * 4);
    if (hipHostMalloc((void **)&s->out_base, (size_t)out_bytes, hipHostMallocDefault) != hipSuccess)
        return cleanup(HOG_E_NOMEM, "pinned output arena");
    s->out_arena.reset(out_bytes);
    s->slots.resize(c.streams);
    for (Slot &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
            return cleanup(HOG_E_NOMEM, "stream slot");
    }
    s->copies.start(c.copy_threads);
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
            ++s->events;
            s->pending.clear();  // queued, never started
        }
        s->cv.notify_all();
        s->worker.join();
    }
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (s->host_base) (void)hipHostFree(s->host_base);
    if (s->out_base) (void)hipHostFree(s->out_base);
    for (auto &kv : s->plans) hog_plan_destroy(kv.second.plan);
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
        plan_release(s, key);
    }
    if (fp > s->cfg.memory_budget)
        return srv_fail(HOG_E_INVALID, "a %dx%d image needs %lld bytes, over the memory budget", w, h,
                        (long long)fp);
    auto r = std::make_shared<Request>();
    r->w = w;
    r->h = h;
    r->img_bytes = (int64_t)w * h * s->cfg.channels;
    r->footprint = fp;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int)s->pending.size() >= s->cfg.max_queue) return srv_fail(HOG_E_BUSY, "queue full");
        if (!s->host_arena.alloc(align256(r->img_bytes), &r->img_off))
            return srv_fail(HOG_E_BUSY, "pinned host arena full");
    }
    // The region is this request's alone until its batch finishes.
    s->copies.copy(s->host_base + r->img_off, host_img, (size_t)r->img_bytes);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next_ticket++;
        s->pending.push_back(r);
        s->live[r->ticket] = r;
        ++s->events;
    }
    s->cv.notify_all();
    *ticket = r->ticket;
    return HOG_OK;
}

extern "C" hog_status hog_poll(hog_server *s, uint64_t ticket, float *scores, size_t cap, int *nwx, int *nwy,
                               double *latency_s)
{
    if (!s) return srv_fail(HOG_E_INVALID, "server is NULL");
    ReqPtr r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->live.find(ticket);
        if (it == s->live.end())
            return srv_fail(HOG_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
        r = it->second;
        if (!r->ready) return HOG_E_NOT_READY;
        if (r->status == HOG_OK && ((size_t)r->n_scores > cap || (!scores && r->n_scores > 0)))
            return srv_fail(HOG_E_INVALID, "scores needs %lld floats", (long long)r->n_scores);
        s->live.erase(it);  // the request is the caller's alone from here
        forget_done(s);
    }
    if (r->status != HOG_OK) return srv_fail(r->status, "request failed on the device");
    if (r->n_scores > 0) std::memcpy(scores, s->out_base + r->out_off, (size_t)r->n_scores * 4);
    if (nwx) *nwx = r->nwx;
    if (nwy) *nwy = r->nwy;
    if (latency_s) *latency_s = r->latency;
    if (r->out_off >= 0) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->out_arena.release(r->out_off, align256(r->n_scores * 4));
        ++s->events;
        s->cv.notify_all();  // output space for the worker
    }
    return HOG_OK;
}

extern "C" hog_status hog_wait_any(hog_server *s, uint64_t *tickets, int cap, int64_t timeout_us, int *count)
{
    if (count) *count = 0;
    if (!s || !tickets || !count) return srv_fail(HOG_E_INVALID, "NULL argument");
    if (cap < 1 || timeout_us < 0) return srv_fail(HOG_E_INVALID, "need cap >= 1 and timeout_us >= 0");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done_q.empty() && timeout_us > 0)
        s->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !s->done_q.empty(); });
    int n = 0;
    while (n < cap && !s->done_q.empty()) {
        const uint64_t t = s->done_q.front();
        s->done_q.pop_front();
        if (s->live.count(t)) tickets[n++] = t;  // not yet taken by hog_poll
    }
    *count = n;
    return HOG_OK;
}

extern "C" hog_status hog_server_warm(hog_server *s, int w, int h)
{
    if (!s) return srv_fail(HOG_E_INVALID, "server is NULL");
    if (w < 1 || h < 1 || w > s->cfg.max_width || h > s->cfg.max_height)
        return srv_fail(HOG_E_INVALID, "image %dx%d outside [1, %d] x [1, %d]", w, h, s->cfg.max_width,
                        s->cfg.max_height);
    std::vector<std::pair<int, int>> key;
    for (int n = 1; n <= s->cfg.max_batch; ++n) {
        key.emplace_back(w, h);
        if (!plan_for(s, key)) {
            const std::string why = hog_last_error();
            return srv_fail(HOG_E_INVALID, "cannot plan %d images of %dx%d: %s", n, w, h, why.c_str());
        }
        plan_release(s, key);
    }
    return HOG_OK;
}
