// Host-side copy helper of the request server: a few threads that split a
// large memcpy with the calling thread. Plain C++ (no HIP), so that it can be
// built and race-checked on its own.
#pragma once

#include <algorithm>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

namespace hogk {

// Helper threads that split large host copies with the caller. copy() may be
// called from several threads at once; each call returns once its own bytes
// are copied.
class CopyPool {
  public:
    void start(int n)
    {
        for (int i = 0; i < n; ++i) th_.emplace_back([this] { loop(); });
    }
    ~CopyPool()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    // dst[0, n) = src[0, n), in pieces of at least kMinPiece bytes spread
    // over the helpers and the calling thread; returns when all are done.
    void copy(uint8_t *dst, const uint8_t *src, size_t n)
    {
        const size_t parts = std::min<size_t>(th_.size() + 1, n / kMinPiece);
        if (parts <= 1) {
            std::memcpy(dst, src, n);
            return;
        }
        const size_t piece = (n / parts + 63) & ~(size_t)63;
        int left = 0;
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (size_t o = piece; o < n; o += piece) {
                q_.push_back({dst + o, src + o, std::min(piece, n - o), &left});
                ++left;
            }
        }
        cv_.notify_all();
        std::memcpy(dst, src, std::min(piece, n));
        // Take back pieces no helper has started (the queue may change while
        // the lock is dropped: search again each time), then wait for the rest.
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            auto it = std::find_if(q_.begin(), q_.end(), [&](const Piece &t) { return t.left == &left; });
            if (it == q_.end()) break;
            const Piece t = *it;
            q_.erase(it);
            lk.unlock();
            std::memcpy(t.dst, t.src, t.n);
            lk.lock();
            --left;
        }
        done_cv_.wait(lk, [&] { return left == 0; });
    }

  private:
    static constexpr size_t kMinPiece = size_t(1) << 20;
    struct Piece {
        uint8_t *dst;
        const uint8_t *src;
        size_t n;
        int *left;  // guarded by mu_
    };
    void loop()
    {
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
            if (stop_) return;
            const Piece t = q_.front();
            q_.pop_front();
            lk.unlock();
            std::memcpy(t.dst, t.src, t.n);
            lk.lock();
            if (--*t.left == 0) done_cv_.notify_all();
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<Piece> q_;
    bool stop_ = false;
};

}  // namespace hogk
