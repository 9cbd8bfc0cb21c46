// Race and correctness check of the server's copy pool (host code only):
// several threads copy buffers of assorted sizes through one pool at once
// and each checks its destination byte for byte.
#include "copy_pool.h"

#include <cstdio>
#include <cstdlib>
#include <random>

int main(int argc, char **argv)
{
    const int helpers = argc > 1 ? std::atoi(argv[1]) : 3;
    hogk::CopyPool pool;
    pool.start(helpers);
    const size_t sizes[] = {0, 1, 4096, (1 << 20) - 1, 1 << 20, (2 << 20) + 17, 5 << 20, 9 << 20};
    int bad = 0;
    std::mutex bad_mu;
    auto worker = [&](int id) {
        std::mt19937 rng(1000 + id);
        for (int round = 0; round < 6; ++round) {
            for (size_t n : sizes) {
                std::vector<uint8_t> src(n + 64), dst(n + 64, 0xAB);
                for (auto &b : src) b = (uint8_t)rng();
                const size_t off = rng() % 64;  // unaligned starts
                pool.copy(dst.data() + off, src.data() + off, n);
                bool ok = std::memcmp(dst.data() + off, src.data() + off, n) == 0;
                for (size_t i = 0; i < off; ++i) ok = ok && dst[i] == 0xAB;
                for (size_t i = off + n; i < dst.size(); ++i) ok = ok && dst[i] == 0xAB;
                if (!ok) {
                    std::lock_guard<std::mutex> lk(bad_mu);
                    ++bad;
                    std::fprintf(stderr, "thread %d: %zu bytes at +%zu wrong\n", id, n, off);
                }
            }
        }
    };
    std::vector<std::thread> th;
    for (int i = 0; i < 4; ++i) th.emplace_back(worker, i);
    for (auto &t : th) t.join();
    std::printf("%s\n", bad ? "FAIL" : "OK");
    return bad ? 1 : 0;
}
