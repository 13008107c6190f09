// Host thread pool of the library's per-call descriptor work: every index of
// a parallel_for runs exactly once, the parts are the documented ranges, and
// concurrent callers (which fall back to running on their own thread) and
// thousands of back-to-back jobs neither lose nor repeat work.  Built with and
// without ThreadSanitizer by tests/test_host_pool.py.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../../paper_2607_02630_amd/csrc/host_pool.h"

using aesctr::HostPool;

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);    \
            std::exit(1);                                               \
        }                                                               \
    } while (0)

// Every index in [0, n) is visited once and each part is the range the
// header defines.
static void check_cover(size_t n, size_t grain)
{
    std::vector<std::atomic<int>> hits(n);
    for (auto &h : hits)
        h.store(0);
    const size_t parts = HostPool::parts(n, grain);
    const size_t per = n ? (n + parts - 1) / parts : 0;
    std::vector<std::atomic<int>> part_runs(parts);
    for (auto &p : part_runs)
        p.store(0);
    std::atomic<int> bad{0};
    HostPool::get().parallel_for(n, grain, [&](size_t p, size_t b, size_t e) {
        if (p >= parts || b != std::min(n, p * per) || e != std::min(n, (p + 1) * per) || b > e)
            bad.fetch_add(1);
        else
            part_runs[p].fetch_add(1);
        for (size_t i = b; i < e; ++i)
            hits[i].fetch_add(1);
    });
    CHECK(bad.load() == 0);
    for (size_t i = 0; i < n; ++i)
        CHECK(hits[i].load() == 1);
    if (n > 0)
        for (size_t p = 0; p < parts; ++p)
            CHECK(part_runs[p].load() == 1);
}

int main()
{
    // Part counts: about n / grain, clamped to [1, kMaxParts].
    CHECK(HostPool::parts(0, 16) == 1);
    CHECK(HostPool::parts(15, 16) == 1);
    CHECK(HostPool::parts(64, 16) == 4);
    CHECK(HostPool::parts(1 << 20, 1) == HostPool::kMaxParts);
    CHECK(HostPool::parts(10, 0) == 10);

    const size_t sizes[] = {0, 1, 15, 16, 17, 65, 1000, 4096, 262144 + 77};
    const size_t grains[] = {1, 2, 16, 256, 16384};
    for (size_t n : sizes)
        for (size_t g : grains)
            check_cover(n, g);

    // Many short jobs back to back: workers that wake late must neither run
    // a finished job nor miss a new one.
    for (int it = 0; it < 3000; ++it)
        check_cover(static_cast<size_t>(64 + it % 200), 1);

    // Concurrent callers: one holds the pool, the others run serially; all
    // results are complete.
    std::vector<std::thread> callers;
    std::atomic<int> failures{0};
    for (int t = 0; t < 6; ++t)
        callers.emplace_back([&, t] {
            for (int it = 0; it < 300; ++it) {
                const size_t n = 1000 + 37 * t + it;
                std::vector<std::atomic<int>> hits(n);
                for (auto &h : hits)
                    h.store(0);
                HostPool::get().parallel_for(n, 8, [&](size_t, size_t b, size_t e) {
                    for (size_t i = b; i < e; ++i)
                        hits[i].fetch_add(1);
                });
                for (size_t i = 0; i < n; ++i)
                    if (hits[i].load() != 1)
                        failures.fetch_add(1);
            }
        });
    for (auto &c : callers)
        c.join();
    CHECK(failures.load() == 0);
    std::printf("host pool ok\n");
    return 0;
}
