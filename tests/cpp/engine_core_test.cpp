// Host-logic test of the serving engine's scheduling core (no GPU, no AES):
// a stand-in driver thread takes batches and completes them after a short
// delay, while several submitter threads push requests of mixed sizes.
// Checks: the byte budget is never exceeded, admission is FIFO, every ticket
// completes exactly once, poll/wait semantics, oversize rejection, shutdown.
// Built with g++ -fsanitize=thread by tests/test_engine_core.py.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "../../paper_2607_02630_amd/csrc/engine_core.h"

using namespace aesctr;
struct Rec {
    uint64_t tag;
};
using Core = EngineCore<Rec>;

#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "CHECK failed: %s (line %d)\n", #c, __LINE__);   \
            std::exit(1);                                                         \
        }                                                                         \
    } while (0)

int main()
{
    const uint64_t budget = 64 << 20;
    Core core(budget, 256, budget);
    std::atomic<uint64_t> inflight{0}, max_inflight{0};
    std::atomic<bool> stop{false};
    std::atomic<uint64_t> last_taken{0};
    std::atomic<int> order_violations{0};

    // Stand-in driver: up to two batches in flight, each "runs" ~50 us.
    std::thread driver([&] {
        std::vector<Core::Req> slots[2];
        std::vector<Core::Req> b;
        for (;;) {
            bool any = false;
            for (auto &s : slots) {
                if (!s.empty()) {
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
                    uint64_t bytes = 0;
                    for (auto &r : s) bytes += r.bytes;
                    inflight -= bytes;
                    core.complete(s, AES_OK, Core::now_ns());
                    s.clear();
                    any = true;
                }
                if (core.take_batch(b)) {
                    uint64_t bytes = 0;
                    for (auto &r : b) {
                        bytes += r.bytes;
                        if (r.ticket <= last_taken.load()) ++order_violations;
                        last_taken = r.ticket;
                    }
                    uint64_t now = inflight += bytes;
                    uint64_t m = max_inflight.load();
                    while (now > m && !max_inflight.compare_exchange_weak(m, now)) {}
                    s.swap(b);
                    any = true;
                }
            }
            if (!any) {
                if (core.closing_and_drained()) break;
                core.wait_for_work(1000000);
            }
        }
    });

    // Oversize request is rejected outright.
    uint64_t t;
    Core::Req big;
    big.bytes = budget + 1;
    CHECK(core.submit(std::move(big), &t) == AES_EAGAIN);

    // Submitters.
    const int nthreads = 4, per = 3000;
    std::vector<std::vector<uint64_t>> tickets(nthreads);
    std::vector<std::thread> subs;
    for (int k = 0; k < nthreads; ++k) {
        subs.emplace_back([&, k] {
            std::mt19937_64 g(k);
            const uint64_t sizes[3] = {64 << 10, 1 << 20, 8 << 20};
            for (int i = 0; i < per; ++i) {
                Core::Req r;
                double u = std::uniform_real_distribution<double>(0, 1)(g);
                r.bytes = sizes[u < 0.70 ? 0 : u < 0.95 ? 1 : 2];
                r.payload = r.bytes;
                uint64_t tk;
                CHECK(core.submit(std::move(r), &tk) == AES_OK);
                tickets[k].push_back(tk);
            }
        });
    }
    for (auto &s : subs) s.join();

    // Wait for all; each ticket retires exactly once.
    for (auto &v : tickets)
        for (uint64_t tk : v) {
            CHECK(core.wait(tk, 20 * 1000 * 1000) == AES_OK);
            CHECK(core.poll(tk) == AES_ENOTFOUND);
        }
    CHECK(max_inflight.load() <= budget);
    CHECK(order_violations.load() == 0);

    aes_stats_t st;
    core.stats(&st);
    CHECK(st.submitted == uint64_t(nthreads * per));
    CHECK(st.completed == st.submitted);
    CHECK(st.rejected == 1);
    CHECK(st.budget_high_water <= budget && st.budget_high_water > 0);
    CHECK(st.p50_us > 0 && st.p99_us >= st.p50_us && st.p999_us >= st.p99_us);
    CHECK(st.queued_now == 0 && st.inflight_now == 0);

    // Unknown ticket, and a wait that times out on a request still queued.
    CHECK(core.poll(999999999) == AES_ENOTFOUND);
    core.close();
    Core::Req late;
    late.bytes = 16;
    CHECK(core.submit(std::move(late), &t) == AES_ECLOSED);
    driver.join();

    // A fresh core with no driver: the request stays pending; cancel fails it.
    Core idle(budget, 8, budget);
    Core::Req r;
    r.bytes = 100;
    uint64_t tk;
    CHECK(idle.submit(std::move(r), &tk) == AES_OK);
    CHECK(idle.poll(tk) == 0);
    CHECK(idle.wait(tk, 1000) == AES_ETIMEDOUT);
    idle.cancel_queued(AES_ECANCELED);
    CHECK(idle.poll(tk) == AES_ECANCELED);
    // The per-launch cap counts payload bytes, the budget counts the weight
    // (buffers + records): out-of-place requests of 400 payload bytes weigh
    // 800 + 320; a 1000-byte cap takes two per launch, and the budget of
    // 3 * 1120 admits three in flight.
    {
        Core capq(3 * 1120, 64, 1000);
        for (int i = 0; i < 5; ++i) {
            Core::Req rq;
            rq.payload = 400;
            rq.bytes = 2 * 400 + 320;
            uint64_t tk3;
            CHECK(capq.submit(std::move(rq), &tk3) == AES_OK);
        }
        std::vector<Core::Req> b1, b2, b3;
        CHECK(capq.take_batch(b1) && b1.size() == 2);
        CHECK(capq.take_batch(b2) && b2.size() == 1);     // budget: 3 in flight
        CHECK(!capq.take_batch(b3));
        capq.complete(b1, AES_OK, Core::now_ns());
        CHECK(capq.take_batch(b3) && b3.size() == 2);
        aes_stats_t cs;
        capq.stats(&cs);
        CHECK(cs.budget_high_water == 3 * 1120 && cs.bytes_completed == 800);
        capq.complete(b2, AES_OK, Core::now_ns());
        capq.complete(b3, AES_OK, Core::now_ns());
    }
    // Back-pressure: with no driver the ring fills; the next submitter waits
    // until the driver takes requests, then goes on.
    {
        Core q(uint64_t(1) << 40, 4096, uint64_t(1) << 40);
        const uint64_t cap = Core::kQueueCap;
        std::atomic<uint64_t> done_subs{0};
        std::thread sub([&] {
            for (uint64_t i = 0; i < cap + 100; ++i) {
                Core::Req rq;
                rq.bytes = 16;
                uint64_t tk2;
                CHECK(q.submit(std::move(rq), &tk2) == AES_OK);
                done_subs.fetch_add(1);
            }
        });
        while (done_subs.load() < cap)
            std::this_thread::yield();
        std::this_thread::sleep_for(std::chrono::milliseconds(20));
        CHECK(done_subs.load() == cap);                   // blocked on the full ring
        aes_stats_t qs;
        q.stats(&qs);
        CHECK(qs.queued_now == cap);
        std::vector<Core::Req> b2;
        uint64_t taken = 0, expect = 1;
        while (taken < cap + 100) {
            if (q.take_batch(b2)) {
                for (auto &r2 : b2) CHECK(r2.ticket == expect++);
                taken += b2.size();
                q.complete(b2, AES_OK, Core::now_ns());
            } else {
                std::this_thread::yield();
            }
        }
        sub.join();
        // Two threads polling one finished ticket: exactly one retires it.
        std::atomic<int> ones{0}, notfound{0};
        std::thread p1([&] { int r1 = q.poll(7); (r1 == 1 ? ones : notfound).fetch_add(1); });
        std::thread p2([&] { int r2 = q.poll(7); (r2 == 1 ? ones : notfound).fetch_add(1); });
        p1.join();
        p2.join();
        CHECK(ones.load() == 1 && notfound.load() == 1);
        CHECK(q.wait(8, 0) == AES_OK && q.poll(8) == AES_ENOTFOUND);
    }

    // A submitter blocked on a full ring gives up with AES_ECLOSED at close;
    // cancel_queued then fails everything that was queued.
    {
        Core q(uint64_t(1) << 40, 4096, uint64_t(1) << 40);
        std::atomic<int> closed_rc{0};
        std::atomic<uint64_t> n_ok{0};
        std::thread sub([&] {
            for (;;) {
                Core::Req rq;
                rq.bytes = 16;
                uint64_t tk2;
                int rc2 = q.submit(std::move(rq), &tk2);
                if (rc2 != AES_OK) {
                    closed_rc = rc2;
                    return;
                }
                n_ok.fetch_add(1);
            }
        });
        while (n_ok.load() < Core::kQueueCap)
            std::this_thread::yield();
        q.close();
        sub.join();
        CHECK(closed_rc.load() == AES_ECLOSED);
        q.cancel_queued(AES_ECANCELED);
        CHECK(q.poll(1) == AES_ECANCELED && q.poll(Core::kQueueCap) == AES_ECANCELED);
        CHECK(q.closing_and_drained());
    }

    // Submission rate with four threads and a draining driver (printed only).
    {
        Core q(uint64_t(1) << 40, 4096, uint64_t(1) << 40);
        std::atomic<bool> fin{false};
        std::thread drv([&] {
            std::vector<Core::Req> b3;
            while (!fin.load() || q.take_batch(b3)) {
                if (q.take_batch(b3))
                    q.complete(b3, AES_OK, Core::now_ns());
                else
                    std::this_thread::yield();
            }
        });
        const int per2 = 200000;
        const int64_t t0 = Core::now_ns();
        std::vector<std::thread> ss;
        for (int k = 0; k < 4; ++k)
            ss.emplace_back([&] {
                for (int i = 0; i < per2; ++i) {
                    Core::Req rq;
                    rq.bytes = 65536;
                    uint64_t tk2;
                    CHECK(q.submit(std::move(rq), &tk2) == AES_OK);
                }
            });
        for (auto &th : ss) th.join();
        const double el = (Core::now_ns() - t0) * 1e-9;
        fin = true;
        drv.join();
        std::printf("submit rate, 4 threads: %.2f M/s\n", 4.0 * per2 / el / 1e6);
    }

    std::printf("engine core ok: max in flight %llu of %llu bytes, %llu batches, mean %.1f req/batch\n",
                (unsigned long long)max_inflight.load(), (unsigned long long)budget,
                (unsigned long long)st.batches, st.mean_batch_reqs);
    return 0;
}
