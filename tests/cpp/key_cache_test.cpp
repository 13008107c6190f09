// Host-logic test of the engine's resident key cache (no GPU, no AES).
//
// A stand-in driver forms "launches" of requests drawn from a pool of keys,
// keeps up to three launches in flight and completes them in random order
// (some failing).  A shadow model of the device key table checks what the
// cache promises the kernels:
//   - a hit names a slot whose installed key equals the request's key and
//     whose installing launch has completed successfully;
//   - a slot is never handed out for an install while any launch in flight
//     reads it or installs into it;
//   - hits and misses add up to the requests, and a key pool no larger than
//     the slot count ends up hitting almost always;
//   - the LRU list and index stay consistent throughout.
// Built by tests/test_engine_core.py (plain, ThreadSanitizer and
// AddressSanitizer builds).
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "../../paper_2607_02630_amd/csrc/key_cache.h"

using namespace aesctr;

#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "CHECK failed: %s (line %d)\n", #c, __LINE__);   \
            std::exit(1);                                                         \
        }                                                                         \
    } while (0)

struct Key {
    uint32_t rk[60];
    uint32_t nr;
};

static Key make_key(std::mt19937_64 &g, bool aes256)
{
    Key k{};
    k.nr = aes256 ? 14 : 10;
    for (uint32_t i = 0; i < 4 * (k.nr + 1); ++i)
        k.rk[i] = static_cast<uint32_t>(g());
    return k;
}

struct Launch {
    std::vector<KeyCache::Ref> refs;
    std::vector<int> key_of_ref;   // pool index per ref
};

// Shadow of the device table: which key each slot holds once its install
// completed, and how many launches in flight touch it.
struct Shadow {
    std::vector<int> key;       // pool index, -1 = nothing valid
    std::vector<int> touching;  // launches in flight that read or install the slot
};

static void run(int slots, int pool_size, int launches, uint64_t seed, double fail_rate, bool expect_hits)
{
    std::mt19937_64 g(seed);
    std::vector<Key> pool;
    for (int i = 0; i < pool_size; ++i)
        pool.push_back(make_key(g, i % 2 == 1));
    KeyCache cache(slots);
    Shadow sh{std::vector<int>(slots, -1), std::vector<int>(slots, 0)};
    std::deque<Launch> inflight;
    uint64_t requests = 0;
    std::uniform_int_distribution<int> pick(0, pool_size - 1);
    std::uniform_int_distribution<int> size(1, 24);
    std::uniform_real_distribution<double> u(0, 1);

    auto complete = [&](size_t i) {
        Launch l = std::move(inflight[i]);
        inflight.erase(inflight.begin() + static_cast<long>(i));
        const bool ok = u(g) >= fail_rate;
        for (size_t j = 0; j < l.refs.size(); ++j) {
            const KeyCache::Ref &r = l.refs[j];
            CHECK(r.slot >= 0);
            CHECK(sh.touching[r.slot] > 0);
            --sh.touching[r.slot];
            if (r.install)
                sh.key[r.slot] = ok ? l.key_of_ref[j] : -1;
            cache.release(r, ok);
        }
        CHECK(cache.consistent());
    };

    for (int n = 0; n < launches; ++n) {
        // Complete launches in random order while three are in flight.
        while (inflight.size() >= 3)
            complete(static_cast<size_t>(g() % inflight.size()));
        Launch l;
        const int m = size(g);
        for (int q = 0; q < m; ++q) {
            const int k = pick(g);
            const KeyCache::Ref r = cache.acquire(pool[k].rk, pool[k].nr);
            ++requests;
            CHECK(!(r.resident && r.install));
            if (r.resident) {
                CHECK(r.slot >= 0 && r.slot < slots);
                CHECK(sh.key[r.slot] == k);        // the installed key, completed
            }
            if (r.install) {
                CHECK(r.slot >= 0 && r.slot < slots);
                CHECK(sh.touching[r.slot] == 0);   // nobody in flight reads or fills it
                sh.key[r.slot] = -1;               // contents undefined until it completes
            }
            if (r.pending >= 0)
                CHECK(r.slot < 0 && !r.resident && !r.install);
            if (r.slot >= 0) {
                ++sh.touching[r.slot];
                l.refs.push_back(r);
                l.key_of_ref.push_back(k);
            }
        }
        inflight.push_back(std::move(l));
        CHECK(cache.consistent());
    }
    while (!inflight.empty())
        complete(0);
    CHECK(cache.hits() + cache.misses() == requests);
    for (int s = 0; s < slots; ++s)
        CHECK(sh.touching[s] == 0);
    if (expect_hits)
        CHECK(cache.hits() > requests * 8 / 10);
    std::printf("slots %d pool %d: %llu requests, %llu hits, %llu misses, %llu installs, %llu evictions\n", slots,
                pool_size, static_cast<unsigned long long>(requests), static_cast<unsigned long long>(cache.hits()),
                static_cast<unsigned long long>(cache.misses()), static_cast<unsigned long long>(cache.installs()),
                static_cast<unsigned long long>(cache.evictions()));
}

int main()
{
    // Hand-checked sequence: one slot.
    {
        std::mt19937_64 g(1);
        Key a = make_key(g, false), b = make_key(g, true);
        KeyCache c(1);
        KeyCache::Ref r1 = c.acquire(a.rk, a.nr);       // miss, install into slot 0
        CHECK(r1.install && r1.slot == 0 && !r1.resident);
        KeyCache::Ref r2 = c.acquire(a.rk, a.nr);       // same key, install in flight
        CHECK(!r2.install && !r2.resident && r2.slot < 0 && r2.pending == 0);
        KeyCache::Ref r3 = c.acquire(b.rk, b.nr);       // no free slot: inline only
        CHECK(r3.slot < 0 && !r3.install && r3.pending < 0);
        c.release(r1, true);
        KeyCache::Ref r4 = c.acquire(a.rk, a.nr);       // now resident
        CHECK(r4.resident && r4.slot == 0);
        KeyCache::Ref r5 = c.acquire(b.rk, b.nr);       // slot 0 is read in flight: no eviction
        CHECK(r5.slot < 0);
        c.release(r4, true);
        KeyCache::Ref r6 = c.acquire(b.rk, b.nr);       // evicts a
        CHECK(r6.install && r6.slot == 0 && c.evictions() == 1);
        c.release(r6, false);                           // failed install: slot free again
        KeyCache::Ref r7 = c.acquire(b.rk, b.nr);
        CHECK(r7.install && r7.slot == 0);
        c.release(r7, true);
        KeyCache::Ref r8 = c.acquire(a.rk, a.nr);       // a was evicted
        CHECK(r8.install);
        c.release(r8, true);
        CHECK(c.consistent());
        CHECK(c.hits() == 1 && c.misses() == 7);
    }
    // Two schedules with the same cipher key words (the hash) that differ in
    // a later round key are different keys: neither may hit the other's slot.
    {
        std::mt19937_64 g(3);
        Key a = make_key(g, false);
        Key t = a;
        t.rk[37] ^= 1u;
        KeyCache c(2);
        KeyCache::Ref r1 = c.acquire(a.rk, a.nr);
        CHECK(r1.install && r1.slot >= 0);
        c.release(r1, true);
        KeyCache::Ref r2 = c.acquire(t.rk, t.nr);       // same hash, other schedule
        CHECK(!r2.resident && !r2.install && r2.slot < 0 && r2.pending < 0);
        KeyCache::Ref r3 = c.acquire(a.rk, a.nr);
        CHECK(r3.resident && r3.slot == r1.slot);
        c.release(r3, true);
        CHECK(c.consistent());
    }
    // Zero slots: every request inline, nothing counted.
    {
        std::mt19937_64 g(2);
        Key a = make_key(g, false);
        KeyCache c(0);
        KeyCache::Ref r = c.acquire(a.rk, a.nr);
        CHECK(r.slot < 0 && !r.resident && !r.install && c.hits() == 0 && c.misses() == 0);
    }
    run(64, 64, 20000, 11, 0.0, true);     // every key fits: nearly all hits
    run(64, 48, 20000, 12, 0.02, true);    // with failed launches
    run(64, 256, 20000, 13, 0.0, false);   // pool larger than the table: LRU churn
    run(4, 16, 20000, 14, 0.05, false);    // tiny table, most slots busy
    run(1024, 100000, 5000, 15, 0.0, false);
    std::printf("key cache ok\n");
    return 0;
}
