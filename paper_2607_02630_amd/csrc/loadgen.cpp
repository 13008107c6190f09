// loadgen.cpp -- open-loop load generation against the serving engine and
// against the synchronous per-request path (see include/aesloadgen.h).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <hip/hip_runtime.h>
#include <thread>
#include <vector>

#include "../../include/aesloadgen.h"

namespace {

constexpr size_t kSubmitters = 4;

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

void spin_until(int64_t t)
{
    while (now_ns() < t) {
    }
}

void fill_percentiles(std::vector<double> &lat, aes_load_result_t *o)
{
    if (lat.empty())
        return;
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) {
        size_t i = static_cast<size_t>(p * (lat.size() - 1) + 0.5);
        return lat[std::min(i, lat.size() - 1)];
    };
    o->p50_us = pct(0.50);
    o->p99_us = pct(0.99);
    o->p999_us = pct(0.999);
    o->max_us = lat.back();
}

}  // namespace

extern "C" int aes_load_engine(aes_engine_t *e, const aes_ctr_desc_t *pool, size_t npool, const double *arrival_s,
                               size_t n, aes_load_result_t *out)
{
    if (!e || !pool || !npool || (!arrival_s && n) || !out)
        return AES_EINVAL;
    *out = aes_load_result_t{};
    aes_engine_reset_stats(e);
    // Several submitter threads share the schedule (thread k takes arrivals
    // k, k + T, ...), so the offered rate is not capped by one thread's
    // submission cost; a collector retires tickets in arrival order.
    const unsigned hw = std::thread::hardware_concurrency();
    const size_t nthreads = std::min<size_t>(kSubmitters, std::max<unsigned>(1, hw > 2 ? hw - 2 : 1));
    std::vector<uint64_t> tickets(n);
    std::vector<std::atomic<uint8_t>> state(n);        // 0 pending, 1 submitted, 2 failed
    for (auto &st : state)
        st.store(0, std::memory_order_relaxed);
    std::atomic<int> first_err{AES_OK};
    std::atomic<uint64_t> bytes{0};
    const int64_t t0 = now_ns() + 2000000;   // start 2 ms from now
    int64_t last_done = t0;
    uint64_t errors = 0;

    std::thread collector([&] {
        for (size_t i = 0; i < n; ++i) {
            uint8_t st;
            while ((st = state[i].load(std::memory_order_acquire)) == 0)
                std::this_thread::yield();
            if (st == 2) {
                ++errors;
                continue;
            }
            if (aes_wait(e, tickets[i], -1) != AES_OK)
                ++errors;
            last_done = now_ns();
        }
    });
    std::vector<double> lag(nthreads, 0.0);
    std::vector<std::thread> subs;
    for (size_t k = 0; k < nthreads; ++k) {
        subs.emplace_back([&, k] {
            for (size_t i = k; i < n; i += nthreads) {
                const int64_t t = t0 + static_cast<int64_t>(arrival_s[i] * 1e9);
                spin_until(t);
                lag[k] = std::max(lag[k], (now_ns() - t) * 1e-3);
                const aes_ctr_desc_t &d = pool[i % npool];
                int rc = first_err.load(std::memory_order_relaxed) == AES_OK ? aes_submit_at(e, &d, t, &tickets[i])
                                                                             : AES_ECANCELED;
                if (rc != AES_OK) {
                    int expect = AES_OK;
                    first_err.compare_exchange_strong(expect, rc);
                    state[i].store(2, std::memory_order_release);
                    continue;
                }
                bytes.fetch_add(d.len, std::memory_order_relaxed);
                state[i].store(1, std::memory_order_release);
            }
        });
    }
    for (auto &th : subs)
        th.join();
    collector.join();

    aes_stats_t st;
    aes_engine_stats(e, &st);
    out->wall_s = (last_done - t0) * 1e-9;
    out->completed = st.completed;
    out->errors = errors;
    out->achieved_rps = out->wall_s > 0 ? st.completed / out->wall_s : 0;
    out->gbps = out->wall_s > 0 ? bytes.load() / out->wall_s / 1e9 : 0;
    out->max_lag_us = *std::max_element(lag.begin(), lag.end());
    out->p50_us = st.p50_us;
    out->p99_us = st.p99_us;
    out->p999_us = st.p999_us;
    out->max_us = st.max_us;
    return first_err.load();
}

namespace {

// One request at a time: [H2D into dev_buf,] crypt, [D2H,] synchronise.
int run_sync(const aes_ctr_desc_t *pool, size_t npool, const double *arrival_s, size_t n, void *dev_buf,
             size_t dev_bytes, void *stream, aes_load_result_t *out)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<double> lat;
    lat.reserve(n);
    uint64_t bytes = 0;
    double max_lag = 0;
    const int64_t t0 = now_ns() + 2000000;
    int64_t last = t0;
    for (size_t i = 0; i < n; ++i) {
        const int64_t t = t0 + static_cast<int64_t>(arrival_s[i] * 1e9);
        spin_until(t);    // no-op once the server has fallen behind
        max_lag = std::max(max_lag, (now_ns() - t) * 1e-3);
        const aes_ctr_desc_t &d = pool[i % npool];
        int rc;
        if (dev_buf) {
            if (d.len > dev_bytes)
                return AES_EINVAL;
            if (hipMemcpyAsync(dev_buf, d.in, d.len, hipMemcpyHostToDevice, st) != hipSuccess) {
                (void)hipGetLastError();
                return AES_EDEVICE;
            }
            rc = aes_ctr_crypt(d.sched, d.nonce, d.ctr0, dev_buf, dev_buf, d.len, stream);
            if (rc == AES_OK && hipMemcpyAsync(d.out, dev_buf, d.len, hipMemcpyDeviceToHost, st) != hipSuccess) {
                (void)hipGetLastError();
                return AES_EDEVICE;
            }
        } else {
            rc = aes_ctr_crypt(d.sched, d.nonce, d.ctr0, d.in, d.out, d.len, stream);
        }
        if (rc != AES_OK)
            return rc;
        if (hipStreamSynchronize(st) != hipSuccess) {
            (void)hipGetLastError();
            return AES_EDEVICE;
        }
        last = now_ns();
        lat.push_back((last - t) * 1e-3);
        bytes += d.len;
    }
    out->wall_s = (last - t0) * 1e-9;
    out->completed = n;
    out->achieved_rps = out->wall_s > 0 ? n / out->wall_s : 0;
    out->gbps = out->wall_s > 0 ? bytes / out->wall_s / 1e9 : 0;
    out->max_lag_us = max_lag;
    fill_percentiles(lat, out);
    return AES_OK;
}

}  // namespace

extern "C" int aes_load_sync(const aes_ctr_desc_t *pool, size_t npool, const double *arrival_s, size_t n,
                             void *stream, aes_load_result_t *out)
{
    if (!pool || !npool || (!arrival_s && n) || !out)
        return AES_EINVAL;
    *out = aes_load_result_t{};
    return run_sync(pool, npool, arrival_s, n, nullptr, 0, stream, out);
}

extern "C" int aes_load_sync_host(const aes_ctr_desc_t *pool, size_t npool, const double *arrival_s, size_t n,
                                  void *dev_buf, size_t dev_bytes, void *stream, aes_load_result_t *out)
{
    if (!pool || !npool || (!arrival_s && n) || !out || !dev_buf)
        return AES_EINVAL;
    *out = aes_load_result_t{};
    return run_sync(pool, npool, arrival_s, n, dev_buf, dev_bytes, stream, out);
}
