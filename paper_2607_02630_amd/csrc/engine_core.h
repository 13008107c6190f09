// engine_core.h -- host-side scheduling state of the serving engine.
//
// Pure C++ (no HIP), so it can be exercised on the CPU by itself.  It holds
// the FIFO of submitted requests, admits them into launches while the bytes
// in flight stay within the budget, keeps the ticket table, and records
// submit-to-completion latencies.  The HIP driver (engine.cpp) calls
// take_batch() whenever a stream is free and complete() when a launch's event
// has fired; callers use submit/poll/wait from any thread.
//
// Shape of the paper's reroute (Sec. 3, Listing 1): submit hands the job to
// the executor and returns at once; the ticket exists before the work can
// complete, so a completion can never race the caller's suspension; resume
// happens when poll/wait observes the completion.
//
// Concurrency.  Submitting threads never take a lock: the FIFO is a bounded
// ring of sequence-numbered cells (a producer claims a position with one
// compare-exchange, writes its request, then publishes the cell), and a
// ticket is its ring position + 1.  A ticket's state lives in a ring of
// atomic words, (ticket << 16) | code, so poll() is a load and, for a
// finished ticket, one compare-exchange that retires it.  The driver is the
// only consumer: take_batch, complete, cancel_queued and wait_for_work run on
// one thread at a time.  Counters and latency samples sit behind a mutex the
// driver takes once per batch; complete() updates them before it publishes
// the tickets' states, so a caller that has seen its ticket finish also sees
// it counted.  Sleeping is the exception, not the rule: the driver sleeps on
// a condition variable only when the ring is empty and nothing is in flight,
// and a submitter signals it only if it is asleep; a waiter spins briefly and
// then blocks, and complete() signals only when a waiter is blocked.  Both
// hand-offs pair a sequentially consistent store of one side's flag with a
// sequentially consistent load of the other side's, so a wake-up cannot be
// lost.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <stdint.h>
#include <string.h>
#include <thread>
#include <vector>

#include "../../include/aesctr.h"

namespace aesctr {

template <class Record>
struct EngineReq {
    uint64_t ticket = 0;
    uint64_t bytes = 0;        // admission weight: bytes the request holds in flight
    uint64_t payload = 0;      // payload bytes, counted against the per-launch cap
    int64_t t_submit_ns = 0;
    Record rec{};
};

template <class Record>
class EngineCore {
public:
    using Req = EngineReq<Record>;
    // Queued (not yet admitted) requests; a full ring makes submit wait.
    static constexpr uint64_t kQueueCap = 1u << 15;
    // Ticket states kept; a finished ticket that is never polled is
    // forgotten once this many later tickets have been issued.
    static constexpr uint64_t kTicketCap = 1u << 20;

    EngineCore(uint64_t budget, size_t max_batch_reqs, uint64_t max_batch_bytes)
        : budget_(budget), max_reqs_(max_batch_reqs), max_bytes_(max_batch_bytes),
          ring_(new Cell[kQueueCap]), state_(new std::atomic<uint64_t>[kTicketCap])
    {
        for (uint64_t i = 0; i < kQueueCap; ++i)
            ring_[i].seq.store(i, std::memory_order_relaxed);
        for (uint64_t i = 0; i < kTicketCap; ++i)
            state_[i].store(0, std::memory_order_relaxed);
        lat_us_.reserve(1 << 16);
    }

    static int64_t now_ns()
    {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(
                   std::chrono::steady_clock::now().time_since_epoch())
            .count();
    }

    void set_on_complete(std::function<void()> f) { on_complete_ = std::move(f); }

    // Caller threads ------------------------------------------------------

    // t_arrival_ns < 0: the request arrives now.  Waits (yielding) while the
    // ring holds kQueueCap queued requests.
    int submit(Req &&r, uint64_t *ticket, int64_t t_arrival_ns = -1)
    {
        producers_.fetch_add(1, std::memory_order_seq_cst);
        const int rc = submit_inner(std::move(r), ticket, t_arrival_ns);
        producers_.fetch_sub(1, std::memory_order_seq_cst);
        if (rc == AES_OK && driver_sleeping_.load(std::memory_order_seq_cst)) {
            std::lock_guard<std::mutex> lk(work_mu_);
            work_cv_.notify_one();
        }
        return rc;
    }

    int poll(uint64_t t)
    {
        if (t == 0)
            return AES_ENOTFOUND;
        std::atomic<uint64_t> &sw = state_[t & (kTicketCap - 1)];
        uint64_t w = sw.load(std::memory_order_acquire);
        if ((w >> 16) != t)
            return AES_ENOTFOUND;
        const uint32_t code = static_cast<uint32_t>(w & 0xffff);
        if (code == kPending)
            return 0;
        if (code == kRetired)
            return AES_ENOTFOUND;
        if (!sw.compare_exchange_strong(w, (t << 16) | kRetired, std::memory_order_acq_rel))
            return AES_ENOTFOUND;       // another thread retired it first
        return code == kOk ? 1 : -static_cast<int>(code - kErrBase);
    }

    int wait(uint64_t t, int64_t timeout_us)
    {
        auto done = [&] {
            const uint64_t w = state_[t & (kTicketCap - 1)].load(std::memory_order_seq_cst);
            return (w >> 16) != t || (w & 0xffff) != kPending;
        };
        // Completions arrive every few tens of microseconds under load: spin
        // a little before blocking.
        const int64_t spin_until = now_ns() + 20000;
        bool ok = done();
        while (!ok && now_ns() < spin_until) {
            std::this_thread::yield();
            ok = done();
        }
        if (!ok) {
            waiters_.fetch_add(1, std::memory_order_seq_cst);
            {
                std::unique_lock<std::mutex> lk(wait_mu_);
                if (timeout_us < 0)
                    done_cv_.wait(lk, done);
                else
                    ok = done_cv_.wait_for(lk, std::chrono::microseconds(timeout_us), done);
            }
            waiters_.fetch_sub(1, std::memory_order_seq_cst);
            if (timeout_us >= 0 && !ok)
                return AES_ETIMEDOUT;
        }
        const int rc = poll(t);
        return rc == 1 ? AES_OK : rc;
    }

    void stats(aes_stats_t *o)
    {
        std::vector<float> v;
        {
            std::lock_guard<std::mutex> lk(stats_mu_);
            memset(o, 0, sizeof(*o));
            const uint64_t enq = enq_.load(std::memory_order_acquire);
            const uint64_t deq = deq_.load(std::memory_order_acquire);
            o->submitted = enq - submitted_base_;
            o->completed = completed_;
            o->rejected = rejected_.load(std::memory_order_relaxed);
            o->batches = batches_;
            o->bytes_completed = bytes_completed_;
            o->budget_high_water = high_water_;
            o->queued_now = enq - deq;
            o->inflight_now = inflight_reqs_.load(std::memory_order_acquire);
            o->mean_batch_reqs = batches_ ? static_cast<double>(batched_reqs_) / batches_ : 0.0;
            o->busy_s = busy_ns_ * 1e-9;
            v = lat_us_;
        }
        if (!v.empty()) {
            std::sort(v.begin(), v.end());
            auto pct = [&](double p) {
                size_t i = static_cast<size_t>(p * (v.size() - 1) + 0.5);
                return static_cast<double>(v[std::min(i, v.size() - 1)]);
            };
            o->p50_us = pct(0.50);
            o->p99_us = pct(0.99);
            o->p999_us = pct(0.999);
            o->max_us = v.back();
        }
    }

    void reset_stats()
    {
        std::lock_guard<std::mutex> lk(stats_mu_);
        submitted_base_ = enq_.load(std::memory_order_acquire);
        completed_ = batches_ = batched_reqs_ = bytes_completed_ = 0;
        rejected_.store(0, std::memory_order_relaxed);
        high_water_ = inflight_bytes_.load(std::memory_order_acquire);
        busy_ns_ = 0;
        lat_us_.clear();
    }

    // Driver thread -------------------------------------------------------

    // Move the longest FIFO prefix that fits the budget (and the per-launch
    // limits: requests, and payload bytes) into `out`.  A head that does not
    // fit blocks the ones behind it, so no request is overtaken forever.
    bool take_batch(std::vector<Req> &out)
    {
        out.clear();
        uint64_t batch_payload = 0;
        uint64_t inflight = inflight_bytes_.load(std::memory_order_relaxed);
        uint64_t deq = deq_.load(std::memory_order_relaxed);
        while (out.size() < max_reqs_) {
            Cell &c = ring_[deq & (kQueueCap - 1)];
            if (c.seq.load(std::memory_order_acquire) != deq + 1)
                break;                                  // empty, or not yet published
            const uint64_t b = c.req.bytes;
            if (inflight + b > budget_)
                break;
            if (!out.empty() && batch_payload + c.req.payload > max_bytes_)
                break;
            inflight += b;
            batch_payload += c.req.payload;
            out.push_back(std::move(c.req));
            c.seq.store(deq + kQueueCap, std::memory_order_release);   // free for a producer
            ++deq;
        }
        if (out.empty())
            return false;
        inflight_bytes_.store(inflight, std::memory_order_release);
        inflight_reqs_.fetch_add(out.size(), std::memory_order_acq_rel);
        deq_.store(deq, std::memory_order_release);
        std::lock_guard<std::mutex> lk(stats_mu_);
        high_water_ = std::max(high_water_, inflight);
        ++batches_;
        batched_reqs_ += out.size();
        return true;
    }

    void complete(const std::vector<Req> &batch, int status, int64_t now)
    {
        uint64_t bytes = 0, payload = 0;
        for (const Req &r : batch) {
            bytes += r.bytes;
            payload += r.payload;
        }
        {
            std::lock_guard<std::mutex> lk(stats_mu_);
            if (status == AES_OK) {
                completed_ += batch.size();
                bytes_completed_ += payload;
                for (const Req &r : batch)
                    if (lat_us_.size() < kMaxSamples)
                        lat_us_.push_back(static_cast<float>((now - r.t_submit_ns) * 1e-3));
            }
        }
        inflight_bytes_.fetch_sub(bytes, std::memory_order_acq_rel);
        inflight_reqs_.fetch_sub(batch.size(), std::memory_order_acq_rel);
        const uint64_t code = status == AES_OK ? kOk : kErrBase + static_cast<uint64_t>(-status);
        for (const Req &r : batch)
            state_[r.ticket & (kTicketCap - 1)].store((r.ticket << 16) | code, std::memory_order_seq_cst);
        if (waiters_.load(std::memory_order_seq_cst) > 0) {
            std::lock_guard<std::mutex> lk(wait_mu_);
            done_cv_.notify_all();
        }
        if (on_complete_)
            on_complete_();
    }

    void add_busy(int64_t ns)
    {
        std::lock_guard<std::mutex> lk(stats_mu_);
        busy_ns_ += ns;
    }

    // Sleep until there is queued work, the engine closes, or the timeout.
    void wait_for_work(int64_t timeout_ns)
    {
        std::unique_lock<std::mutex> lk(work_mu_);
        driver_sleeping_.store(true, std::memory_order_seq_cst);
        work_cv_.wait_for(lk, std::chrono::nanoseconds(timeout_ns),
                          [&] { return head_published() || closing_.load(std::memory_order_seq_cst); });
        driver_sleeping_.store(false, std::memory_order_seq_cst);
    }

    void close()
    {
        closing_.store(true, std::memory_order_seq_cst);
        std::lock_guard<std::mutex> lk(work_mu_);
        work_cv_.notify_all();
    }

    bool closing_and_drained()
    {
        return closing_.load(std::memory_order_seq_cst) && producers_.load(std::memory_order_seq_cst) == 0 &&
               enq_.load(std::memory_order_acquire) == deq_.load(std::memory_order_relaxed) &&
               inflight_reqs_.load(std::memory_order_acquire) == 0;
    }

    // Fail every queued request (used when the device cannot be driven).
    // After close() this also waits out submissions already under way, so
    // none is left behind.
    void cancel_queued(int status)
    {
        std::vector<Req> dropped;
        for (;;) {
            uint64_t deq = deq_.load(std::memory_order_relaxed);
            for (;;) {
                Cell &c = ring_[deq & (kQueueCap - 1)];
                if (c.seq.load(std::memory_order_acquire) != deq + 1)
                    break;
                dropped.push_back(std::move(c.req));
                c.seq.store(deq + kQueueCap, std::memory_order_release);
                ++deq;
            }
            deq_.store(deq, std::memory_order_release);
            if (!closing_.load(std::memory_order_seq_cst) ||
                (producers_.load(std::memory_order_seq_cst) == 0 && enq_.load(std::memory_order_acquire) == deq))
                break;
            std::this_thread::yield();
        }
        if (dropped.empty())
            return;
        uint64_t bytes = 0;
        for (const Req &r : dropped)
            bytes += r.bytes;
        inflight_bytes_.fetch_add(bytes, std::memory_order_acq_rel);        // complete() subtracts them
        inflight_reqs_.fetch_add(dropped.size(), std::memory_order_acq_rel);
        complete(dropped, status, now_ns());
    }

private:
    static constexpr uint64_t kRetired = 0, kPending = 1, kOk = 2, kErrBase = 0x100;
    static constexpr size_t kMaxSamples = 4u << 20;

    struct Cell {
        std::atomic<uint64_t> seq;
        Req req;
    };

    int submit_inner(Req &&r, uint64_t *ticket, int64_t t_arrival_ns)
    {
        if (closing_.load(std::memory_order_seq_cst))
            return AES_ECLOSED;
        if (r.bytes > budget_) {
            rejected_.fetch_add(1, std::memory_order_relaxed);
            return AES_EAGAIN;
        }
        // Claim a ring position.
        uint64_t pos = enq_.load(std::memory_order_relaxed);
        Cell *c;
        for (;;) {
            c = &ring_[pos & (kQueueCap - 1)];
            const uint64_t seq = c->seq.load(std::memory_order_acquire);
            const int64_t dif = static_cast<int64_t>(seq - pos);
            if (dif == 0) {
                if (enq_.compare_exchange_weak(pos, pos + 1, std::memory_order_acq_rel))
                    break;
            } else if (dif < 0) {                 // full: the driver has not taken this cell yet
                if (closing_.load(std::memory_order_seq_cst))
                    return AES_ECLOSED;
                std::this_thread::yield();
                pos = enq_.load(std::memory_order_relaxed);
            } else {
                pos = enq_.load(std::memory_order_relaxed);
            }
        }
        const uint64_t t = pos + 1;
        // The ticket's state word: its previous user (kTicketCap tickets ago)
        // must have finished; with a 2^15-entry ring and bounded batches it
        // has, unless the budget admits more than 2^20 requests at once.
        std::atomic<uint64_t> &sw = state_[t & (kTicketCap - 1)];
        while ((sw.load(std::memory_order_acquire) & 0xffff) == kPending)
            std::this_thread::yield();
        sw.store((t << 16) | kPending, std::memory_order_release);   // registered before it can complete
        r.ticket = t;
        r.t_submit_ns = t_arrival_ns >= 0 ? t_arrival_ns : now_ns();
        *ticket = t;
        c->req = std::move(r);
        c->seq.store(pos + 1, std::memory_order_seq_cst);              // publish
        return AES_OK;
    }

    bool head_published()
    {
        const uint64_t deq = deq_.load(std::memory_order_relaxed);
        return ring_[deq & (kQueueCap - 1)].seq.load(std::memory_order_seq_cst) == deq + 1;
    }

    const uint64_t budget_;
    const size_t max_reqs_;
    const uint64_t max_bytes_;
    std::unique_ptr<Cell[]> ring_;
    std::unique_ptr<std::atomic<uint64_t>[]> state_;
    std::function<void()> on_complete_;

    alignas(64) std::atomic<uint64_t> enq_{0};            // next position a producer claims
    alignas(64) std::atomic<uint64_t> deq_{0};            // next position the driver takes
    alignas(64) std::atomic<int> producers_{0};
    std::atomic<uint64_t> rejected_{0};
    alignas(64) std::atomic<uint64_t> inflight_bytes_{0}, inflight_reqs_{0};
    std::atomic<bool> closing_{false}, driver_sleeping_{false};
    std::atomic<int> waiters_{0};

    std::mutex work_mu_, wait_mu_;
    std::condition_variable work_cv_, done_cv_;

    std::mutex stats_mu_;
    uint64_t submitted_base_ = 0, high_water_ = 0;
    uint64_t completed_ = 0, batches_ = 0, batched_reqs_ = 0, bytes_completed_ = 0;
    int64_t busy_ns_ = 0;
    std::vector<float> lat_us_;
};

}  // namespace aesctr
