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
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <stdint.h>
#include <string.h>
#include <unordered_map>
#include <vector>

#include "../../include/aesctr.h"

namespace aesctr {

template <class Record>
struct EngineReq {
    uint64_t ticket = 0;
    uint64_t bytes = 0;        // admission weight: payload bytes
    int64_t t_submit_ns = 0;
    Record rec{};
};

template <class Record>
class EngineCore {
public:
    using Req = EngineReq<Record>;
    static constexpr int kPending = 1;

    EngineCore(uint64_t budget, size_t max_batch_reqs, uint64_t max_batch_bytes)
        : budget_(budget), max_reqs_(max_batch_reqs), max_bytes_(max_batch_bytes)
    {
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

    // t_arrival_ns < 0: the request arrives now.
    int submit(Req &&r, uint64_t *ticket, int64_t t_arrival_ns = -1)
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (closing_)
            return AES_ECLOSED;
        if (r.bytes > budget_) {
            ++rejected_;
            return AES_EAGAIN;
        }
        r.ticket = ++last_ticket_;
        r.t_submit_ns = t_arrival_ns >= 0 ? t_arrival_ns : now_ns();
        status_[r.ticket] = kPending;      // registered before it can complete
        *ticket = r.ticket;
        queue_.push_back(std::move(r));
        ++submitted_;
        work_cv_.notify_one();
        return AES_OK;
    }

    int poll(uint64_t t)
    {
        std::lock_guard<std::mutex> lk(mu_);
        return poll_locked(t);
    }

    int wait(uint64_t t, int64_t timeout_us)
    {
        std::unique_lock<std::mutex> lk(mu_);
        auto done = [&] {
            auto it = status_.find(t);
            return it == status_.end() || it->second != kPending;
        };
        if (timeout_us < 0) {
            done_cv_.wait(lk, done);
        } else if (!done_cv_.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
            return AES_ETIMEDOUT;
        }
        int rc = poll_locked(t);
        return rc == 1 ? AES_OK : rc;
    }

    void stats(aes_stats_t *o)
    {
        std::vector<float> v;
        {
            std::lock_guard<std::mutex> lk(mu_);
            memset(o, 0, sizeof(*o));
            o->submitted = submitted_;
            o->completed = completed_;
            o->rejected = rejected_;
            o->batches = batches_;
            o->bytes_completed = bytes_completed_;
            o->budget_high_water = high_water_;
            o->queued_now = queue_.size();
            o->inflight_now = inflight_reqs_;
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
        }
    }

    void reset_stats()
    {
        std::lock_guard<std::mutex> lk(mu_);
        submitted_ = completed_ = rejected_ = batches_ = batched_reqs_ = bytes_completed_ = 0;
        high_water_ = inflight_bytes_;
        busy_ns_ = 0;
        lat_us_.clear();
    }

    // Driver thread -------------------------------------------------------

    // Move the longest FIFO prefix that fits the budget (and the per-launch
    // limits) into `out`.  A head that does not fit blocks the ones behind it,
    // so no request is overtaken forever.
    bool take_batch(std::vector<Req> &out)
    {
        out.clear();
        std::lock_guard<std::mutex> lk(mu_);
        uint64_t batch_bytes = 0;
        while (!queue_.empty() && out.size() < max_reqs_) {
            Req &h = queue_.front();
            if (inflight_bytes_ + h.bytes > budget_)
                break;
            if (!out.empty() && batch_bytes + h.bytes > max_bytes_)
                break;
            inflight_bytes_ += h.bytes;
            batch_bytes += h.bytes;
            out.push_back(std::move(h));
            queue_.pop_front();
        }
        if (out.empty())
            return false;
        high_water_ = std::max(high_water_, inflight_bytes_);
        inflight_reqs_ += out.size();
        ++batches_;
        batched_reqs_ += out.size();
        return true;
    }

    void complete(const std::vector<Req> &batch, int status, int64_t now)
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (const Req &r : batch) {
                inflight_bytes_ -= r.bytes;
                auto it = status_.find(r.ticket);
                if (it != status_.end())
                    it->second = status;
                if (status == AES_OK) {
                    ++completed_;
                    bytes_completed_ += r.bytes;
                    if (lat_us_.size() < kMaxSamples)
                        lat_us_.push_back(static_cast<float>((now - r.t_submit_ns) * 1e-3));
                }
            }
            inflight_reqs_ -= batch.size();
        }
        done_cv_.notify_all();
        if (on_complete_)
            on_complete_();
    }

    void add_busy(int64_t ns)
    {
        std::lock_guard<std::mutex> lk(mu_);
        busy_ns_ += ns;
    }

    // Sleep until there is queued work, the engine closes, or the timeout.
    void wait_for_work(int64_t timeout_ns)
    {
        std::unique_lock<std::mutex> lk(mu_);
        work_cv_.wait_for(lk, std::chrono::nanoseconds(timeout_ns), [&] { return !queue_.empty() || closing_; });
    }

    void close()
    {
        std::lock_guard<std::mutex> lk(mu_);
        closing_ = true;
        work_cv_.notify_all();
    }

    bool closing_and_drained()
    {
        std::lock_guard<std::mutex> lk(mu_);
        return closing_ && queue_.empty() && inflight_reqs_ == 0;
    }

    // Fail every queued request (used when the device cannot be driven).
    void cancel_queued(int status)
    {
        std::vector<Req> dropped;
        {
            std::lock_guard<std::mutex> lk(mu_);
            while (!queue_.empty()) {
                dropped.push_back(std::move(queue_.front()));
                queue_.pop_front();
            }
            for (Req &r : dropped)
                inflight_bytes_ += r.bytes;     // complete() subtracts it again
            inflight_reqs_ += dropped.size();
        }
        if (!dropped.empty())
            complete(dropped, status, now_ns());
    }

private:
    int poll_locked(uint64_t t)
    {
        auto it = status_.find(t);
        if (it == status_.end())
            return AES_ENOTFOUND;
        if (it->second == kPending)
            return 0;
        int st = it->second;
        status_.erase(it);
        return st == AES_OK ? 1 : st;
    }

    static constexpr size_t kMaxSamples = 4u << 20;

    std::mutex mu_;
    std::condition_variable work_cv_, done_cv_;
    std::deque<Req> queue_;
    std::unordered_map<uint64_t, int> status_;
    std::function<void()> on_complete_;
    const uint64_t budget_;
    const size_t max_reqs_;
    const uint64_t max_bytes_;
    uint64_t last_ticket_ = 0;
    uint64_t inflight_bytes_ = 0, inflight_reqs_ = 0, high_water_ = 0;
    uint64_t submitted_ = 0, completed_ = 0, rejected_ = 0, batches_ = 0, batched_reqs_ = 0;
    uint64_t bytes_completed_ = 0;
    int64_t busy_ns_ = 0;
    bool closing_ = false;
    std::vector<float> lat_us_;
};

}  // namespace aesctr
