// host_pool.h -- a small persistent pool of host threads for the per-call
// descriptor work of large batches (validation, building and staging device
// records).  That work is memory-bound and sits before the first launch of a
// call, so a few threads shorten the time to the first kernel.
#pragma once

#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <stddef.h>
#include <thread>
#include <vector>

namespace aesctr {

class HostPool {
public:
    // fn(part, begin, end) for the parts of [0, n).
    using PartFn = std::function<void(size_t, size_t, size_t)>;

    // The process-wide pool (created on first use, never destroyed: its
    // threads sleep until the process ends).
    static HostPool &get();

    // Number of parts parallel_for cuts n items into: about n / grain,
    // between 1 and kMaxParts.  Part p is [min(n, p * per), min(n, (p + 1) *
    // per)) with per = ceil(n / parts): contiguous, in index order, and
    // possibly empty at the end.
    static size_t parts(size_t n, size_t grain);

    // Runs fn over every part of [0, n) (as parts(n, grain) defines them) and
    // returns when all have run.  The calling thread takes parts too; when
    // another call holds the pool, or there is a single part, every part
    // runs on the calling thread.  fn must not throw.
    void parallel_for(size_t n, size_t grain, const PartFn &fn);

    static constexpr size_t kMaxParts = 64;
    static constexpr int kMaxWorkers = 4;

private:
    struct Job {
        const PartFn *fn;
        size_t n, parts, per;
        std::atomic<size_t> next{0};
    };

    HostPool() = default;
    void start();
    void worker();
    static size_t run_parts(Job *j);

    std::mutex call_mu_;            // one parallel_for at a time
    std::mutex mu_;                 // guards everything below
    std::condition_variable work_cv_, done_cv_;
    std::vector<std::thread> threads_;
    bool started_ = false;
    Job *job_ = nullptr;
    uint64_t gen_ = 0;              // bumped for every job
    int users_ = 0;                 // workers holding job_
    size_t done_parts_ = 0;
};

}  // namespace aesctr
