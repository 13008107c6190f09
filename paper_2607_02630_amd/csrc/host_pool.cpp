// host_pool.cpp -- see host_pool.h.
#include "host_pool.h"

#include <algorithm>

namespace aesctr {

HostPool &HostPool::get()
{
    static HostPool *pool = new HostPool();
    return *pool;
}

size_t HostPool::parts(size_t n, size_t grain)
{
    if (grain == 0)
        grain = 1;
    const size_t p = n / grain;
    return p < 1 ? 1 : p > kMaxParts ? kMaxParts : p;
}

void HostPool::start()
{
    // Called with call_mu_ held.  No threads when the machine has one CPU.
    started_ = true;
    const unsigned hw = std::thread::hardware_concurrency();
    const int workers = std::min<int>(kMaxWorkers, hw > 1 ? static_cast<int>(hw) - 1 : 0);
    for (int i = 0; i < workers; ++i)
        threads_.emplace_back([this] { worker(); });
    for (std::thread &t : threads_)
        t.detach();
}

size_t HostPool::run_parts(Job *j)
{
    size_t did = 0;
    for (size_t p = j->next.fetch_add(1); p < j->parts; p = j->next.fetch_add(1)) {
        const size_t b = std::min(j->n, p * j->per);
        const size_t e = std::min(j->n, b + j->per);
        (*j->fn)(p, b, e);
        ++did;
    }
    return did;
}

void HostPool::worker()
{
    std::unique_lock<std::mutex> lk(mu_);
    uint64_t seen = 0;
    for (;;) {
        work_cv_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
        Job *j = job_;
        if (!j)
            continue;   // woke after that job was over
        ++users_;
        lk.unlock();
        const size_t did = run_parts(j);
        lk.lock();
        --users_;
        done_parts_ += did;
        if (done_parts_ == j->parts && users_ == 0)
            done_cv_.notify_all();
    }
}

void HostPool::parallel_for(size_t n, size_t grain, const PartFn &fn)
{
    if (n == 0)
        return;
    const size_t parts = HostPool::parts(n, grain);
    const size_t per = (n + parts - 1) / parts;
    std::unique_lock<std::mutex> call(call_mu_, std::try_to_lock);
    if (parts == 1 || !call.owns_lock()) {
        for (size_t p = 0; p < parts; ++p)
            fn(p, std::min(n, p * per), std::min(n, (p + 1) * per));
        return;
    }
    if (!started_)
        start();
    Job j;
    j.fn = &fn;
    j.n = n;
    j.parts = parts;
    j.per = per;
    {
        std::lock_guard<std::mutex> lk(mu_);
        job_ = &j;
        done_parts_ = 0;
        ++gen_;
    }
    work_cv_.notify_all();
    const size_t did = run_parts(&j);
    std::unique_lock<std::mutex> lk(mu_);
    done_parts_ += did;
    // Every part has run and no worker still holds the job: it may go.
    done_cv_.wait(lk, [&] { return done_parts_ == parts && users_ == 0; });
    job_ = nullptr;
}

}  // namespace aesctr
