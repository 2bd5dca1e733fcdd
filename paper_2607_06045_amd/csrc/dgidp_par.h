// Host-side parallel loops for the mesh builders: a small pool of worker
// threads, started on first use and kept until the process ends, that runs
// the chunks of one loop at a time.  The calling thread takes chunks too (so a
// loop also completes when no worker is scheduled).  A call made while another
// one runs (another thread adapting another context) runs serially.  Results
// must not depend on the chunking: the loops given here write disjoint entries
// or reduce with order-free operations.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

namespace dgidp {

class HostPool {
public:
    static HostPool& get()
    {
        static HostPool pool;
        return pool;
    }

    int threads() const { return (int)workers_.size() + 1; }

    // fn(lo, hi) over [0, n) in chunks of at least `grain` items
    void run(int64_t n, const std::function<void(int64_t, int64_t)>& fn, int64_t grain = 8192)
    {
        if (n <= 0) return;
        const int64_t want = std::min<int64_t>(threads(), (n + grain - 1) / grain);
        std::unique_lock<std::mutex> busy(run_lock_, std::try_to_lock);
        if (want <= 1 || !busy.owns_lock()) {
            fn(0, n);
            return;
        }
        auto job = std::make_shared<Job>();
        job->fn = &fn;
        job->n = n;
        job->nch = want * 4;  // a few chunks per thread for balance
        {
            std::lock_guard<std::mutex> g(m_);
            job_ = job;
            ++gen_;
        }
        cv_.notify_all();
        job->work();
        std::unique_lock<std::mutex> g(job->m);
        job->cv.wait(g, [&] { return job->done == job->nch; });
    }

private:
    // one loop: its chunks are taken through an atomic counter; a worker that
    // picks up a job after it finished finds no chunk left
    struct Job {
        const std::function<void(int64_t, int64_t)>* fn = nullptr;
        int64_t n = 0, nch = 0;
        std::atomic<int64_t> next{0};
        std::mutex m;
        std::condition_variable cv;
        int64_t done = 0;
        void work()
        {
            for (;;) {
                const int64_t c = next.fetch_add(1);
                if (c >= nch) return;
                const int64_t lo = n * c / nch, hi = n * (c + 1) / nch;
                if (lo < hi) (*fn)(lo, hi);
                std::lock_guard<std::mutex> g(m);
                if (++done == nch) cv.notify_all();
            }
        }
    };

    HostPool()
    {
        const unsigned hw = std::thread::hardware_concurrency();
        const int nt = (int)std::min<unsigned>(hw ? hw : 1, 16) - 1;
        for (int t = 0; t < nt; ++t) workers_.emplace_back([this] { loop(); });
    }
    ~HostPool()
    {
        {
            std::lock_guard<std::mutex> g(m_);
            stop_ = true;
            ++gen_;
        }
        cv_.notify_all();
        for (auto& w : workers_) w.join();
    }

    void loop()
    {
        uint64_t seen = 0;
        for (;;) {
            std::shared_ptr<Job> job;
            {
                std::unique_lock<std::mutex> g(m_);
                cv_.wait(g, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                job = job_;
            }
            if (job) job->work();
        }
    }

    std::vector<std::thread> workers_;
    std::mutex run_lock_;  // one loop at a time
    std::mutex m_;
    std::condition_variable cv_;
    std::shared_ptr<Job> job_;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

// fn(lo, hi) over [0, n) on the pool
inline void par_for(int64_t n, const std::function<void(int64_t, int64_t)>& fn, int64_t grain = 8192)
{
    HostPool::get().run(n, fn, grain);
}

// sort v (distinct keys) on the pool: chunks sorted in parallel, then merged
// pairwise; with distinct keys the result is the serial std::sort's
template <class T>
void par_sort(std::vector<T>& v, int64_t grain = 16384)
{
    const int64_t n = (int64_t)v.size();
    const int64_t nch = std::min<int64_t>(HostPool::get().threads(), (n + grain - 1) / grain);
    if (nch <= 1) {
        std::sort(v.begin(), v.end());
        return;
    }
    const int64_t w0 = (n + nch - 1) / nch;
    par_for(nch, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c)
            std::sort(v.begin() + std::min(n, c * w0), v.begin() + std::min(n, (c + 1) * w0));
    }, 1);
    for (int64_t w = w0; w < n; w *= 2) {
        const int64_t pairs = (n + 2 * w - 1) / (2 * w);
        par_for(pairs, [&](int64_t p0, int64_t p1) {
            for (int64_t pr = p0; pr < p1; ++pr) {
                const int64_t lo = pr * 2 * w, mid = std::min(n, lo + w), hi = std::min(n, lo + 2 * w);
                if (mid < hi) std::inplace_merge(v.begin() + lo, v.begin() + mid, v.begin() + hi);
            }
        }, 1);
    }
}

}  // namespace dgidp
