// A small pool of host threads for per-system host work of a batch (pair
// updates of independent systems): run(n, f) calls f(0) .. f(n-1) over the
// workers and the calling thread and returns when all calls have finished.
// One caller at a time (a context is used by one thread).
#pragma once
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

struct WorkPool {
    explicit WorkPool(unsigned workers) {
        for (unsigned i = 0; i < workers; ++i) th_.emplace_back([this] { loop(); });
    }
    ~WorkPool() {
        {
            std::lock_guard<std::mutex> g(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    WorkPool(const WorkPool&) = delete;
    WorkPool& operator=(const WorkPool&) = delete;

    void run(unsigned n, const std::function<void(unsigned)>& f) {
        if (n == 0) return;
        if (th_.empty() || n == 1) {
            for (unsigned i = 0; i < n; ++i) f(i);
            return;
        }
        {
            std::lock_guard<std::mutex> g(m_);
            job_ = &f;
            n_ = n;
            next_.store(0);
            finished_ = 0;
            ++gen_;
        }
        cv_.notify_all();
        work();
        std::unique_lock<std::mutex> g(m_);
        done_cv_.wait(g, [this] { return finished_ == n_; });
        job_ = nullptr;
    }

private:
    // take jobs until none is left
    void work() {
        for (;;) {
            const unsigned i = next_.fetch_add(1);
            if (i >= n_) return;
            (*job_)(i);
            std::lock_guard<std::mutex> g(m_);
            if (++finished_ == n_) done_cv_.notify_all();
        }
    }
    void loop() {
        unsigned long long seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> g(m_);
                cv_.wait(g, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
            }
            work();
        }
    }

    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(unsigned)>* job_ = nullptr;
    unsigned n_ = 0, finished_ = 0;
    std::atomic<unsigned> next_{0};
    unsigned long long gen_ = 0;
    bool stop_ = false;
};
