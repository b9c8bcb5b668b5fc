// Host-side data parallelism for the symbolic phases (no device code).
#pragma once

#include <algorithm>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace vag {

namespace detail {

// A process-wide pool of worker threads, started at first use: a call of
// parallel_chunks costs a queue push per chunk instead of a thread start.
// Several host threads (serving workers) may submit at once; a submitter
// runs queued chunks itself while it waits for its own.
class ChunkPool {
public:
    static ChunkPool &get() {
        static ChunkPool p;
        return p;
    }
    int workers() const { return (int)th_.size(); }
    void push(std::function<void()> task) {
        {
            std::lock_guard<std::mutex> l(m_);
            q_.push_back(std::move(task));
        }
        cv_.notify_one();
    }
    // runs one queued task if there is one
    bool run_one() {
        std::function<void()> task;
        {
            std::lock_guard<std::mutex> l(m_);
            if (q_.empty()) return false;
            task = std::move(q_.front());
            q_.pop_front();
        }
        task();
        return true;
    }
    ~ChunkPool() {
        {
            std::lock_guard<std::mutex> l(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }

private:
    ChunkPool() {
        const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        for (unsigned k = 1; k < hw; ++k) th_.emplace_back([this] { loop(); });
    }
    void loop() {
        in_task() = true;
        for (;;) {
            std::function<void()> task;
            {
                std::unique_lock<std::mutex> l(m_);
                cv_.wait(l, [&] { return stop_ || !q_.empty(); });
                if (q_.empty()) return;  // stop
                task = std::move(q_.front());
                q_.pop_front();
            }
            task();
        }
    }

public:
    // true on pool threads: a chunk that calls parallel_chunks runs it alone
    static bool &in_task() {
        static thread_local bool t = false;
        return t;
    }

private:
    std::mutex m_;
    std::condition_variable cv_;
    std::deque<std::function<void()>> q_;
    std::vector<std::thread> th_;
    bool stop_ = false;
};

}  // namespace detail

// the number of chunks parallel_chunks uses for n items
inline int chunk_count(int64_t n, int64_t min_items = 32768) {
    const int64_t hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    return (int)std::max<int64_t>(1, std::min<int64_t>(hw, n / min_items));
}

// Runs f(t, begin, end) over [0, n) split into contiguous chunks (at most 16,
// at least min_items items each) on the pool; the first exception thrown by
// a chunk is rethrown.
template <class F>
void parallel_chunks(int64_t n, F &&f, int64_t min_items = 32768) {
    const int T = chunk_count(n, min_items);
    if (T == 1 || detail::ChunkPool::in_task()) {
        f(0, (int64_t)0, n);
        return;
    }
    detail::ChunkPool &pool = detail::ChunkPool::get();
    std::vector<std::exception_ptr> err(T);
    std::mutex m;
    std::condition_variable cv;
    int left = T - 1;
    auto chunk = [&](int t) {
        try {
            f(t, n * t / T, n * (t + 1) / T);
        } catch (...) {
            err[t] = std::current_exception();
        }
    };
    for (int t = 1; t < T; ++t)
        pool.push([&, t] {
            const bool was = detail::ChunkPool::in_task();
            detail::ChunkPool::in_task() = true;
            chunk(t);
            detail::ChunkPool::in_task() = was;
            std::lock_guard<std::mutex> l(m);
            if (--left == 0) cv.notify_all();
        });
    {
        const bool was = detail::ChunkPool::in_task();
        detail::ChunkPool::in_task() = true;
        chunk(0);
        detail::ChunkPool::in_task() = was;
    }
    // help with queued chunks (this call's or others') until this call's are done
    for (;;) {
        {
            std::lock_guard<std::mutex> l(m);
            if (left == 0) break;
        }
        if (!pool.run_one()) {
            std::unique_lock<std::mutex> l(m);
            cv.wait(l, [&] { return left == 0; });
            break;
        }
    }
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

}  // namespace vag
