// Host-side data parallelism for the symbolic phases (no device code).
#pragma once

#include <algorithm>
#include <cstdint>
#include <exception>
#include <thread>
#include <vector>

namespace vag {

// Runs f(t, begin, end) over [0, n) split into contiguous chunks, one per
// thread (at most 16, at least min_items items each); the first exception
// thrown by a chunk is rethrown.
template <class F>
void parallel_chunks(int64_t n, F &&f, int64_t min_items = 32768) {
    const int64_t hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(hw, n / min_items));
    if (T == 1) {
        f(0, (int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> err(T);
    for (int t = 0; t < T; ++t)
        th.emplace_back([&, t] {
            try {
                f(t, n * t / T, n * (t + 1) / T);
            } catch (...) {
                err[t] = std::current_exception();
            }
        });
    for (auto &x : th) x.join();
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

// the number of chunks parallel_chunks uses for n items
inline int chunk_count(int64_t n, int64_t min_items = 32768) {
    const int64_t hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    return (int)std::max<int64_t>(1, std::min<int64_t>(hw, n / min_items));
}

}  // namespace vag
