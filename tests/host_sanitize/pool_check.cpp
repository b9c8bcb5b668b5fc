// Drives the host chunk pool (parallel_chunks on a process-wide set of worker
// threads) the way the library uses it, for a build with the host thread
// sanitizer (or the address one): several host threads submit at once, as
// serving workers do; a chunk calls parallel_chunks again (it then runs
// alone); a chunk throws and the submitter receives the exception.  Every
// sum is checked against the serial one.  Exit code 0: all correct.
#include <atomic>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "host_parallel.h"

using namespace vag;

namespace {

int64_t serial_sum(int64_t n, int64_t salt) {
    int64_t s = 0;
    for (int64_t i = 0; i < n; ++i) s += (i * 7 + salt) % 13;
    return s;
}

// per-chunk partial sums written to a chunk-owned slot, combined in order
int64_t chunked_sum(int64_t n, int64_t salt) {
    std::vector<int64_t> part((size_t)chunk_count(n, 1024), 0);
    parallel_chunks(n, [&](int t, int64_t i0, int64_t i1) {
        int64_t s = 0;
        for (int64_t i = i0; i < i1; ++i) s += (i * 7 + salt) % 13;
        part[t] = s;
    }, 1024);
    int64_t s = 0;
    for (int64_t v : part) s += v;
    return s;
}

}  // namespace

int main() {
    std::atomic<int> bad{0};
    // concurrent submitters
    std::vector<std::thread> th;
    for (int w = 0; w < 8; ++w)
        th.emplace_back([&, w] {
            for (int rep = 0; rep < 20; ++rep) {
                const int64_t n = 20000 + 3517 * ((w * 20 + rep) % 11);
                if (chunked_sum(n, w + rep) != serial_sum(n, w + rep)) ++bad;
            }
        });
    for (auto &t : th) t.join();
    if (bad) {
        std::printf("concurrent sums wrong: %d\n", bad.load());
        return 1;
    }
    // a chunk that calls parallel_chunks: the inner call runs in that chunk
    {
        const int64_t n = 64 * 1024;
        std::vector<int64_t> part((size_t)chunk_count(n, 1024), 0);
        parallel_chunks(n, [&](int t, int64_t i0, int64_t i1) { part[t] = chunked_sum(i1 - i0, i0); }, 1024);
        int64_t s = 0, ref = 0;
        for (int64_t v : part) s += v;
        const int T = chunk_count(n, 1024);
        for (int t = 0; t < T; ++t) {
            const int64_t i0 = n * t / T, i1 = n * (t + 1) / T;
            ref += serial_sum(i1 - i0, i0);
        }
        if (s != ref) {
            std::printf("nested sums wrong\n");
            return 1;
        }
    }
    // an exception in one chunk reaches the submitter; the pool goes on working
    {
        bool caught = false;
        try {
            parallel_chunks(100000, [&](int t, int64_t, int64_t) {
                if (t == 2) throw std::runtime_error("chunk 2");
            }, 1024);
        } catch (const std::runtime_error &e) {
            caught = std::string(e.what()) == "chunk 2";
        }
        if (!caught && chunk_count(100000, 1024) > 2) {
            std::printf("exception lost\n");
            return 1;
        }
        if (chunked_sum(50000, 5) != serial_sum(50000, 5)) {
            std::printf("sum after an exception wrong\n");
            return 1;
        }
    }
    std::printf("pool ok: %d chunks at most\n", chunk_count(1 << 30, 1));
    return 0;
}
