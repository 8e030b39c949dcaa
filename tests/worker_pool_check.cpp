// Stress check of the batch worker pool (csrc/worker_pool.h) with stub jobs:
// many calls of varying width, each job claiming indices from a shared
// counter and writing its own slot, run under ThreadSanitizer by the CPU test.
#include <atomic>
#include <cstdio>
#include <vector>

#include "worker_pool.h"

int main() {
    eses::WorkerPool &pool = eses::WorkerPool::get();
    long long total = 0;
    for (int call = 0; call < 400; ++call) {
        const int n = 1 + (call * 7) % 37;     // jobs of this call
        const int P = 1 + (call % 8);          // workers used
        std::vector<int> done(n, 0), by(n, -1);
        std::atomic<int> next{0};
        const std::function<void(int)> fn = [&](int p) {
            for (int q = next++; q < n; q = next++) {
                done[q] += q + 1;
                by[q] = p;
            }
        };
        {
            std::lock_guard<std::mutex> one(pool.call);
            pool.run(P, fn);
        }
        for (int q = 0; q < n; ++q) {
            if (done[q] != q + 1 || by[q] < 0 || by[q] >= P) {
                std::printf("FAIL call %d job %d: %d by %d\n", call, q, done[q], by[q]);
                return 1;
            }
            total += done[q];
        }
    }
    std::printf("OK %lld\n", total);
    return 0;
}
