// Persistent host worker threads of the batched forms (plain C++, no HIP).
#pragma once

#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace eses {

// Persistent host threads for the per-molecule work of a batch, started on
// first use and kept until the process ends (never joined: they wait on a
// condition variable between calls).  One batch call uses them at a time;
// run(P, fn) runs fn(p) on workers p = 0 .. P-1 and returns when all are done.
// Threads that live as long as the process keep one pinned read-back slot
// each, instead of a new thread (and a new pinned slot) per worker and call.
class WorkerPool {
  public:
    static WorkerPool &get() {
        static WorkerPool *w = new WorkerPool();  // outlives static destruction
        return *w;
    }
    std::mutex call;  // held by the caller for the whole of one batch call

    void run(int P, const std::function<void(int)> &fn) {
        std::unique_lock<std::mutex> lk(mu_);
        while ((int)threads_.size() < P) {
            const int id = (int)threads_.size();
            threads_.emplace_back([this, id]() { loop(id); });
            threads_.back().detach();
        }
        fn_ = &fn;
        active_ = P;
        pending_ = P;
        ++gen_;
        cv_work_.notify_all();
        cv_done_.wait(lk, [&]() { return pending_ == 0; });
        fn_ = nullptr;
    }

  private:
    void loop(int id) {
        unsigned long long seen = 0;
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_work_.wait(lk, [&]() { return gen_ != seen; });
            seen = gen_;
            if (id >= active_) continue;
            const std::function<void(int)> *f = fn_;
            lk.unlock();
            (*f)(id);
            lk.lock();
            if (--pending_ == 0) cv_done_.notify_all();
        }
    }
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::vector<std::thread> threads_;
    const std::function<void(int)> *fn_ = nullptr;
    unsigned long long gen_ = 0;
    int active_ = 0, pending_ = 0;
};

}  // namespace eses
