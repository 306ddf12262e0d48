// Host-only helpers shared by the runtime (no HIP types): the worker pool
// that validates and plans the patterns of a batch, and the plan cache.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dm_common.hpp"

namespace dm {

// Host workers for the per-pattern validation and planning of a batch.
// One parallel_for at a time (a concurrent caller runs its loop itself);
// every worker checks in for every generation, so the loop body and its
// count stay valid until the call returns.
class HostPool {
  public:
    static HostPool& get() {
        static HostPool pool;
        return pool;
    }
    void parallel_for(int n, const std::function<void(int)>& f) {
        std::unique_lock<std::mutex> busy(call_mu_, std::try_to_lock);
        if (!busy.owns_lock() || workers_.empty() || n < 8) {
            for (int i = 0; i < n; i++) f(i);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            fn_ = &f;
            n_ = n;
            next_.store(0);
            checked_in_ = 0;
            gen_++;
        }
        cv_.notify_all();
        run();
        std::unique_lock<std::mutex> lk(mu_);
        cv_done_.wait(lk, [&] { return checked_in_ == (int)workers_.size(); });
        fn_ = nullptr;
    }
    ~HostPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : workers_) t.join();
    }

    // workers < 0: up to 15 workers + the calling thread, one GPU's share of
    // host CPUs
    explicit HostPool(int workers = -1) {
        const unsigned hw = std::thread::hardware_concurrency();
        const int w = workers >= 0 ? workers : (int)std::min<unsigned>(hw > 1 ? hw - 1 : 0, 15);
        for (int i = 0; i < w; i++) workers_.emplace_back([this] { loop(); });
    }

  private:
    void run() {
        for (int i; (i = next_.fetch_add(1)) < n_;) (*fn_)(i);
    }
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
            }
            run();
            {
                std::lock_guard<std::mutex> lk(mu_);
                checked_in_++;
            }
            cv_done_.notify_all();
        }
    }
    std::vector<std::thread> workers_;
    std::mutex call_mu_, mu_;
    std::condition_variable cv_, cv_done_;
    const std::function<void(int)>* fn_ = nullptr;
    std::atomic<int> next_{0};
    int n_ = 0, checked_in_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

// Plans by key (pattern, motif set, table statistics): a repeated pattern
// shape on a data graph with the same tables skips the decomposition.  Safe
// for concurrent use; it is emptied when it reaches `max_entries`.
class PlanCache {
  public:
    explicit PlanCache(size_t max_entries = 8192) : max_(max_entries) {}
    bool get(const std::string& key, Plan* out) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = map_.find(key);
        if (it == map_.end()) return false;
        *out = it->second;
        return true;
    }
    void put(std::string key, const Plan& plan) {
        std::lock_guard<std::mutex> lk(mu_);
        if (map_.size() >= max_) map_.clear();
        map_.emplace(std::move(key), plan);
    }
    size_t size() {
        std::lock_guard<std::mutex> lk(mu_);
        return map_.size();
    }
    // what the last sort of the plan's table learned (Plan::sort_stream)
    void set_sort_stream(const std::string& key, int32_t v) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = map_.find(key);
        if (it != map_.end()) it->second.sort_stream = v;
    }

  private:
    size_t max_;
    std::mutex mu_;
    std::unordered_map<std::string, Plan> map_;
};

}  // namespace dm
