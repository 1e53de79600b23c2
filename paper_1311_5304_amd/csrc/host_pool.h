// Parallel loops on host threads: `ParallelFor` runs fn(0..n_tasks-1) and
// returns when all are done.  spawn_for starts threads for the one loop;
// WorkerPool keeps its threads between loops (a condition variable wakes
// them), for callers that run many short loops per image.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace mjd {

using TaskFn = std::function<void(int)>;
using ParallelFor = std::function<void(int n_tasks, const TaskFn& fn)>;

// Up to n_threads threads (the caller one of them) pulling task indices.
inline void spawn_for(int n_threads, int n_tasks, const TaskFn& fn) {
  std::atomic<int> next{0};
  auto worker = [&]() {
    for (int i; (i = next.fetch_add(1, std::memory_order_relaxed)) < n_tasks;) fn(i);
  };
  const int nt = std::max(1, std::min(n_threads, n_tasks));
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
}

class WorkerPool {
 public:
  explicit WorkerPool(int n_threads) {
    for (int t = 1; t < n_threads; ++t) th_.emplace_back([this] { loop(); });
  }
  ~WorkerPool() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_ = true;
    }
    wake_.notify_all();
    for (auto& t : th_) t.join();
  }
  WorkerPool(const WorkerPool&) = delete;
  WorkerPool& operator=(const WorkerPool&) = delete;

  int size() const { return static_cast<int>(th_.size()) + 1; }

  // One loop at a time (the caller's thread works too).
  void run(int n_tasks, const TaskFn& fn) {
    if (n_tasks <= 0) return;
    {
      std::lock_guard<std::mutex> g(mu_);
      fn_ = &fn;
      n_tasks_ = n_tasks;
      next_.store(0, std::memory_order_relaxed);
      active_ = static_cast<int>(th_.size());
      ++gen_;
    }
    wake_.notify_all();
    pull(fn, n_tasks);
    std::unique_lock<std::mutex> g(mu_);
    done_.wait(g, [this] { return active_ == 0; });
    fn_ = nullptr;
  }

 private:
  void pull(const TaskFn& fn, int n) {
    for (int i; (i = next_.fetch_add(1, std::memory_order_relaxed)) < n;) fn(i);
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      const TaskFn* fn;
      int n;
      {
        std::unique_lock<std::mutex> g(mu_);
        wake_.wait(g, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
        fn = fn_;
        n = n_tasks_;
      }
      pull(*fn, n);
      std::lock_guard<std::mutex> g(mu_);
      if (--active_ == 0) done_.notify_one();
    }
  }

  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable wake_, done_;
  const TaskFn* fn_ = nullptr;
  int n_tasks_ = 0;
  std::atomic<int> next_{0};
  int active_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

}  // namespace mjd
