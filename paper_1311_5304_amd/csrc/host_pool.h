// Parallel loops on host threads: `ParallelFor` runs fn(0..n_tasks-1) and
// returns when all are done.  spawn_for starts threads for the one loop;
// WorkerPool keeps its threads between loops (a condition variable wakes
// them), for callers that run many short loops per image.  A pinned pool
// gives each of its threads a CPU of its own from the process's affinity
// set (the caller's thread too, for the duration of each loop), so that no
// two of them share a core and none migrates in the middle of a loop; with
// fewer allowed CPUs than threads it stays unpinned.
#pragma once

#include <pthread.h>
#include <sched.h>

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

// The CPUs of the process's affinity set, in order.
inline std::vector<int> allowed_cpus() {
  std::vector<int> cpus;
  cpu_set_t set;
  CPU_ZERO(&set);
  if (sched_getaffinity(0, sizeof(set), &set) != 0) return cpus;
  for (int c = 0; c < CPU_SETSIZE; ++c)
    if (CPU_ISSET(c, &set)) cpus.push_back(c);
  return cpus;
}

inline bool pin_thread(pthread_t t, int cpu) {
  cpu_set_t set;
  CPU_ZERO(&set);
  CPU_SET(cpu, &set);
  return pthread_setaffinity_np(t, sizeof(set), &set) == 0;
}

class WorkerPool {
 public:
  explicit WorkerPool(int n_threads, bool pin = false) {
    if (pin) {
      const std::vector<int> cpus = allowed_cpus();
      if (static_cast<int>(cpus.size()) >= n_threads) cpus_ = cpus;
    }
    for (int t = 1; t < n_threads; ++t) {
      th_.emplace_back([this] { loop(); });
      if (!cpus_.empty()) pin_thread(th_.back().native_handle(), cpus_[t]);
    }
  }
  bool pinned() const { return !cpus_.empty(); }
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
    // a pinned pool runs the caller on the one CPU no worker holds, and
    // gives it its own affinity back afterwards
    cpu_set_t saved;
    const bool repin = !cpus_.empty() && pthread_getaffinity_np(pthread_self(), sizeof(saved), &saved) == 0 &&
                       pin_thread(pthread_self(), cpus_[0]);
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
    if (repin) pthread_setaffinity_np(pthread_self(), sizeof(saved), &saved);
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
  std::vector<int> cpus_;  // pinned: the CPU of thread t (0: the caller)
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
