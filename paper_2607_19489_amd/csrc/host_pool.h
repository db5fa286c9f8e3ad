// Host-side parallel loops of the plan builder (no HIP dependency).
#pragma once

#include <stdint.h>
#include <unistd.h>

#include <algorithm>
#include <condition_variable>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

namespace afmm {

// Host loops over cells, groups and table entries run on up to 16 threads (a
// GPU's share of the host cores).  Each worker takes one contiguous range of
// [0, n); workers write disjoint outputs or integer partial counts that the
// caller sums in range order, so results do not depend on the thread count.
// An exception in a range is rethrown in the calling thread once every range
// has ended.
inline int host_threads() {
  static const int n = [] {
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(16u, h));
  }();
  return n;
}
inline int parts_for(int64_t n, int64_t grain = 1 << 14) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / grain));
}

// Workers started once per process (starting threads for every loop cost
// about 0.5 ms per loop, several milliseconds per plan).  The calling thread
// takes parts of its own job too.  A loop inside a part, a loop in a forked
// child and a loop when no worker could be started run in the calling thread.
class HostPool {
 public:
  static HostPool* get() {
    static HostPool* pool = new HostPool();  // never destroyed: workers live until the process ends
    return pool->pid_ == getpid() && pool->workers_ > 0 ? pool : nullptr;
  }
  static bool& in_part() {
    static thread_local bool inside = false;
    return inside;
  }
  // fn(t) for t = 0 .. parts - 1; fn must not throw
  template <typename F>
  void run(int parts, F& fn) {
    Job j;
    j.call = [](void* f, int t) { (*static_cast<F*>(f))(t); };
    j.fn = &fn;
    j.parts = parts;
    j.left = parts;
    std::unique_lock<std::mutex> lk(mu_);
    q_.push_back(&j);
    cv_.notify_all();
    while (j.next < j.parts) {
      const int t = take(&j);
      lk.unlock();
      exec(&j, t);
      lk.lock();
      --j.left;
    }
    done_.wait(lk, [&] { return j.left == 0; });
  }

 private:
  struct Job {
    void (*call)(void*, int);
    void* fn;
    int parts = 0, next = 0, left = 0;
  };
  HostPool() : pid_(getpid()) {
    for (int i = 1; i < host_threads(); ++i) {
      try {
        std::thread(&HostPool::loop, this).detach();
        ++workers_;
      } catch (...) {
        break;
      }
    }
  }
  // next part of j (called with the lock held); a job whose parts are all
  // handed out leaves the queue, so no worker touches it after its caller returns
  int take(Job* j) {
    const int t = j->next++;
    if (j->next >= j->parts) q_.erase(std::find(q_.begin(), q_.end(), j));
    return t;
  }
  static void exec(Job* j, int t) {
    in_part() = true;
    j->call(j->fn, t);
    in_part() = false;
  }
  void loop() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return !q_.empty(); });
      Job* j = q_.front();
      const int t = take(j);
      lk.unlock();
      exec(j, t);
      lk.lock();
      if (--j->left == 0) done_.notify_all();
    }
  }
  const pid_t pid_;
  int workers_ = 0;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  std::vector<Job*> q_;
};

// fn(begin, end, part) for part = 0 .. parts - 1
template <typename F>
void parallel_ranges(int64_t n, int parts, F&& fn) {
  parts = std::max(parts, 1);
  std::vector<std::exception_ptr> err((size_t)parts);
  auto run = [&](int t) {
    try {
      fn(n * t / parts, n * (t + 1) / parts, t);
    } catch (...) {
      err[(size_t)t] = std::current_exception();
    }
  };
  HostPool* pool = parts > 1 && !HostPool::in_part() ? HostPool::get() : nullptr;
  if (pool) {
    pool->run(parts, run);
  } else {
    for (int t = 0; t < parts; ++t) run(t);
  }
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

}  // namespace afmm
