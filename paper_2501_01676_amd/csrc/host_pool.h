// A fixed pool of host threads for the data-parallel host loops of assembly
// and setup (index maps over subdomains, objects, faces and edges), which
// otherwise leave the GPU idle while one core builds them.  ABDDC_HOST_THREADS
// sets the pool size (default: the hardware threads, at most 16; 1 runs every
// loop on the calling thread).  Loop bodies must not call HIP.
//
// The loops come in bursts between device waits and are short (tens of
// microseconds of work), so dispatch is lock-free: the job is published
// through atomics, chunks are claimed and counted with atomics, and idle
// workers spin for a while before they sleep on a condition variable.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace abddc {

class HostPool {
 public:
  static HostPool& get() {
    static HostPool* p = new HostPool();   // intentionally never destroyed (workers detach at exit)
    return *p;
  }
  int threads() const { return nworkers_ + 1; }

  // body(begin, end) over [0, n) in contiguous chunks, at least `grain`
  // indices each, on the workers and the calling thread; returns when every
  // chunk is done and rethrows the first exception a chunk threw.
  void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)>& body) {
    if (n <= 0) return;
    const int64_t nchunk = std::min<int64_t>(threads(), std::max<int64_t>(1, n / std::max<int64_t>(grain, 1)));
    if (nchunk <= 1 || nworkers_ == 0) {
      body(0, n);
      return;
    }
    std::lock_guard<std::mutex> call(call_mu_);   // one parallel loop at a time
    body_ = &body;
    n_ = n;
    nchunk_ = nchunk;
    next_.store(0);
    finished_.store(0);
    error_ = nullptr;
    open_.store(true);   // publishes the fields above
    gen_.fetch_add(1);
    {
      std::lock_guard<std::mutex> g(sleep_mu_);   // no lost wake-up: sleepers test gen_ under it
    }
    sleep_cv_.notify_all();
    run_chunks();
    while (finished_.load() < nchunk_) spin_pause();
    // withdraw the job, then wait for every worker still inside it: a worker
    // registers in active_ before it reads open_, so one that saw the job
    // open is counted here (both sides sequentially consistent)
    open_.store(false);
    while (active_.load() != 0) spin_pause();
    if (error_) std::rethrow_exception(error_);
  }

 private:
  HostPool() {
    int nt = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
    if (const char* e = std::getenv("ABDDC_HOST_THREADS")) nt = std::max(1, std::atoi(e));
    nworkers_ = nt - 1;
    for (int i = 0; i < nworkers_; ++i) std::thread([this] { worker(); }).detach();
  }

  static void spin_pause() {
#if defined(__x86_64__)
    __builtin_ia32_pause();
#endif
  }

  void run_chunks() {
    for (;;) {
      const int64_t c = next_.fetch_add(1);
      if (c >= nchunk_) return;
      const int64_t b = n_ * c / nchunk_, e = n_ * (c + 1) / nchunk_;
      try {
        (*body_)(b, e);
      } catch (...) {
        std::lock_guard<std::mutex> g(err_mu_);
        if (!error_) error_ = std::current_exception();
      }
      finished_.fetch_add(1);
    }
  }

  void worker() {
    uint64_t seen = gen_.load();
    for (;;) {
      // a new job: spin for up to ~200 us (the loops of one call follow each
      // other closely), then sleep
      const auto t0 = std::chrono::steady_clock::now();
      int spins = 0;
      while (gen_.load() == seen) {
        spin_pause();
        if (++spins == 256) {
          spins = 0;
          if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(200)) {
            std::unique_lock<std::mutex> g(sleep_mu_);
            sleep_cv_.wait(g, [&] { return gen_.load() != seen; });
          }
        }
      }
      seen = gen_.load();
      active_.fetch_add(1);
      if (open_.load()) run_chunks();
      active_.fetch_sub(1);
    }
  }

  int nworkers_ = 0;
  std::mutex call_mu_, sleep_mu_, err_mu_;
  std::condition_variable sleep_cv_;
  // the current job (written by the caller before open_ is set)
  const std::function<void(int64_t, int64_t)>* body_ = nullptr;
  int64_t n_ = 0, nchunk_ = 0;
  std::exception_ptr error_;   // guarded by err_mu_ while the job is open
  std::atomic<int64_t> next_{0}, finished_{0};
  std::atomic<bool> open_{false};
  std::atomic<int> active_{0};
  std::atomic<uint64_t> gen_{0};
};

inline void host_parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)>& body) {
  HostPool::get().parallel_for(n, grain, body);
}

}  // namespace abddc
