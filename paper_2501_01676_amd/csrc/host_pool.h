// A fixed pool of host threads for the data-parallel host loops of assembly
// and setup (index maps over subdomains, objects, faces and edges), which
// otherwise leave the GPU idle while one core builds them.  ABDDC_HOST_THREADS
// sets the pool size (default: the hardware threads, at most 16; 1 runs every
// loop on the calling thread).  Loop bodies must not call HIP.
#pragma once

#include <algorithm>
#include <atomic>
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
  int threads() const { return (int)workers_.size() + 1; }

  // body(begin, end) over [0, n) in contiguous chunks, at least `grain`
  // indices each, on the workers and the calling thread; returns when every
  // chunk is done and rethrows the first exception a chunk threw.
  void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)>& body) {
    if (n <= 0) return;
    const int64_t nchunk = std::min<int64_t>(threads(), std::max<int64_t>(1, n / std::max<int64_t>(grain, 1)));
    if (nchunk <= 1 || workers_.empty()) {
      body(0, n);
      return;
    }
    std::unique_lock<std::mutex> call(call_mu_);   // one parallel loop at a time
    Job job;
    job.body = &body;
    job.n = n;
    job.nchunk = nchunk;
    {
      std::lock_guard<std::mutex> g(mu_);
      job_ = &job;
      ++gen_;
    }
    cv_.notify_all();
    run_chunks(job);
    {
      // every chunk finished and no worker still inside the job; the job is
      // withdrawn under the same lock, so no worker can take it afterwards
      std::unique_lock<std::mutex> g(mu_);
      done_cv_.wait(g, [&] { return job.finished == job.nchunk && job.active == 0; });
      job_ = nullptr;
    }
    if (job.error) std::rethrow_exception(job.error);
  }

 private:
  struct Job {
    const std::function<void(int64_t, int64_t)>* body = nullptr;
    int64_t n = 0, nchunk = 0;
    std::atomic<int64_t> next{0};
    int64_t finished = 0;          // guarded by mu_
    int active = 0;                // workers inside run_chunks, guarded by mu_
    std::exception_ptr error;      // guarded by mu_
  };

  HostPool() {
    int nt = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
    if (const char* e = std::getenv("ABDDC_HOST_THREADS")) nt = std::max(1, std::atoi(e));
    for (int i = 1; i < nt; ++i) {
      workers_.emplace_back([this] { worker(); });
      workers_.back().detach();
    }
  }

  void run_chunks(Job& job) {
    for (;;) {
      const int64_t c = job.next.fetch_add(1);
      if (c >= job.nchunk) return;
      const int64_t b = job.n * c / job.nchunk, e = job.n * (c + 1) / job.nchunk;
      std::exception_ptr err;
      try {
        (*job.body)(b, e);
      } catch (...) {
        err = std::current_exception();
      }
      std::lock_guard<std::mutex> g(mu_);
      if (err && !job.error) job.error = err;
      if (++job.finished == job.nchunk) done_cv_.notify_all();
    }
  }

  void worker() {
    uint64_t seen = 0;
    for (;;) {
      Job* job = nullptr;
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [&] { return gen_ != seen && job_ != nullptr; });
        seen = gen_;
        job = job_;
        ++job->active;
      }
      run_chunks(*job);
      {
        std::lock_guard<std::mutex> g(mu_);
        if (--job->active == 0) done_cv_.notify_all();
      }
    }
  }

  std::vector<std::thread> workers_;
  std::mutex mu_, call_mu_;
  std::condition_variable cv_, done_cv_;
  Job* job_ = nullptr;
  uint64_t gen_ = 0;
};

inline void host_parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)>& body) {
  HostPool::get().parallel_for(n, grain, body);
}

}  // namespace abddc
