// Live per-kernel timing with HIP events on the launch stream.  An entry
// point sets the thread's sink to its context; instrumented launchers take
// an event pair that hipExtLaunchKernel stamps at the start and the end of
// the kernel itself, and record the launch's algorithmic work (flops or
// bytes).  resolve() turns finished pairs into accumulated seconds.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

namespace abddc {

// Timing events kept for the process, per device: contexts come and go once
// per solve, and creating and destroying a few hundred events each time
// would cost milliseconds of host time.
struct EventPool {
  static hipEvent_t take() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
      std::lock_guard<std::mutex> g(mu());
      std::vector<hipEvent_t>& v = pools()[dev];
      if (!v.empty()) {
        hipEvent_t e = v.back();
        v.pop_back();
        return e;
      }
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  // events recorded on device dev, once the work that stamps them has
  // finished or will never run
  static void give(int dev, hipEvent_t e) {
    if (!e) return;
    std::lock_guard<std::mutex> g(mu());
    pools()[dev].push_back(e);
  }

 private:
  static std::mutex& mu() {
    static std::mutex m;
    return m;
  }
  static std::map<int, std::vector<hipEvent_t>>& pools() {
    static auto* p = new std::map<int, std::vector<hipEvent_t>>();   // kept until the process ends
    return *p;
  }
};

enum KernelClass {
  KC_PLU_UPDATE = 0,
  KC_GEMV = 1,
  KC_PLU_LEAD = 2,
  KC_PLU_DIAG = 3,
  KC_PLU_TRSM = 4,
  KC_PLU_BAND = 5,
  KC_COUNT = 6
};

struct KStats {
  double seconds[KC_COUNT] = {};
  double work[KC_COUNT] = {};
  int64_t launches[KC_COUNT] = {};
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double work;
  };
  std::vector<Pending> pending;
  int device = -1;   // device of the pending events

  void events(int cls, double work_amount, hipEvent_t* start, hipEvent_t* stop) {
    if (device < 0) (void)hipGetDevice(&device);
    Pending p{cls, EventPool::take(), EventPool::take(), work_amount};
    pending.push_back(p);
    *start = p.a;
    *stop = p.b;
  }
  // call after the stream has been synchronised
  void resolve() {
    for (auto& p : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        seconds[p.cls] += ms * 1e-3;
        work[p.cls] += p.work;
        launches[p.cls] += 1;
      }
      EventPool::give(device, p.a);
      EventPool::give(device, p.b);
    }
    pending.clear();
  }
  ~KStats() {
    // unresolved pairs (a call that failed before its synchronisation): an
    // event may still be stamped by queued work, so it is not reused
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
  }
};

extern thread_local KStats* g_kstats;
// Classes timed with events, process-wide (bit k: class k); a timed launch
// waits for its events, so classes outside the mask run untimed.
extern std::atomic<uint32_t> g_kstats_mask;

inline bool kstats_on(int cls) {
  return g_kstats && ((g_kstats_mask.load(std::memory_order_relaxed) >> cls) & 1u);
}

// Event pair for one launch of a tracked kernel (both null when no sink is
// set or the class is not timed; hipExtLaunchKernel then launches without
// timing).
inline void tracked_events(int cls, double work_amount, hipEvent_t* start, hipEvent_t* stop) {
  *start = *stop = nullptr;
  if (kstats_on(cls) && work_amount > 0) g_kstats->events(cls, work_amount, start, stop);
}

// RAII: route the launches of one entry point into ctx stats.
struct KStatsScope {
  KStats* prev;
  explicit KStatsScope(KStats* k) : prev(g_kstats) { g_kstats = k; }
  ~KStatsScope() { g_kstats = prev; }
};

}  // namespace abddc
