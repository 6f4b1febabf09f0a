// Two rings of pinned host memory per stream.  put() writes a kernel
// descriptor array into the descriptor ring (device-coherent, mapped) and
// returns the device view of it: kernels read their descriptor once, at the
// start, straight from host memory, so no copy is queued.  upload() stages
// bytes in the upload ring (ordinary pinned memory, the fast path of the
// copy engines) and queues a stream-ordered async copy into caller-owned
// device memory.  Each ring is split in two halves; an event is recorded on
// the stream whenever the write position leaves a half, and before a half
// is reused the event of its previous use is awaited -- work issued half a
// ring earlier, normally long finished -- so a region is never rewritten
// before the copies and kernels that read it have run, and the host rarely
// waits.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>
#include <map>
#include <mutex>

#include "host_pool.h"
#include "htrace.h"
#include "internal.h"

namespace abddc {

class Ring {
 public:
  Ring(hipStream_t s, bool coherent) : s_(s), coherent_(coherent) {}
  ~Ring() {
    if (h_) (void)hipHostFree(h_);
    for (int i = 0; i < 2; ++i)
      if (ev_[i]) (void)hipEventDestroy(ev_[i]);
  }
  // offset of a fresh region of at least bytes (256-byte aligned)
  size_t reserve(size_t bytes) {
    const size_t need = (bytes + 255) & ~size_t(255);
    if (2 * need > cap_) grow(2 * need);
    const size_t half = cap_ / 2;
    const int cur = off_ < half ? 0 : 1;
    if (off_ + need > (size_t)(cur + 1) * half) {
      // leave the current half; wait for the previous use of the next one
      ABDDC_HIP(hipEventRecord(ev_[cur], s_));
      used_[cur] = true;
      const int nxt = 1 - cur;
      if (used_[nxt]) {
        HostTrace ht;
        ABDDC_HIP(hipEventSynchronize(ev_[nxt]));
        ht.mark("staging ring: wait for the other half");
      }
      off_ = (size_t)nxt * half;
    }
    const size_t off = off_;
    off_ += need;
    return off;
  }
  char* host() const { return h_; }
  char* dev() const { return dh_; }

 private:
  void grow(size_t need) {
    HostTrace ht;
    ABDDC_HIP(hipStreamSynchronize(s_));
    size_t cap = cap_ ? 2 * cap_ : (size_t(32) << 20);
    while (cap < need) cap *= 2;
    if (h_) ABDDC_HIP(hipHostFree(h_));
    h_ = nullptr;
    dh_ = nullptr;
    h_ = alloc_writable(cap, coherent_ ? (hipHostMallocMapped | hipHostMallocCoherent) : hipHostMallocDefault);
    if (coherent_) ABDDC_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&dh_), h_, 0));
    for (int i = 0; i < 2; ++i) {
      if (!ev_[i]) ABDDC_HIP(hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming));
      used_[i] = false;
    }
    cap_ = cap;
    off_ = 0;
    ht.mark("staging ring: grow");
  }
  // Pinned host memory the host writes at cache speed.  Every page is
  // touched once here, so that no host store into the ring later pays a
  // first-touch fault; and since some pinned allocations come back mapped
  // uncached on the host side (stores then run at a few GB/s), a timed
  // 1 MiB store pass checks the mapping and up to three more allocations
  // are tried, the fastest kept.
  static char* alloc_writable(size_t cap, unsigned flags) {
    char* best = nullptr;
    double best_rate = -1.0;
    std::vector<char*> spare;
    const size_t probe = std::min<size_t>(cap, size_t(1) << 20);
    for (int attempt = 0; attempt < 4; ++attempt) {
      char* h = nullptr;
      ABDDC_HIP(hipHostMalloc(reinterpret_cast<void**>(&h), cap, flags));
      std::memset(h, 0, cap);   // touch every page once
      const auto t0 = std::chrono::steady_clock::now();
      std::memset(h, 1, probe);
      const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
      const double rate = probe / std::max(us, 1e-3) / 1e3;   // GB/s
      if (rate > best_rate) {
        if (best) spare.push_back(best);
        best = h;
        best_rate = rate;
      } else {
        spare.push_back(h);
      }
      if (best_rate >= 20.0) break;
    }
    for (char* h : spare) ABDDC_HIP(hipHostFree(h));
    return best;
  }
  hipStream_t s_;
  bool coherent_;
  char* h_ = nullptr;    // host view
  char* dh_ = nullptr;   // device view (coherent ring only)
  size_t cap_ = 0, off_ = 0;
  hipEvent_t ev_[2] = {nullptr, nullptr};
  bool used_[2] = {false, false};
};

class Arena {
 public:
  explicit Arena(hipStream_t s) : desc_(s, true), up_(s, false), s_(s) {}
  void* put(const void* src, size_t bytes) {
    const size_t off = desc_.reserve(bytes);
    std::memcpy(desc_.host() + off, src, bytes);
    return desc_.dev() + off;
  }
  // Stream-ordered upload into caller-owned device memory through the ring
  // (the staging copy of a large upload split over the host pool).
  void upload(void* dst, const void* src, size_t bytes) {
    const size_t off = up_.reserve(bytes);
    char* stage = up_.host() + off;
    constexpr size_t PIECE = size_t(128) << 10;
    if (bytes >= 4 * PIECE) {
      const int64_t np = (int64_t)((bytes + PIECE - 1) / PIECE);
      host_parallel_for(np, 1, [&](int64_t b, int64_t e) {
        const size_t lo = (size_t)b * PIECE, hi = std::min(bytes, (size_t)e * PIECE);
        std::memcpy(stage + lo, static_cast<const char*>(src) + lo, hi - lo);
      });
    } else {
      std::memcpy(stage, src, bytes);
    }
    ABDDC_HIP(hipMemcpyAsync(dst, stage, bytes, hipMemcpyHostToDevice, s_));
  }
  template <class T>
  T* put(const std::vector<T>& v) {
    return static_cast<T*>(put(v.data(), v.size() * sizeof(T)));
  }

  static Arena& for_stream(hipStream_t s) {
    static std::mutex mu;
    static std::map<hipStream_t, Arena*> table;
    std::lock_guard<std::mutex> g(mu);
    auto it = table.find(s);
    if (it != table.end()) return *it->second;
    Arena* a = new Arena(s);
    table[s] = a;
    return *a;
  }

 private:
  Ring desc_, up_;
  hipStream_t s_;
};

}  // namespace abddc
