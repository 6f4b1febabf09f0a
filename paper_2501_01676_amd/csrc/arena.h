// Ring of kernel descriptor arrays and host->device uploads in pinned,
// device-coherent host memory.  put() writes a descriptor array into the
// ring and returns the device view of it: kernels read their descriptor
// once, at the start, straight from host memory, so no copy is queued.
// upload() stages bytes in the ring and queues a stream-ordered async copy
// into caller-owned device memory.  The ring is split in two halves; an
// event is recorded on the stream whenever the write position leaves a half,
// and before a half is reused the event of its previous use is awaited --
// work issued half a ring earlier, normally long finished -- so a region is
// never rewritten before the copies and kernels that read it have run, and
// the host rarely waits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>

#include "htrace.h"
#include "internal.h"

namespace abddc {

class Arena {
 public:
  explicit Arena(hipStream_t s) : s_(s) {}
  ~Arena() {
    if (h_) (void)hipHostFree(h_);
    for (int i = 0; i < 2; ++i)
      if (ev_[i]) (void)hipEventDestroy(ev_[i]);
  }
  void* put(const void* src, size_t bytes) {
    const size_t off = reserve(bytes);
    std::memcpy(h_ + off, src, bytes);
    return dh_ + off;
  }
  // Stream-ordered upload into caller-owned device memory through the ring.
  void upload(void* dst, const void* src, size_t bytes) {
    const size_t off = reserve(bytes);
    std::memcpy(h_ + off, src, bytes);
    ABDDC_HIP(hipMemcpyAsync(dst, h_ + off, bytes, hipMemcpyHostToDevice, s_));
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
  void grow(size_t need) {
    HostTrace ht;
    ABDDC_HIP(hipStreamSynchronize(s_));
    size_t cap = cap_ ? 2 * cap_ : (size_t(32) << 20);
    while (cap < need) cap *= 2;
    if (h_) ABDDC_HIP(hipHostFree(h_));
    h_ = nullptr;
    dh_ = nullptr;
    ABDDC_HIP(hipHostMalloc(&h_, cap, hipHostMallocMapped | hipHostMallocCoherent));
    ABDDC_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&dh_), h_, 0));
    for (int i = 0; i < 2; ++i) {
      if (!ev_[i]) ABDDC_HIP(hipEventCreateWithFlags(&ev_[i], hipEventDisableTiming));
      used_[i] = false;
    }
    cap_ = cap;
    off_ = 0;
    ht.mark("staging ring: grow");
  }
  hipStream_t s_;
  char* h_ = nullptr;    // pinned ring, host view
  char* dh_ = nullptr;   // the same memory as the device sees it
  size_t cap_ = 0, off_ = 0;
  hipEvent_t ev_[2] = {nullptr, nullptr};
  bool used_[2] = {false, false};
};

}  // namespace abddc
