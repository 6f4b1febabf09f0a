// Bump arena for kernel descriptor arrays: a pinned host mirror and a device
// buffer; each put() copies into pinned memory and issues a stream-ordered
// async copy to the device.  When full it synchronises the stream and starts
// over, so a region is never rewritten before the kernels that read it ran.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>

#include "internal.h"

namespace abddc {

class Arena {
 public:
  explicit Arena(hipStream_t s) : s_(s) {}
  ~Arena() {
    if (d_) (void)hipFree(d_);
    if (h_) (void)hipHostFree(h_);
  }
  void* put(const void* src, size_t bytes) {
    size_t need = (bytes + 255) & ~size_t(255);
    if (off_ + need > cap_) {
      ABDDC_HIP(hipStreamSynchronize(s_));
      off_ = 0;
      if (need > cap_) grow(need);
    }
    std::memcpy(h_ + off_, src, bytes);
    void* dst = d_ + off_;
    ABDDC_HIP(hipMemcpyAsync(dst, h_ + off_, bytes, hipMemcpyHostToDevice, s_));
    off_ += need;
    return dst;
  }
  // Stream-ordered upload into caller-owned device memory through the same
  // pinned ring (no synchronisation unless the ring wraps).
  void upload(void* dst, const void* src, size_t bytes) {
    size_t need = (bytes + 255) & ~size_t(255);
    if (off_ + need > cap_) {
      ABDDC_HIP(hipStreamSynchronize(s_));
      off_ = 0;
      if (need > cap_) grow(need);
    }
    std::memcpy(h_ + off_, src, bytes);
    ABDDC_HIP(hipMemcpyAsync(dst, h_ + off_, bytes, hipMemcpyHostToDevice, s_));
    off_ += need;
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
  void grow(size_t need) {
    size_t cap = cap_ ? cap_ : (size_t(8) << 20);
    while (cap < need) cap *= 2;
    if (d_) ABDDC_HIP(hipFree(d_));
    if (h_) ABDDC_HIP(hipHostFree(h_));
    d_ = nullptr;
    h_ = nullptr;
    ABDDC_HIP(hipMalloc(&d_, cap));
    ABDDC_HIP(hipHostMalloc(&h_, cap, hipHostMallocDefault));
    cap_ = cap;
  }
  hipStream_t s_;
  char* d_ = nullptr;
  char* h_ = nullptr;
  size_t cap_ = 0, off_ = 0;
};

}  // namespace abddc
