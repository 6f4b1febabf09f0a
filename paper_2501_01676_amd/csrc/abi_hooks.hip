// C ABI: error reporting and the batched-primitive test hooks.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <map>
#include <unordered_map>
#include <mutex>
#include <string>
#include <tuple>

#include "arena.h"
#include "guard.h"
#include "htrace.h"
#include "internal.h"
#include "kstats.h"

namespace abddc {
thread_local std::string g_last_error;
thread_local KStats* g_kstats = nullptr;
std::atomic<uint32_t> g_kstats_mask{(1u << KC_COUNT) - 1};

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
}  // namespace abddc

namespace abddc {
thread_local const DevAlloc* g_dev_alloc = nullptr;

void* hooked_alloc(const DevAlloc& h, size_t bytes) {
  void* p = h.alloc(bytes, h.user);
  if (!p) throw Error(ABDDC_ENOMEM, "the caller's device allocation hook returned NULL for " +
                                        std::to_string(bytes) + " bytes");
  return p;
}

thread_local hipStream_t g_stream = nullptr;

namespace {
// A cached block is kept under the stream whose work may still use it.  On
// that same stream it is reused at once (stream order protects it); another
// stream takes it only behind an event recorded on the first one at that
// moment, which it waits for on the device.
struct Cache {
  std::mutex mu;
  // (device, releasing stream, block size) -> block
  std::multimap<std::tuple<int, hipStream_t, size_t>, void*> free_blocks;
  std::unordered_map<void*, size_t> block_size;   // every block ever allocated
};
Cache& cache() {
  static Cache* c = new Cache();  // intentionally never destroyed
  return *c;
}
// allocations served by the cache per device since the process started
constexpr int STAT_DEVICES = 64;
std::atomic<int64_t> g_cache_allocs[STAT_DEVICES];
std::atomic<int64_t> g_cache_bytes[STAT_DEVICES];
void count_alloc(int dev, size_t bytes) {
  if (dev >= 0 && dev < STAT_DEVICES) {
    g_cache_allocs[dev].fetch_add(1, std::memory_order_relaxed);
    g_cache_bytes[dev].fetch_add((int64_t)bytes, std::memory_order_relaxed);
  }
}
size_t round_size(size_t b) {
  if (b <= (size_t(1) << 20)) {
    size_t r = 256;
    while (r < b) r <<= 1;
    return r;
  }
  const size_t g = size_t(1) << 20;  // 1 MiB granules above 1 MiB
  return (b + g - 1) / g * g;
}
}  // namespace

void staged_upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes) Arena::for_stream(s).upload(dst, src, bytes);
}

int32_t* pinned_ints(size_t n) {
  static thread_local int32_t* p = nullptr;
  static thread_local size_t cap = 0;
  if (n > cap) {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    ABDDC_HIP(hipHostMalloc((void**)&p, n * sizeof(int32_t), hipHostMallocDefault));
    cap = n;
  }
  return p;
}

void* cache_alloc(size_t bytes) {
  int dev = 0;
  ABDDC_HIP(hipGetDevice(&dev));
  const size_t r = round_size(bytes);
  const size_t rmax = 2 * r + (size_t(1) << 20);   // best fit wasting at most r + 1 MiB
  Cache& c = cache();
  void* blk = nullptr;
  hipStream_t from = nullptr;
  {
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.free_blocks.lower_bound({dev, g_stream, r});
    if (it != c.free_blocks.end() && std::get<0>(it->first) == dev && std::get<1>(it->first) == g_stream &&
        std::get<2>(it->first) <= rmax) {
      blk = it->second;
      from = g_stream;
      c.free_blocks.erase(it);
    } else {
      // the smallest fitting block released on another stream of the device
      auto best = c.free_blocks.end();
      for (auto jt = c.free_blocks.lower_bound({dev, nullptr, 0}); jt != c.free_blocks.end() && std::get<0>(jt->first) == dev;
           ++jt) {
        const size_t sz = std::get<2>(jt->first);
        if (std::get<1>(jt->first) != g_stream && sz >= r && sz <= rmax &&
            (best == c.free_blocks.end() || sz < std::get<2>(best->first)))
          best = jt;
      }
      if (best != c.free_blocks.end()) {
        blk = best->second;
        from = std::get<1>(best->first);
        c.free_blocks.erase(best);
      }
    }
  }
  count_alloc(dev, bytes);
  if (blk) {
    if (from != g_stream) {
      // the work queued on the releasing stream so far comes first
      hipEvent_t ev = nullptr;
      bool ok = hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
      ok = ok && hipEventRecord(ev, from) == hipSuccess && hipStreamWaitEvent(g_stream, ev, 0) == hipSuccess;
      if (ev) (void)hipEventDestroy(ev);
      if (!ok) {
        (void)hipGetLastError();
        ABDDC_HIP(hipDeviceSynchronize());
      }
    }
    return blk;
  }
  void* p = nullptr;
  HostTrace ht;
  hipError_t e = hipMalloc(&p, r);
  if (ht.on) ht.mark(("allocator: hipMalloc " + std::to_string(r >> 10) + " KiB").c_str());
  if (e == hipErrorOutOfMemory) {
    // return cached blocks of this device to the driver and retry once
    ABDDC_HIP(hipDeviceSynchronize());
    std::lock_guard<std::mutex> g(c.mu);
    for (auto it = c.free_blocks.begin(); it != c.free_blocks.end();) {
      if (std::get<0>(it->first) == dev) {
        c.block_size.erase(it->second);
        (void)hipFree(it->second);
        it = c.free_blocks.erase(it);
      } else {
        ++it;
      }
    }
    (void)hipGetLastError();
    e = hipMalloc(&p, r);
  }
  if (e != hipSuccess)
    throw Error(e == hipErrorOutOfMemory ? ABDDC_ENOMEM : ABDDC_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
  {
    std::lock_guard<std::mutex> g(c.mu);
    c.block_size[p] = r;
  }
  return p;
}

void cache_free(void* p, size_t bytes) {
  if (!p) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  auto sz = c.block_size.find(p);
  c.free_blocks.insert({{dev, g_stream, sz != c.block_size.end() ? sz->second : round_size(bytes)}, p});
}
}  // namespace abddc

using namespace abddc;

extern "C" const char* abddc_last_error(void) { return g_last_error.c_str(); }

extern "C" int abddc_cache_stats(int32_t device, int64_t* allocations, int64_t* bytes) {
  if (device < 0 || device >= STAT_DEVICES) return fail(ABDDC_EINVAL, "device index out of range");
  if (allocations) *allocations = g_cache_allocs[device].load();
  if (bytes) *bytes = g_cache_bytes[device].load();
  return ABDDC_OK;
}

extern "C" uint32_t abddc_set_kernel_stats(uint32_t mask) {
  return g_kstats_mask.exchange(mask & ((1u << KC_COUNT) - 1));
}

namespace {

int check_flag(int* dflag, hipStream_t s) {
  int h = 0;
  ABDDC_HIP(hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  ABDDC_HIP(hipStreamSynchronize(s));
  if (h & 1) return fail(ABDDC_ESINGULAR, "zero or non-finite pivot");
  if (h & 2) return fail(ABDDC_EEIG, "eigenproblem metric not positive definite");
  return ABDDC_OK;
}
}  // namespace

extern "C" int abddc_test_partial_lu(int32_t batch, void* buf, const int64_t* off, const int32_t* nrow,
                                     const int32_t* ncol, const int32_t* ld, const int32_t* k,
                                     int32_t precision, void* stream) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(batch >= 0 && buf && off && nrow && ncol && ld && k, ABDDC_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    StreamScope ss(s);
    DevBuf<int> flag(1);
    flag.zero(s);
    if (precision == 0) {
      std::vector<PluDesc<double>> d(batch);
      for (int b = 0; b < batch; ++b) d[b] = {(double*)buf + off[b], nrow[b], ncol[b], ld[b], k[b]};
      partial_lu<double>(d, flag.p, s);
    } else {
      std::vector<PluDesc<float>> d(batch);
      for (int b = 0; b < batch; ++b) d[b] = {(float*)buf + off[b], nrow[b], ncol[b], ld[b], k[b]};
      partial_lu<float>(d, flag.p, s);
    }
    return check_flag(flag.p, s);
  });
}

extern "C" int abddc_test_gemm(int32_t batch, double* buf, const int64_t* offA, const int64_t* offB,
                               const int64_t* offC, const int32_t* m, const int32_t* n, const int32_t* k,
                               const int32_t* lda, const int32_t* ldb, const int32_t* ldc, int32_t transA,
                               int32_t transB, double alpha, double beta, void* stream) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(batch >= 0 && buf, ABDDC_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    StreamScope ss(s);
    std::vector<GemmDesc<double>> d(batch);
    for (int b = 0; b < batch; ++b)
      d[b] = {buf + offA[b], buf + offB[b], buf + offC[b], m[b], n[b], k[b], lda[b], ldb[b], ldc[b]};
    gemm_batched<double>(d, transA != 0, transB != 0, alpha, beta, s);
    ABDDC_HIP(hipStreamSynchronize(s));
    return ABDDC_OK;
  });
}

extern "C" int abddc_test_sygv(int32_t batch, double* buf, const int64_t* offA, const int64_t* offB,
                               const int64_t* offW, const int64_t* offX, const int32_t* n, void* stream) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(batch >= 0 && buf, ABDDC_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    StreamScope ss(s);
    DevBuf<int> flag(1);
    flag.zero(s);
    std::vector<SygvDesc> d(batch);
    for (int b = 0; b < batch; ++b) d[b] = {buf + offA[b], buf + offB[b], buf + offW[b], buf + offX[b], n[b]};
    sygv_batched(d, flag.p, s);
    return check_flag(flag.p, s);
  });
}

extern "C" int abddc_test_parallel_sum(int32_t batch, double* buf, const int64_t* offA, const int64_t* offB,
                                       const int64_t* offOut, const int32_t* n, double rtol, void* stream) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(batch >= 0 && buf && offA && offB && offOut && n, ABDDC_EINVAL, "null argument");
    ABDDC_REQUIRE(rtol >= 0, ABDDC_EINVAL, "negative tolerance");
    hipStream_t s = (hipStream_t)stream;
    StreamScope ss(s);
    std::vector<PsumDesc> d(batch);
    for (int b = 0; b < batch; ++b) d[b] = {buf + offA[b], buf + offB[b], buf + offOut[b], n[b], n[b], n[b]};
    parallel_sum_batched(d, rtol, s);
    ABDDC_HIP(hipStreamSynchronize(s));
    return ABDDC_OK;
  });
}

extern "C" int abddc_test_sygv_select(int32_t batch, double* buf, const int64_t* offA, const int64_t* offB,
                                      const int64_t* offW, const int64_t* offX, const int32_t* n, double sel,
                                      void* stream) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(batch >= 0 && buf, ABDDC_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    StreamScope ss(s);
    DevBuf<int> flag(1);
    flag.zero(s);
    std::vector<SygvDesc> d(batch);
    for (int b = 0; b < batch; ++b) d[b] = {buf + offA[b], buf + offB[b], buf + offW[b], buf + offX[b], n[b]};
    sygv_select_batched(d, sel, flag.p, s);
    return check_flag(flag.p, s);
  });
}

extern "C" int abddc_test_schur_pinv(int32_t batch, double* buf, const int64_t* off, const int32_t* nv,
                                     const int32_t* k, double rtol, void* stream) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(batch >= 0 && buf && off && nv && k, ABDDC_EINVAL, "null argument");
    ABDDC_REQUIRE(rtol >= 0, ABDDC_EINVAL, "negative tolerance");
    hipStream_t s = (hipStream_t)stream;
    StreamScope ss(s);
    DevBuf<int> flag(1);
    flag.zero(s);
    std::vector<SchurPinvDesc> d(batch);
    for (int b = 0; b < batch; ++b) d[b] = {buf + off[b], nv[b], k[b], nv[b]};
    schur_pinv_batched(d, rtol, flag.p, s);
    return check_flag(flag.p, s);
  });
}
