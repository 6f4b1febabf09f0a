// Internal declarations of the gfx950 adaptive BDDC library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/abddc.h"

namespace abddc {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define ABDDC_HIP(call)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::abddc::Error(e_ == hipErrorOutOfMemory ? ABDDC_ENOMEM : ABDDC_EDEVICE,         \
                           std::string(#call) + ": " + hipGetErrorString(e_));               \
  } while (0)

#define ABDDC_REQUIRE(cond, code, msg)                 \
  do {                                                 \
    if (!(cond)) throw ::abddc::Error((code), (msg));  \
  } while (0)

// Caching device allocator: blocks are rounded up and kept in per-device
// free lists for reuse (setup temporaries and repeated solves would
// otherwise pay hipMalloc / hipFree and their implicit synchronisation).
// Memory returns to the driver only at process exit.
void* cache_alloc(size_t bytes);
void cache_free(void* p, size_t bytes);
// Stream-ordered host -> device copy through the stream's pinned staging ring.
void staged_upload(void* dst, const void* src, size_t bytes, hipStream_t s);

// Pinned host memory for at least n ints, per thread, for device-to-host
// readbacks the host waits for by event (grown as needed; the caller waits
// for every readback before it calls again).
int32_t* pinned_ints(size_t n);

// Stream on which the current entry point works (released blocks are tagged
// with it).
extern thread_local hipStream_t g_stream;
struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : prev(g_stream) { g_stream = s; }
  ~StreamScope() { g_stream = prev; }
};

// Caller-supplied device allocation hooks (abddc_device alloc / free /
// user); a null alloc means the library's caching allocator.
struct DevAlloc {
  void* (*alloc)(size_t bytes, void* user) = nullptr;
  void (*free)(void* p, void* user) = nullptr;
  void* user = nullptr;
};
// Hooks of the entry point running on this thread (null: the library's
// cache).  Buffers remember the hooks they were allocated with and release
// through them, wherever they are destroyed.
extern thread_local const DevAlloc* g_dev_alloc;
struct AllocScope {
  const DevAlloc* prev;
  explicit AllocScope(const DevAlloc* a) : prev(g_dev_alloc) { g_dev_alloc = a; }
  ~AllocScope() { g_dev_alloc = prev; }
};
void* hooked_alloc(const DevAlloc& h, size_t bytes);   // throws ENOMEM on a null result

// Owning device allocation.
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevAlloc hooks{};
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), hooks(o.hooks) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    release();
    p = o.p; n = o.n; hooks = o.hooks; o.p = nullptr; o.n = 0;
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (!count) return;
    if (g_dev_alloc && g_dev_alloc->alloc) {
      hooks = *g_dev_alloc;
      p = static_cast<T*>(hooked_alloc(hooks, count * sizeof(T)));
    } else {
      hooks = DevAlloc{};
      p = static_cast<T*>(cache_alloc(count * sizeof(T)));
    }
  }
  void release() {
    if (p) {
      if (hooks.alloc) {
        if (hooks.free) hooks.free(p, hooks.user);
      } else {
        cache_free(p, n * sizeof(T));
      }
    }
    p = nullptr;
    n = 0;
  }
  void upload(const std::vector<T>& h, hipStream_t s) {
    if (h.size() > n) alloc(h.size());
    if (!h.empty()) staged_upload(p, h.data(), h.size() * sizeof(T), s);
  }
  void zero(hipStream_t s) {
    if (n) ABDDC_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s));
  }
};

// Groups (key, value) pairs by key into CSR arrays (ptr of nkeys + 1, idx),
// values of one key in input order (counting sort).
inline void csr_group(int64_t nkeys, const std::vector<int32_t>& keys, const std::vector<int32_t>& vals,
                      std::vector<int32_t>& ptr, std::vector<int32_t>& idx) {
  ptr.assign(nkeys + 1, 0);
  for (int32_t k : keys) ++ptr[k + 1];
  for (int64_t k = 0; k < nkeys; ++k) ptr[k + 1] += ptr[k];
  idx.assign(keys.size(), 0);
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (size_t i = 0; i < keys.size(); ++i) idx[fill[keys[i]]++] = vals[i];
}

// Stream-ordered host -> device copy through the stream's pinned staging
// ring: the host data is copied out before return, so the caller may free
// it at once; the device copy completes in stream order.
template <class T>
inline DevBuf<T> to_device(const std::vector<T>& h, hipStream_t s) {
  DevBuf<T> d(h.size());
  if (!h.empty()) staged_upload(d.p, h.data(), h.size() * sizeof(T), s);
  return d;
}
template <class T>
inline DevBuf<T> to_device(const T* h, size_t n, hipStream_t s) {
  DevBuf<T> d(n);
  if (n) staged_upload(d.p, h, n * sizeof(T), s);
  return d;
}

template <class T>
inline std::vector<T> to_host(const T* d, size_t n, hipStream_t s) {
  std::vector<T> h(n);
  if (n) {
    ABDDC_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    ABDDC_HIP(hipStreamSynchronize(s));
  }
  return h;
}

// ------------------------------------------------------------ descriptors
// One matrix of a batched in-place partial LU: eliminate the first k pivots
// of an nrow x ncol row-major matrix with leading dimension ld.
template <class T>
struct PluDesc {
  T* a;
  int32_t nrow, ncol, ld, k;
};

// One product of a batched GEMM: C = alpha op(A) op(B) + beta C (row-major).
template <class T>
struct GemmDesc {
  const T* A;
  const T* B;
  T* C;
  int32_t m, n, k, lda, ldb, ldc;
};

// One matrix gather: dst[r][c] = scale * src[rmap[r]][cmap[c]] (map < 0 -> 0,
// null map = identity).
struct GatherDesc {
  const double* src;
  double* dst;
  const int32_t* rmap;
  const int32_t* cmap;
  int32_t nr, nc, lds, ldd;
  double scale;
};

// dst[rows[q]][cols[q]] = val for q < n.
struct SetDesc {
  double* dst;
  const int32_t* rows;
  const int32_t* cols;
  int32_t n, ld;
  double val;
};

// dst = (src + src^T) / 2 (n x n).
struct SymDesc {
  const double* src;
  double* dst;
  int32_t n, lds, ldd;
};

// In place: M22 <- M22 - M21 (sym M11)^+ M12 for the nv x nv matrix M
// (leading dimension ld) whose leading k x k block M11 is eliminated, the
// pseudo-inverse dropping eigenvalues <= rtol lambda_max.
struct SchurPinvDesc {
  double* M;
  int32_t nv, k, ld;
};

// Parallel sum out = sym(A (A + B)^+ B) of two n x n matrices (the face
// operators of Section 3), pseudo-inverse dropping eigenvalues <=
// rtol lambda_max.  A, B: ld lda / ldb; out: ld n.
struct PsumDesc {
  const double* A;
  const double* B;
  double* out;
  int32_t n, lda, ldb;
};

// Householder completion: T (n x n) orthogonal, first p columns span range(X).
struct QrDesc {
  const double* X;
  double* T;
  int32_t n, p, ldx;
};

// Left singular basis of G (n x ncol): T = U sorted by sigma descending,
// rank[0] = #{sigma > rtol sigma_max}.
struct SvdDesc {
  const double* G;
  double* T;
  int32_t* rank;
  int32_t n, ncol, ldg;
};

// Batched symmetric-definite eigenproblem A y = mu B y (n x n, ld n).
struct SygvDesc {
  const double* A;
  const double* B;
  double* w;   // mu ascending
  double* X;   // L Y
  int32_t n;
};

// ---------------------------------------------------------------- launchers
// k_dense.hip
template <class T>
void partial_lu(const std::vector<PluDesc<T>>& d, int* dflag, hipStream_t s);
template <class T>
void gemm_batched(const std::vector<GemmDesc<T>>& d, bool transA, bool transB, T alpha, T beta,
                  hipStream_t s);
void gather_batched(const std::vector<GatherDesc>& d, hipStream_t s);

void set_batched(const std::vector<SetDesc>& d, hipStream_t s);
void sym_batched(const std::vector<SymDesc>& d, hipStream_t s);

// k_eig.hip
void sygv_batched(const std::vector<SygvDesc>& d, int* dflag, hipStream_t s);
// Same outputs, but only the columns of X whose mu <= sel are written.
void sygv_select_batched(const std::vector<SygvDesc>& d, double sel, int* dflag, hipStream_t s);
void parallel_sum_batched(const std::vector<PsumDesc>& d, double rtol, hipStream_t s);
// Matrices the test sends to the eigenvalue fallback need k <= 128; larger
// ones set bit 1 of dflag instead.
void schur_pinv_batched(const std::vector<SchurPinvDesc>& d, double rtol, int* dflag, hipStream_t s);
void qr_complete_batched(const std::vector<QrDesc>& d, hipStream_t s);
void svd_left_batched(const std::vector<SvdDesc>& d, double rtol, hipStream_t s);

}  // namespace abddc
