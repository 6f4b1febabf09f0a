// C ABI: error reporting and the batched-primitive test hooks.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "guard.h"
#include "internal.h"
#include "kstats.h"

namespace abddc {
thread_local std::string g_last_error;
thread_local KStats* g_kstats = nullptr;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
}  // namespace abddc

using namespace abddc;

extern "C" const char* abddc_last_error(void) { return g_last_error.c_str(); }

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
    DevBuf<int> flag(1);
    flag.zero(s);
    std::vector<SygvDesc> d(batch);
    for (int b = 0; b < batch; ++b) d[b] = {buf + offA[b], buf + offB[b], buf + offW[b], buf + offX[b], n[b]};
    sygv_batched(d, flag.p, s);
    return check_flag(flag.p, s);
  });
}
