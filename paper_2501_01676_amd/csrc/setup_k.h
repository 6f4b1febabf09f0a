// Setup helper kernel descriptors and launchers (k_setup.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace abddc {

struct DeluxeDesc {
  const double* src[8];
  int32_t lds[8];
  double* dst;       // 2n x (m+1)n, ld (m+1)n
  int32_t n, m;
};

struct EdgeAsmDesc {
  const double* D[4];    // deluxe blocks n_E x n_E (member order)
  const double* BE[4];   // B_E^(k) (original basis), ld ldBE
  const double* Bt[4];   // Btilde^(k) over [E; H_k], ld ldBt
  const int32_t* R[4];   // positions of H_k in the union
  int32_t ldBE[4], ldBt[4], nHk[4];
  double* ME;            // (m-1) n_E square
  double* Q;             // nv square, nv = m n_E + n_H
  int32_t nE, m, nH, nv;
};

// The metric of the earlier edge eigenproblem for one edge of m <= 4 members
// and n_E <= 16 dofs: out = sym(B_E), B_E = sum_i sum_{k != i}
// D^(k)^T B_E^(i) D^(k) (eq. equ-4-8-E), out n_E x n_E with ld n_E.
struct EdgeOldDesc {
  const double* D[4];    // deluxe blocks n_E x n_E (member order)
  const double* BE[4];   // B_E^(i), ld ldBE
  int32_t ldBE[4];
  double* out;
  int32_t nE, m;
};

struct CoarseAddDesc {
  const double* src;
  const int32_t* gid;
  int32_t n, ld;
};

struct AxpbyDesc {
  const double* X;
  const double* Y;
  double* dst;
  int32_t nr, nc, ldx, ldy, ldd;
  double alpha, beta;
};

void convert_f64_f32(const double* src, float* dst, int64_t n, hipStream_t s);
void convert_f32_f64(const float* src, double* dst, int64_t n, hipStream_t s);
void deluxe_build_batched(const std::vector<DeluxeDesc>& d, hipStream_t s);
void edge_assemble_batched(const std::vector<EdgeAsmDesc>& d, hipStream_t s);
void edge_old_metric_batched(const std::vector<EdgeOldDesc>& d, hipStream_t s);
void coarse_add_batched(const std::vector<CoarseAddDesc>& d, double* SPi, int64_t ldc, hipStream_t s);
void axpby_batched(const std::vector<AxpbyDesc>& d, hipStream_t s);

}  // namespace abddc
