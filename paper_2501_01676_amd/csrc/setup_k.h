// Setup helper kernel descriptors and launchers (k_setup.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace abddc {

// Largest number of subdomains sharing one edge that the edge stages take.
constexpr int MAX_EDGE_MEMBERS = 8;

struct DeluxeDesc {
  const double* src[8];
  int32_t lds[8];
  double* dst;       // 2n x (m+1)n, ld (m+1)n
  int32_t n, m;
};

struct EdgeAsmDesc {
  const double* D[MAX_EDGE_MEMBERS];    // deluxe blocks n_E x n_E (member order)
  const double* BE[MAX_EDGE_MEMBERS];   // B_E^(k) (original basis), ld ldBE
  const double* Bt[MAX_EDGE_MEMBERS];   // Btilde^(k) over [E; H_k], ld ldBt
  const int32_t* R[MAX_EDGE_MEMBERS];   // positions of H_k in the union
  int32_t ldBE[MAX_EDGE_MEMBERS], ldBt[MAX_EDGE_MEMBERS], nHk[MAX_EDGE_MEMBERS];
  double* ME;            // (m-1) n_E square
  double* Q;             // nv square, nv = m n_E + n_H
  int32_t nE, m, nH, nv;
};

// The metric of the earlier edge eigenproblem for one edge of
// m <= MAX_EDGE_MEMBERS members and n_E <= 32 dofs: out = sym(B_E), B_E = sum_i sum_{k != i}
// D^(k)^T B_E^(i) D^(k) (eq. equ-4-8-E), out n_E x n_E with ld n_E.
struct EdgeOldDesc {
  const double* D[MAX_EDGE_MEMBERS];    // deluxe blocks n_E x n_E (member order)
  const double* BE[MAX_EDGE_MEMBERS];   // B_E^(i), ld ldBE
  int32_t ldBE[MAX_EDGE_MEMBERS];
  double* out;
  int32_t nE, m;
};

// The local constrained system of one subdomain with the averaging folded
// in: Aug = [[Sbar_r, W_r^T], [-W_r, 0]] of order 2 nB, Sbar_r the rotated
// Schur complement with rows and columns in the order am = [Delta; Pi] of
// rotated local coordinates, W_r = W(:, am), W block diagonal by interface
// object (W_X = D_X T_X, n_X x n_X, rows original and columns rotated
// coordinates of the object).  Objects occupy contiguous coordinate ranges;
// slot maps a local coordinate to its object, whose first coordinate, size
// and W_X offset (in wx) are obj_off, obj_n and obj_w.
struct AugDesc {
  const double* sbar;     // nB x nB, ld nB
  void* aug;              // 2 nB x 2 nB, ld 2 nB (double, or float for the FP32 factorisation)
  const int32_t* am;      // nB
  const int32_t* slot;    // nB
  const int32_t* obj_off;
  const int32_t* obj_n;
  const int32_t* obj_w;
  const double* wx;
  int32_t nB;
};

// Rows (rows = 1) or columns (rows = 0) idx[0..nidx) of an n x n matrix
// (ld n) copied from src to dst: the lines a block rotation leaves as they are.
struct LinesDesc {
  const double* src;
  double* dst;
  const int32_t* idx;
  int32_t nidx, n, rows;
};

// M = [L; V] ((nB + nP) x nB, ld nB) and U (nB x nP, ld nP) read off the
// trailing block of an eliminated augmented system (AugDesc layout, nD
// pivots): M(r, c) = Aug(nB + r, nB + c) for r < nB, Aug(nD + r - nB, nB + c)
// below; U(m, l) = -Aug(nB + m, nD + l).  All three in one element type.
struct AugOutDesc {
  const void* aug;
  void* M;
  void* U;
  int32_t nB, nD;
};

// SPi[gid[a]][gid[b]] += src[a][b] (n x n, ld ld); src32 instead of src
// when set.
struct CoarseAddDesc {
  const double* src;
  const int32_t* gid;
  int32_t n, ld;
  const float* src32;
};

struct AxpbyDesc {
  const double* X;
  const double* Y;
  double* dst;
  int32_t nr, nc, ldx, ldy, ldd;
  double alpha, beta;
};

void deluxe_build_batched(const std::vector<DeluxeDesc>& d, hipStream_t s);
void aug_build_batched(const std::vector<AugDesc>& d, bool f32, hipStream_t s);
void aug_extract_batched(const std::vector<AugOutDesc>& d, bool f32, hipStream_t s);
void copy_lines_batched(const std::vector<LinesDesc>& d, hipStream_t s);
void edge_assemble_batched(const std::vector<EdgeAsmDesc>& d, hipStream_t s);
void edge_old_metric_batched(const std::vector<EdgeOldDesc>& d, hipStream_t s);
void coarse_add_batched(const std::vector<CoarseAddDesc>& d, double* SPi, int64_t ldc, hipStream_t s);
void axpby_batched(const std::vector<AxpbyDesc>& d, hipStream_t s);

}  // namespace abddc
