// Small dense symmetric eigen / SVD / QR kernels for the face and edge
// eigenproblems (eq. equ-4-8 and equ-5-21), the parallel sum pseudo-inverse
// and the SVD + QR change of basis of the edge constraints.
//
// One workgroup per problem, matrices staged in LDS.  The symmetric solver
// is the cyclic Jacobi method in round-robin (tournament) order: the n/2
// rotations of a round touch disjoint index pairs and are applied together.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>

#include "arena.h"
#include "htrace.h"
#include "internal.h"
#include "tune.h"

namespace abddc {

namespace {

constexpr int NMAX = 64;
// Threads per eigenproblem: the Jacobi rounds are latency-bound chains of
// LDS accesses, so more waves per problem shorten each round.
constexpr int EIG_THREADS = 1024;
constexpr int LDN = NMAX + 1;

// Wave total by DPP: an inclusive scan inside each 16-lane row (row_shr 1,
// 2, 4, 8), then row 0 into row 1 and row 2 into row 3 (row_bcast 15), then
// rows 0-1 into rows 2-3 (row_bcast 31); lane 63 holds the total, which is
// broadcast.  Every lane of the wave must be active.
template <int CTRL, int RMASK>
__device__ inline double dpp_d(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(x & 0xffffffffll), CTRL, RMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, RMASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double wave_total(double v) {
  v += dpp_d<0x111, 0xF>(v);
  v += dpp_d<0x112, 0xF>(v);
  v += dpp_d<0x114, 0xF>(v);
  v += dpp_d<0x118, 0xF>(v);
  v += dpp_d<0x142, 0xA>(v);
  v += dpp_d<0x143, 0xC>(v);
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double wave_sum64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Round-robin pairing of m (even) indices, round r: slot 0 fixed, the other
// m-1 slots rotate.  Returns the index sitting at slot pos.
__device__ inline int rr_slot(int pos, int r, int m) {
  if (pos == 0) return 0;
  return 1 + (pos - 1 + r) % (m - 1);
}

// Jacobi on the symmetric n x n matrix A (LDS, leading dimension NM + 1),
// accumulating the eigenvectors transposed: row p of Vt is eigenvector p
// (Vt starts as identity; LDS or global scratch with leading dimension ldv).
// Cyclic sweeps in round-robin order; a rotation is skipped when |a_pq| is
// negligible against sqrt(|a_pp a_qq|) (relative threshold 1e-16, half the
// double precision unit roundoff) or against the matrix (1e-17 ||A||_F: below the rounding
// noise the rotations themselves leave, which would otherwise keep a
// singular matrix rotating forever), and the iteration stops after a sweep
// without rotations.  The n/2 rotations of a round act on disjoint index pairs, so
// the two-sided update A <- J^T A J splits into independent 2 x 2 blocks
// (pair a rows, pair b columns): block (a, b) becomes J_a^T A_ab J_b.  One
// pass updates every block and the rotated rows of Vt; a round costs two
// barriers (rotation parameters, then the update).
template <int NM>
__device__ int jacobi(double (*A)[NM + 1], double* Vt, int ldv, int n, double* cs, double* sn, int* pp,
                      int* qq, int* nrot) {
  const int tid = threadIdx.x;
  const int m = (n + 1) & ~1;
  const int half = m / 2;
  const int tj = tid & 63, ti = tid >> 6, nstep = blockDim.x >> 6;
  const int bj = tid & 15, bi = tid >> 4, bstep = blockDim.x >> 4;
  __shared__ double fro2;
  if (tid == 0) fro2 = 0.0;
  __syncthreads();
  double part = 0.0;
  for (int r = ti; r < n; r += nstep)
    for (int j = tj; j < n; j += 64) {
      Vt[r * ldv + j] = (r == j) ? 1.0 : 0.0;
      part += A[r][j] * A[r][j];
    }
  part = wave_sum64(part);
  if ((tid & 63) == 0) atomicAdd(&fro2, part);
  if (tid == 0) *nrot = 0;
  __syncthreads();
  const double abs_tol = 1e-17 * sqrt(fro2);
  for (int sweep = 0; sweep < 60; ++sweep) {
    for (int r = 0; r < m - 1; ++r) {
      for (int t = tid; t < half; t += blockDim.x) {
        const int a = rr_slot(t, r, m), b = rr_slot(m - 1 - t, r, m);
        const int p = min(a, b), q = max(a, b);
        double c = 1.0, s = 0.0;
        int active = 0;
        if (q < n) {
          const double apq = A[p][q];
          const double app = A[p][p], aqq = A[q][q];
          if (fabs(apq) > abs_tol && fabs(apq) > 1e-16 * sqrt(fabs(app) * fabs(aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            active = 1;
            atomicAdd(nrot, 1);
          }
        }
        cs[t] = c;
        sn[t] = s;
        pp[t] = p;
        qq[t] = active ? q : -1 - q;   // negative: pair left unrotated
      }
      __syncthreads();
      for (int a = bi; a < half; a += bstep) {
        const int qa_raw = qq[a];
        const int pa = pp[a], qa = qa_raw >= 0 ? qa_raw : -1 - qa_raw;
        const double ca = cs[a], sa = sn[a];
        const bool hasq_a = qa < n;
        for (int b = bj; b < half; b += 16) {
          const int qb_raw = qq[b];
          if (qa_raw < 0 && qb_raw < 0) continue;
          const int pb = pp[b], qb = qb_raw >= 0 ? qb_raw : -1 - qb_raw;
          const double cb = cs[b], sb = sn[b];
          const bool hasq_b = qb < n;
          const double x00 = A[pa][pb];
          const double x01 = hasq_b ? A[pa][qb] : 0.0;
          const double x10 = hasq_a ? A[qa][pb] : 0.0;
          const double x11 = (hasq_a && hasq_b) ? A[qa][qb] : 0.0;
          const double y00 = ca * x00 - sa * x10, y01 = ca * x01 - sa * x11;
          const double y10 = sa * x00 + ca * x10, y11 = sa * x01 + ca * x11;
          double z00 = cb * y00 - sb * y01, z01 = sb * y00 + cb * y01;
          double z10 = cb * y10 - sb * y11, z11 = sb * y10 + cb * y11;
          if (a == b) z01 = z10 = 0.0;   // the rotation annihilates a_pq
          A[pa][pb] = z00;
          if (hasq_b) A[pa][qb] = z01;
          if (hasq_a) A[qa][pb] = z10;
          if (hasq_a && hasq_b) A[qa][qb] = z11;
        }
      }
      for (int t = ti; t < half; t += nstep) {
        const int q = qq[t];
        if (q < 0) continue;
        const int p = pp[t];
        const double c = cs[t], s = sn[t];
        for (int j = tj; j < n; j += 64) {
          const double vp = Vt[p * ldv + j], vq = Vt[q * ldv + j];
          Vt[p * ldv + j] = c * vp - s * vq;
          Vt[q * ldv + j] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
    const int done = (*nrot == 0);
    __syncthreads();
    if (done) return sweep + 1;
    if (tid == 0) *nrot = 0;
    __syncthreads();
  }
  return 60;
}

// Position of eigenvalue i in ascending order (ties by index).
template <int NM>
__device__ inline int rank_of(const double (*A)[NM + 1], int n, int i) {
  const double v = A[i][i];
  int r = 0;
  for (int j = 0; j < n; ++j) {
    const double u = A[j][j];
    r += (u < v) || (u == v && j < i);
  }
  return r;
}

// Per-problem global scratch of the large variants: L and Vt (NM x NM
// each), and for orders above 128 also the working matrix C (NM x (NM + 1)),
// which no longer fits the LDS.
template <int NM>
struct EigScratch {
  static constexpr bool HUGE = NM > 128;
  static constexpr size_t PER = (size_t)2 * NM * NM + (HUGE ? (size_t)NM * (NM + 1) : 0);
  static __device__ inline double* L(double* base) { return base + (size_t)blockIdx.x * PER; }
  static __device__ inline double* V(double* base) { return base + (size_t)blockIdx.x * PER + NM * NM; }
  static __device__ inline double* C(double* base) { return base + (size_t)blockIdx.x * PER + 2 * NM * NM; }
};
constexpr int EIG_HUGE = 512;   // largest order of the global-memory variants

__device__ inline double read_lane_d(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// In-place Cholesky B = L L^T of the lower triangle of L (n <= NM, leading
// dimension ldl), in 16-column panels: wave 0 factors the panel in
// registers (lane = row, NM / 64 rows per lane; pivot and column
// values broadcast by readlane, no barriers), then all threads update the
// trailing lower triangle.  Bit 2 of dflag on a non-positive pivot.
template <int NM>
__device__ __forceinline__ void cholesky_panels(double* L, int ldl, int n, int* dflag) {
  constexpr int RPL = (NM + 63) / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j0 = 0; j0 < n; j0 += 16) {
    const int jw = min(16, n - j0);
    if (wave == 0) {
      double P[RPL][16];
#pragma unroll
      for (int sl = 0; sl < RPL; ++sl) {
        const int r = lane + 64 * sl;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) P[sl][jj] = (r >= j0 && r < n && jj < jw) ? L[r * ldl + j0 + jj] : 0.0;
      }
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        if (jj < jw) {
          const int pr = j0 + jj;
          // row pr sits in slot pr / 64 of lane pr % 64 (a uniform choice)
          double pv = 0.0;
#pragma unroll
          for (int sl = 0; sl < RPL; ++sl)
            if (sl == (pr >> 6)) pv = read_lane_d(P[sl][jj], pr & 63);
          if (lane == 0 && (!(pv > 0.0) || !isfinite(pv))) atomicOr(dflag, 2);
          const double lpp = sqrt(fmax(pv, 1e-300));
          const double inv = 1.0 / lpp;
#pragma unroll
          for (int sl = 0; sl < RPL; ++sl) {
            const int r = lane + 64 * sl;
            if (r == pr) P[sl][jj] = lpp;
            else if (r > pr) P[sl][jj] *= inv;
          }
#pragma unroll
          for (int j2 = jj + 1; j2 < 16; ++j2) {
            if (j2 < jw) {
              const int cr = j0 + j2;
              double lc = 0.0;
#pragma unroll
              for (int sl = 0; sl < RPL; ++sl)
                if (sl == (cr >> 6)) lc = read_lane_d(P[sl][jj], cr & 63);
#pragma unroll
              for (int sl = 0; sl < RPL; ++sl) {
                const int r = lane + 64 * sl;
                if (r >= cr) P[sl][j2] -= P[sl][jj] * lc;
              }
            }
          }
        }
      }
#pragma unroll
      for (int sl = 0; sl < RPL; ++sl) {
        const int r = lane + 64 * sl;
        if (r >= j0 && r < n)
#pragma unroll
          for (int jj = 0; jj < 16; ++jj)
            if (jj < jw && r >= j0 + jj) L[r * ldl + j0 + jj] = P[sl][jj];
      }
    }
    __syncthreads();
    const int j1 = j0 + jw, m = n - j1;
    for (int idx = tid; idx < m * m; idx += blockDim.x) {
      const int r = j1 + idx / m, c = j1 + idx % m;
      if (c > r) continue;
      double a = 0.0;
      for (int q = 0; q < jw; ++q) a += L[r * ldl + j0 + q] * L[c * ldl + j0 + q];
      L[r * ldl + c] -= a;
    }
    __syncthreads();
  }
}

// X <- L^{-1} X for X (n x n, LDS, leading dimension NM + 1) and the lower
// triangular L: 16-row blocks; in each, one thread per column substitutes
// through the block (reciprocal diagonal), then all threads update the rows
// below.
template <int NM>
__device__ __forceinline__ void lower_solve_blocks(const double* L, int ldl, double (*X)[NM + 1], int n) {
  const int tid = threadIdx.x;
  for (int r0 = 0; r0 < n; r0 += 16) {
    const int rw = min(16, n - r0);
    for (int c = tid; c < n; c += blockDim.x) {
      double x[16], rl[16];   // rl: reciprocal pivots, off the substitution chain
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        x[i] = i < rw ? X[r0 + i][c] : 0.0;
        rl[i] = i < rw ? 1.0 / L[(r0 + i) * ldl + r0 + i] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (i < rw) {
          double v = x[i];
#pragma unroll
          for (int q = 0; q < i; ++q) v -= L[(r0 + i) * ldl + r0 + q] * x[q];
          x[i] = v * rl[i];
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i < rw) X[r0 + i][c] = x[i];
    }
    __syncthreads();
    const int r1 = r0 + rw, m = n - r1;
    for (int idx = tid; idx < m * n; idx += blockDim.x) {
      const int r = r1 + idx / n, c = idx % n;
      double a = 0.0;
      for (int q = 0; q < rw; ++q) a += L[r * ldl + r0 + q] * X[r0 + q][c];
      X[r][c] -= a;
    }
    __syncthreads();
  }
}

// Reduction of A y = mu B y (B SPD) to standard form: B = L L^T
// (Cholesky; bit 2 of dflag when B is not positive definite) into L
// (leading dimension ldl), C = L^{-1} A L^{-T} (symmetrised) into Cm:
// W = L^{-1} A, then C = L^{-1} W^T.  With park, the lower triangle of L is
// also copied to the output X, whose LDS space the caller then reuses.
template <int NM>
__device__ __forceinline__ void reduce_pencil(const SygvDesc& d, double (*Cm)[NM + 1], double* L, int ldl, bool park, int* dflag) {
  const int n = d.n, tid = threadIdx.x;
  const int tj = tid & 63, ti = tid >> 6, nstep = blockDim.x >> 6;
  for (int r = ti; r < n; r += nstep)
    for (int j = tj; j < n; j += 64) {
      L[r * ldl + j] = 0.5 * (d.B[r * n + j] + d.B[j * n + r]);
      Cm[r][j] = 0.5 * (d.A[r * n + j] + d.A[j * n + r]);
    }
  __syncthreads();
  cholesky_panels<NM>(L, ldl, n, dflag);
  lower_solve_blocks<NM>(L, ldl, Cm, n);
  for (int idx = tid; idx < n * n; idx += blockDim.x) {   // W -> W^T
    const int r = idx / n, c = idx % n;
    if (r < c) {
      const double t = Cm[r][c];
      Cm[r][c] = Cm[c][r];
      Cm[c][r] = t;
    }
  }
  __syncthreads();
  lower_solve_blocks<NM>(L, ldl, Cm, n);
  for (int r = ti; r < n; r += nstep)
    for (int j = tj; j < n; j += 64) {
      if (r < j) {
        const double v = 0.5 * (Cm[r][j] + Cm[j][r]);
        Cm[r][j] = v;
        Cm[j][r] = v;
      }
      if (park && j <= r) d.X[r * n + j] = L[r * ldl + j];   // park L
    }
  __syncthreads();
}

// A y = mu B y, B SPD: B = L L^T (Cholesky), C = L^{-1} A L^{-T}, Jacobi
// C = Y diag(mu) Y^T, output mu ascending and X = L Y.  NM = 64: two LDS
// matrices, C and one that holds L until C is formed and Vt during Jacobi
// (L is parked in the output X meanwhile and read back into C's place at
// the end); NM = 128: C in LDS, L and Vt in global scratch.
template <int NM>
__global__ void __launch_bounds__(EIG_THREADS) sygv_kernel(const SygvDesc* __restrict__ descs, int* dflag,
                                                   double* __restrict__ scratch) {
  constexpr bool SMALL = NM <= 64;
  __shared__ double Cm[NM][NM + 1];
  __shared__ double LVsm[SMALL ? NM : 1][SMALL ? NM + 1 : 1];
  __shared__ double cs[NM / 2], sn[NM / 2];
  __shared__ int pp[NM / 2], qq[NM / 2];
  __shared__ int rk[NM];
  __shared__ int nrot;
  const SygvDesc d = descs[blockIdx.x];
  const int n = d.n, tid = threadIdx.x;
  if (n <= 0) return;
  double* L = SMALL ? &LVsm[0][0] : EigScratch<NM>::L(scratch);
  double* Vt = SMALL ? &LVsm[0][0] : EigScratch<NM>::V(scratch);
  const int ldl = SMALL ? NM + 1 : NM;
  const int tj = tid & 63, ti = tid >> 6, nstep = blockDim.x >> 6;
  reduce_pencil<NM>(d, Cm, L, ldl, SMALL, dflag);
  jacobi<NM>(Cm, Vt, ldl, n, cs, sn, pp, qq, &nrot);
  // outputs: mu ascending, X[:, rank(i)] = L y_i
  for (int i = tid; i < n; i += blockDim.x) {
    const int ri = rank_of<NM>(Cm, n, i);
    rk[i] = ri;
    d.w[ri] = Cm[i][i];
  }
  __syncthreads();
  if (SMALL) {
    for (int r = ti; r < n; r += nstep)
      for (int j = tj; j <= r; j += 64) Cm[r][j] = d.X[r * n + j];
    __syncthreads();
  }
  const double* Lr = SMALL ? &Cm[0][0] : L;
  const int ldr = SMALL ? NM + 1 : NM;
  for (int i = ti; i < n; i += nstep) {
    const int col = rk[i];
    for (int r = tj; r < n; r += 64) {
      double v = 0.0;
      for (int q = 0; q <= r; ++q) v += Lr[r * ldr + q] * Vt[i * ldl + q];
      d.X[r * n + col] = v;
    }
  }
}

// ------------------------------------------- selected generalized eigenpairs
// A y = mu B y with every eigenvalue but only the eigenvectors of mu <= sel
// (the adaptive constraints of eq. equ-4-8 and equ-5-21 use just those).
// After the reduction C = L^{-1} A L^{-T}:
//   (1) Householder tridiagonalisation C = Q T Q^T (reflectors kept in the
//       columns of C below the subdiagonal);
//   (2) each eigenvalue of T by multisection on the Sturm count (the k-th
//       smallest bracketed directly, so ascending order);
//   (3) for each selected eigenvalue, inverse iteration on T - mu I (LU with
//       partial pivoting of the tridiagonal matrix, three solves), vectors
//       of a cluster (gap below 1e-3 ||T||) orthogonalised against the
//       cluster's earlier ones (modified Gram-Schmidt), clusters in
//       parallel, one wave each;
//   (4) back-transformation z = Q y and output X = L z, as the full solver.
// Work per problem: about (4/3) n^3 for (1), against tens of n^3 for Jacobi.
// Orders the LDS accesses of the lanes of one wave: a wave's LDS operations
// complete in issue order, so a fence at wavefront scope is enough for the
// other lanes to see what one lane wrote.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Householder tridiagonalisation C = Q T Q^T of the symmetric C (LDS) by
// wave 0 alone (the other waves wait at the closing barrier): no block
// barriers inside.  Lane l owns index k+1+l (and k+65+l for NM = 128) of the
// active block of step k.  A step reads x = C[k+1.., k] and the block's
// first column, forms q = C~ x~ (the block and x without their first row
// and entry) row by row, so that the Householder vector, C v and v^T C v
// follow from three wave sums, |x~|^2, x~ . q and x~ . C e0, and from
// alpha = x_0 and c00 (lane 0);
// then the rank-2 update C -= v w^T + w v^T in groups of eight rows (v and
// w staged in sv, sw for broadcast reads).  T's diagonal in dg, off-diagonal in od; reflector k is
// I - tau_k v v^T with v = (1, v_2..) on rows k+1.., its tail kept in
// column k of C below the subdiagonal.
template <int NM>
__device__ __forceinline__ void tridiagonalize(double (*Cm)[NM + 1], int n, double* dg, double* od, double* tau,
                                               double* sv, double* sw) {
  constexpr int RPL = NM / 64;
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid < 64) {
    for (int k = 0; k + 2 < n; ++k) {
      const int m = n - k - 1, b = k + 1;
      // lanes past the block read a clamped (valid) index and are masked
      // where it matters, so that loads are unconditional and can be batched
      double xr[RPL], c0[RPL], q[RPL];
      int cc[RPL], cs[RPL];
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int r = lane + 64 * s;
        cc[s] = b + min(r, m - 1);
        cs[s] = r < m ? b + r : NM;
        const double xv = Cm[cc[s]][k], cv = Cm[cc[s]][b];
        xr[s] = r < m ? xv : 0.0;
        c0[s] = r < m ? cv : 0.0;
        q[s] = 0.0;
      }
#pragma unroll 8
      for (int j = 1; j < m; ++j) {
        const double xj = Cm[b + j][k];
#pragma unroll
        for (int s = 0; s < RPL; ++s) q[s] += Cm[b + j][cc[s]] * xj;
      }
      double acc[3] = {0.0, 0.0, 0.0};   // |x~|^2, x~ . q, x~ . C e0 (lanes 1.. of the block)
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int r = lane + 64 * s;
        const double xm = r > 0 ? xr[s] : 0.0;   // xr is 0 past the block
        acc[0] += xm * xm;
        acc[1] += xm * q[s];
        acc[2] += xm * c0[s];
      }
#pragma unroll
      for (int t = 0; t < 3; ++t) acc[t] = wave_total(acc[t]);
      const double xn2 = acc[0], alpha = read_lane_d(xr[0], 0), c00 = read_lane_d(c0[0], 0);
      const double dkk = Cm[k][k];
      if (xn2 == 0.0) {   // nothing below the subdiagonal: H = I
        if (lane == 0) {
          dg[k] = dkk;
          od[k] = alpha;
          tau[k] = 0.0;
        }
        wave_sync();
        continue;
      }
      const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      const double t = (beta - alpha) / beta, sc = 1.0 / (alpha - beta);
      const double vcv = c00 + 2.0 * sc * acc[2] + sc * sc * acc[1];
      const double K = 0.5 * t * t * vcv;
      if (lane == 0) {
        dg[k] = dkk;
        od[k] = beta;
        tau[k] = t;
      }
      double vv[RPL], ww[RPL];
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int r = lane + 64 * s;
        vv[s] = r < m ? (r == 0 ? 1.0 : sc * xr[s]) : 0.0;
        ww[s] = r < m ? t * (c0[s] + sc * q[s]) - K * vv[s] : 0.0;
        if (r < m) {
          sv[r] = vv[s];
          sw[r] = ww[s];
        }
      }
      wave_sync();
      // rows in groups of eight: every load of a group before its stores
      for (int r0 = 0; r0 < m; r0 += 8) {
        double cv[8][RPL], vr[8], wr[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int rr = min(r0 + u, m - 1);
          vr[u] = sv[rr];
          wr[u] = sw[rr];
#pragma unroll
          for (int s = 0; s < RPL; ++s) cv[u][s] = Cm[b + rr][cc[s]];
        }
        // unconditional stores: a row past the block repeats the last row's
        // store with identical inputs, a lane past the block writes the
        // padding column NM, which holds nothing
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int s = 0; s < RPL; ++s)
            Cm[b + min(r0 + u, m - 1)][cs[s]] = cv[u][s] - (vr[u] * ww[s] + wr[u] * vv[s]);
      }
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int r = lane + 64 * s;
        if (r >= 1 && r < m) Cm[b + r][k] = vv[s];
      }
      wave_sync();
    }
    if (lane == 0) {
      if (n >= 2) {
        dg[n - 2] = Cm[n - 2][n - 2];
        od[n - 2] = Cm[n - 1][n - 2];
        tau[n - 2] = 0.0;
      }
      dg[n - 1] = Cm[n - 1][n - 1];
      od[n - 1] = 0.0;
      tau[n - 1] = 0.0;
    }
  }
  __syncthreads();
}

// Sturm count at x: the number of negative ratios q_i = p_i / p_{i-1} of
// consecutive leading principal minors of T - x I, p_i = (d_i - x) p_{i-1}
// - e_{i-1}^2 p_{i-2}, which is the number of eigenvalues below x.  Carried
// as minors, not ratios, so a step costs two multiply-adds instead of a
// division; a ratio of magnitude below pivmin is replaced by -pivmin, and
// every eight steps the pair (p_{i-1}, p_i) is rescaled by a power of two,
// which keeps it in range without changing a sign or a ratio.  Needs the
// squared off-diagonal e2 and the padding of tri_prepare_sturm: the last
// group of eight steps runs past n on decoupled diagonal entries above
// every x, which change no sign, so no step needs a branch.
__device__ inline int sturm_count(const double* dg, const double* e2, int n, double x, double pivmin) {
  double pm = 1.0, pc = dg[0] - x;
  if (fabs(pc) < pivmin) pc = -pivmin;
  int cnt = pc < 0.0;
  for (int i0 = 1; i0 < n; i0 += 8) {
    double dv[8], ev[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      dv[u] = dg[i0 + u];
      ev[u] = e2[i0 + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      double pn = (dv[u] - x) * pc - ev[u] * pm;
      if (fabs(pn) < pivmin * fabs(pc)) pn = -pivmin * pc;
      cnt += (int)(((unsigned)__double2hiint(pn) ^ (unsigned)__double2hiint(pc)) >> 31);   // sign change
      pm = pc;
      pc = pn;
    }
    int ex;
    frexp(fmax(fabs(pm), fabs(pc)), &ex);
    pm = ldexp(pm, -ex);
    pc = ldexp(pc, -ex);
  }
  return cnt;
}

// Gershgorin interval of T, widened by the rounding allowance, and the
// pivot floor of the Sturm count.
struct TriBounds {
  double lo, hi, tnorm, pivmin, atol;
};

__device__ inline TriBounds tri_bounds(const double* dg, const double* od, int n) {
  double glo = 0.0, ghi = 0.0, emax2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? fabs(od[i - 1]) : 0.0) + (i + 1 < n ? fabs(od[i]) : 0.0);
    glo = i == 0 ? dg[i] - r : fmin(glo, dg[i] - r);
    ghi = i == 0 ? dg[i] + r : fmax(ghi, dg[i] + r);
    if (i + 1 < n) emax2 = fmax(emax2, od[i] * od[i]);
  }
  const double eps = 1.1102230246251565e-16;   // 2^-53
  TriBounds b;
  b.tnorm = fmax(fabs(glo), fabs(ghi));
  b.pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2) / eps;
  b.lo = glo - (2.0 * eps * b.tnorm + 2.0 * b.pivmin);
  b.hi = ghi + (2.0 * eps * b.tnorm + 2.0 * b.pivmin);
  b.atol = 2.0 * eps * b.tnorm + 4.0 * b.pivmin;
  return b;
}

// e2[i] = e_i^2 (zero from n - 1 on) and eight diagonal entries past n
// set above the Gershgorin interval, for sturm_count.  dg and e2 hold n + 8
// entries.  All threads; a barrier must follow.
__device__ inline void tri_prepare_sturm(double* dg, const double* od, double* e2, int n) {
  const TriBounds tb = tri_bounds(dg, od, n);
  const double pad = tb.hi + (tb.hi - tb.lo) + 1.0;
  for (int i = threadIdx.x; i < n + 8; i += blockDim.x) {
    if (i >= n) dg[i] = pad;
    e2[i] = i + 1 < n ? od[i] * od[i] : 0.0;
  }
}

// The eigenvalues e0 <= e < e1 of the tridiagonal T (the e-th smallest into
// lam[e]) by multisection on the Sturm count (after tri_prepare_sturm): G threads per eigenvalue (a
// power of two up to 64 with G (e1 - e0) <= 256: about one wave per SIMD,
// since a second wave on a SIMD costs nearly as much as the rounds it
// saves), one point each, so a round cuts the bracket into G + 1 pieces; the e-th
// smallest eigenvalue is bracketed directly.  Stops at 2 eps max(||T||,
// |lambda|).
__device__ inline void bisect_range(const double* dg, const double* od, const double* e2, int n, int e0, int e1,
                                    double* lam) {
  const int tid = threadIdx.x, ne = e1 - e0;
  if (ne <= 0) return;
  const TriBounds tb = tri_bounds(dg, od, n);
  const double eps = 1.1102230246251565e-16;   // 2^-53
  int G = 1;
  while (G < 64 && 2 * G * ne <= min(256, (int)blockDim.x)) G *= 2;
  const int e = e0 + tid / G, g = tid % G;
  if (e >= e1) return;
  double lo = tb.lo, hi = tb.hi;
  for (int round = 0; round < 200; ++round) {
    if (hi - lo <= fmax(tb.atol, 2.0 * eps * fmax(fabs(lo), fabs(hi)))) break;
    const double h = (hi - lo) / (double)(G + 1);
    const double x = lo + (double)(g + 1) * h;
    const int cnt = sturm_count(dg, e2, n, x, tb.pivmin);
    double nlo = lo, nhi = hi;
    if (x > lo && x < hi) {
      if (cnt > e) nhi = x;
      else nlo = x;
    }
    for (int o = G / 2; o > 0; o >>= 1) {
      nlo = fmax(nlo, __shfl_xor(nlo, o, G));
      nhi = fmin(nhi, __shfl_xor(nhi, o, G));
    }
    if (nhi - nlo >= hi - lo) break;   // no progress left in floating point
    lo = nlo;
    hi = nhi;
  }
  if (g == 0) lam[e] = 0.5 * (lo + hi);
}

// Ascending order of v[e0..e1) into out[e0..e1) (out != v), by ranks:
// equal eigenvalues may come out of the multisection a rounding apart in
// either order.
__device__ inline void rank_sort(const double* v, int e0, int e1, double* out) {
  for (int t = e0 + (int)threadIdx.x; t < e1; t += blockDim.x) {
    const double x = v[t];
    int r = e0;
    for (int j = e0; j < e1; ++j) {
      const double u = v[j];
      r += (u < x) || (u == x && j < t);
    }
    out[r] = x;
  }
}

__device__ inline double tri_norm_inf(const double* dg, const double* od, int n) {
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i)
    tnorm = fmax(tnorm, fabs(dg[i]) + (i > 0 ? fabs(od[i - 1]) : 0.0) + (i + 1 < n ? fabs(od[i]) : 0.0));
  return tnorm;
}

// Shared-memory arrays of the tridiagonal eigen-pipeline: dg, od, e2, tau,
// q1, lam (NM doubles each, NM + 8 for dg and e2), and nslot inverse-iteration slots of five
// NM-double arrays (U's diagonal and two superdiagonals, the multipliers,
// the iterate) and NM pivot flags.
struct TriArrays {
  double *dg, *od, *e2, *tau, *q1, *lam;   // dg and e2: NM + 8 entries
  double* inv;   // nslot x 5 x nm
  int* ipiv;     // nslot x nm
  int nslot, nm;
};

// Eigenvalues of the symmetric C (LDS, order n): tridiagonalisation (C
// keeps the reflectors), multisection, ascending order into w.lam.  Returns
// ||T||_inf.
template <int NM>
__device__ __forceinline__ double tri_eigenvalues(double (*C)[NM + 1], int n, const TriArrays& w) {
  tridiagonalize<NM>(C, n, w.dg, w.od, w.tau, w.q1, w.lam);
  tri_prepare_sturm(w.dg, w.od, w.e2, n);
  __syncthreads();
  bisect_range(w.dg, w.od, w.e2, n, 0, n, w.q1);
  __syncthreads();
  rank_sort(w.q1, 0, n, w.lam);
  __syncthreads();
  return tri_norm_inf(w.dg, w.od, n);
}

// Eigenvectors of T for the p smallest eigenvalues by inverse iteration
// (rows of Z, leading dimension ldz, tridiagonal coordinates).  Clusters
// (runs of eigenvalues with gaps <= 1e-3 ||T||) are independent: wave w <
// nslot takes the clusters w, w + nslot, ..., and inside a cluster computes
// the vectors in order, each orthogonalised against the cluster's earlier
// ones by modified Gram-Schmidt after every solve.  Lane 0 runs the serial
// recurrences (LU with partial pivoting of T - lam_j I, three rounds of the
// two triangular solves), reading their inputs eight entries at a time; the
// wave shares the reciprocal pivots, dot products and scaling.
__device__ inline void tri_vectors(int n, int p, double tnorm, const TriArrays& w, double* Z, int ldz) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double eps = 1.1102230246251565e-16;   // 2^-53
  const double ortol = 1e-3 * tnorm;
  if (wv < w.nslot && n > 0) {
    double* ud = w.inv + (size_t)wv * 5 * w.nm;   // reciprocal pivots after the factorisation
    double* u1 = ud + w.nm;
    double* u2 = u1 + w.nm;
    double* ml = u2 + w.nm;
    double* yv = ml + w.nm;
    int* pivs = w.ipiv + wv * w.nm;
    int cl = -1, c0 = 0;
    for (int j = 0; j < p; ++j) {
      if (j == 0 || w.lam[j] - w.lam[j - 1] > ortol) {   // j opens a cluster
        ++cl;
        c0 = j;
      }
      if (cl % w.nslot != wv) continue;
      const double x = w.lam[j];
      if (lane == 0) {
        // row i of U: diagonal ud, superdiagonals u1, u2; multipliers ml,
        // row interchanges pivs.  Full groups of eight steps without
        // branches, their inputs loaded first; the tail one step at a time.
        double a = w.dg[0] - x, b = n > 1 ? w.od[0] : 0.0;
        auto lu_step = [&](int i, double c, double a1, double b1) {
          const bool sw = fabs(a) < fabs(c);
          const double pv = sw ? c : a, qv = sw ? a : c;
          const double l = pv != 0.0 ? qv / pv : 0.0;
          ud[i] = pv;
          u1[i] = sw ? a1 : b;
          u2[i] = sw ? b1 : 0.0;
          ml[i] = l;
          pivs[i] = sw;
          const double na = sw ? b - l * a1 : a1 - l * b;
          b = sw ? -l * b1 : b1;
          a = na;
        };
        int i = 0;
        for (; i + 8 < n; i += 8) {
          double cv[8], av[8], bv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            cv[u] = w.od[i + u];
            av[u] = w.dg[i + u + 1] - x;
            bv[u] = i + u + 2 < n ? w.od[i + u + 1] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) lu_step(i + u, cv[u], av[u], bv[u]);
        }
        for (; i + 1 < n; ++i) lu_step(i, w.od[i], w.dg[i + 1] - x, i + 2 < n ? w.od[i + 1] : 0.0);
        ud[n - 1] = a; u1[n - 1] = 0.0; u2[n - 1] = 0.0;
        // start vector: a fixed pseudo-random sequence in (-1, 1)
        unsigned st = 0x9E3779B9u * (unsigned)(j + 1);
        for (int i = 0; i < n; ++i) {
          st = st * 1664525u + 1013904223u;
          yv[i] = ((double)(st >> 8) / 16777216.0) * 2.0 - 1.0;
        }
      }
      wave_sync();
      const double tiny = eps * (tnorm > 0.0 ? tnorm : 1.0);
      for (int i = lane; i < n; i += 64) {
        const double u = fabs(ud[i]) < tiny ? (ud[i] < 0.0 ? -tiny : tiny) : ud[i];
        ud[i] = 1.0 / u;
      }
      wave_sync();
      for (int it = 0; it < 3; ++it) {
        if (lane == 0) {
          // forward: interchanges and multipliers, row i + 1 carried in a register
          double cur = yv[0];
          auto fw_step = [&](int i, double nx, double mv, int pv) {
            yv[i] = pv ? nx : cur;
            cur = pv ? cur - mv * nx : nx - mv * cur;
          };
          int i = 0;
          for (; i + 8 < n; i += 8) {
            double nx[8], mv[8];
            int pv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              nx[u] = yv[i + u + 1];
              mv[u] = ml[i + u];
              pv[u] = pivs[i + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) fw_step(i + u, nx[u], mv[u], pv[u]);
          }
          for (; i + 1 < n; ++i) fw_step(i, yv[i + 1], ml[i], pivs[i]);
          yv[n - 1] = cur;
          // back substitution with the three bands of U (reciprocal pivots);
          // near-singular shifts make the solution grow by 1/tiny per small
          // pivot, so the whole system is rescaled before it could overflow
          double c1 = 0.0, c2 = 0.0;
          auto bk_step = [&](int i, double y, double a1, double a2, double rp, double* pend, int npend) {
            double v = (y - a1 * c1 - a2 * c2) * rp;
            for (int g = 0; g < 4 && !(fabs(v) <= 1e150); ++g) {
              for (int q = 0; q < n; ++q) yv[q] *= 1e-150;
              for (int q = 0; q < npend; ++q) pend[q] *= 1e-150;   // loaded, not yet used
              y *= 1e-150;
              c1 *= 1e-150;
              c2 *= 1e-150;
              v = (y - a1 * c1 - a2 * c2) * rp;
            }
            yv[i] = v;
            c2 = c1;
            c1 = v;
          };
          int i1 = n - 1;
          for (; i1 - 7 >= 0; i1 -= 8) {
            double yb[8], a1[8], a2[8], rp[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              yb[u] = yv[i1 - u];
              a1[u] = u1[i1 - u];
              a2[u] = u2[i1 - u];
              rp[u] = ud[i1 - u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) bk_step(i1 - u, yb[u], a1[u], a2[u], rp[u], yb + u + 1, 7 - u);
          }
          for (; i1 >= 0; --i1) bk_step(i1, yv[i1], u1[i1], u2[i1], ud[i1], nullptr, 0);
        }
        wave_sync();
        // orthogonalise against the cluster's earlier vectors, normalise
        for (int q = c0; q < j; ++q) {
          double part = 0.0;
          for (int i = lane; i < n; i += 64) part += Z[q * ldz + i] * yv[i];
          const double dq = wave_total(part);
          for (int i = lane; i < n; i += 64) yv[i] -= dq * Z[q * ldz + i];
        }
        double part = 0.0;
        for (int i = lane; i < n; i += 64) part += yv[i] * yv[i];
        const double nrm = sqrt(wave_total(part));
        const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        for (int i = lane; i < n; i += 64) yv[i] *= inv;
        wave_sync();
      }
      for (int i = lane; i < n; i += 64) Z[j * ldz + i] = yv[i];
      wave_sync();
    }
  }
  __syncthreads();
}

// z = H_0 H_1 ... H_{n-3} y for the p rows of Z: each wave takes whole
// vectors, holds one in registers (lane l owns the entries l and l + 64)
// and applies the reflectors from the last to the first (no block
// barriers).
template <int NM>
__device__ __forceinline__ void tri_back_transform(const double (*C)[NM + 1], const double* tau, int n, int p,
                                                   double* Z, int ldz) {
  constexpr int RPL = NM / 64;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, nw = blockDim.x >> 6;
  for (int j = wv; j < p; j += nw) {
    double* z = Z + (size_t)j * ldz;
    double zr[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int i = lane + 64 * s;
      zr[s] = i < n ? z[i] : 0.0;
    }
    for (int k = n - 3; k >= 0; --k) {
      const double tk = tau[k];
      if (tk == 0.0) continue;
      double hv[RPL];
      double part = 0.0;
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int i = lane + 64 * s;
        hv[s] = (i > k + 1 && i < n) ? C[i][k] : (i == k + 1 ? 1.0 : 0.0);
        part += hv[s] * zr[s];
      }
      const double f = tk * wave_total(part);
#pragma unroll
      for (int s = 0; s < RPL; ++s) zr[s] -= f * hv[s];
    }
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int i = lane + 64 * s;
      if (i < n) z[i] = zr[s];
    }
  }
  __syncthreads();
}

// LDS of the pipeline for order NM and NT threads: two inverse-iteration
// slots for NM = 64 (clusters are few; this keeps a workgroup under 80 KB of
// LDS, so two share a CU), a single slot for NM = 128 (whose matrix takes
// most of the LDS).
#define TRI_SHARED(NM, NT)                                                                     \
  constexpr int TRI_NSLOT = (NM) <= 64 ? 2 : 1;                                                \
  __shared__ double dg_[(NM) + 8], od_[NM], e2_[(NM) + 8], tau_[NM], q1_[NM], lam_[NM],            \
      inv_[TRI_NSLOT * 5 * (NM)];                                                              \
  __shared__ int ipiv_[TRI_NSLOT * (NM)];                                                      \
  const TriArrays tw{dg_, od_, e2_, tau_, q1_, lam_, inv_, ipiv_, TRI_NSLOT, NM};

template <int NM, int NT>
__global__ void __launch_bounds__(NT) sygv_sel_kernel(const SygvDesc* __restrict__ descs, double sel, int* dflag,
                                                      double* __restrict__ scratch) {
  constexpr bool SMALL = NM <= 64;
  constexpr bool HUGE = NM > 128;
  __shared__ double CmL[HUGE ? 1 : NM][HUGE ? 1 : NM + 1];
  double(*Cm)[NM + 1] = HUGE ? reinterpret_cast<double(*)[NM + 1]>(EigScratch<NM>::C(scratch))
                             : reinterpret_cast<double(*)[NM + 1]>(&CmL[0][0]);
  __shared__ double LZsm[SMALL ? NM : 1][SMALL ? NM + 1 : 1];
  TRI_SHARED(NM, NT)
  const SygvDesc d = descs[blockIdx.x];
  const int n = d.n, tid = threadIdx.x;
  if (n <= 0) return;
  double* L = SMALL ? &LZsm[0][0] : EigScratch<NM>::L(scratch);
  const int ldl = SMALL ? NM + 1 : NM;
  reduce_pencil<NM>(d, Cm, L, ldl, SMALL, dflag);
  // Z: selected vectors (row j = vector j), LDS for the small variant
  double* Z = SMALL ? &LZsm[0][0] : EigScratch<NM>::V(scratch);
  const int ldz = SMALL ? NM + 1 : NM;
  const double tnorm = tri_eigenvalues<NM>(Cm, n, tw);
  for (int t = tid; t < n; t += blockDim.x) d.w[t] = tw.lam[t];
  int p = 0;
  while (p < n && tw.lam[p] <= sel) ++p;
  tri_vectors(n, p, tnorm, tw, Z, ldz);
  tri_back_transform<NM>(Cm, tw.tau, n, p, Z, ldz);
  // X[:, j] = L z_j (L read back into Cm for the small variant)
  if (SMALL) {
    const int tj = tid & 63, ti = tid >> 6, nstep = blockDim.x >> 6;
    for (int r = ti; r < n; r += nstep)
      for (int j = tj; j <= r; j += 64) Cm[r][j] = d.X[r * n + j];
    __syncthreads();
  }
  const double* Lr = SMALL ? &Cm[0][0] : L;
  const int ldr = SMALL ? NM + 1 : NM;
  for (int idx = tid; idx < n * p; idx += blockDim.x) {
    const int r = idx / p, j = idx - r * p;
    double v = 0.0;
    for (int q = 0; q <= r; ++q) v += Lr[r * ldr + q] * Z[j * ldz + q];
    d.X[r * n + j] = v;
  }
}

// ------------------------------------- Schur complement with pseudo-inverse
// M22 - M21 (sym M11)^+ M12 for M = [[M11, M12], [M21, M22]] (M11 of order
// k), the pseudo-inverse dropping eigenvalues <= rtol lambda_max.  When
// M11 is positive definite with ||M11||_F ||M11^{-1}||_F < 1 / rtol (that
// product bounds lambda_max / lambda_min), the pseudo-inverse keeps every
// eigenvalue and equals M11^{-1}: one partial LU of
//   [[M11, M12, I], [M21, M22, 0], [-I, 0, 0]]
// gives the Schur complement and, in its last block, M11^{-1} for the test
// (positive pivots = positive definite, M11 being symmetric up to
// rounding).  A matrix that fails is flagged and takes the eigenvalue
// pseudo-inverse (Jacobi) instead.  The result overwrites M22.

struct SchurWork {
  SchurPinvDesc d;
  double* G;      // (nv + k)^2 augmented matrix, ld nv + k
  double* work;   // k x nv (fallback: dropped eigenvectors, then M'^{-1} M12)
  int32_t* flag;  // 1: take the fallback
};

__global__ void __launch_bounds__(256) spinv_build_kernel(const SchurWork* __restrict__ ws) {
  const SchurWork w = ws[blockIdx.x];
  const int nv = w.d.nv, k = w.d.k, ng = nv + k;
  for (int idx = threadIdx.x; idx < ng * ng; idx += blockDim.x) {
    const int r = idx / ng, c = idx - r * ng;
    double v;
    if (r < nv) v = c < nv ? w.d.M[(size_t)r * w.d.ld + c] : ((r < k && c - nv == r) ? 1.0 : 0.0);
    else v = (c < k && r - nv == c) ? -1.0 : 0.0;
    w.G[idx] = v;
  }
}

__device__ inline double block_sum256(double v, double* red) {
  v = wave_total(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) spinv_finish_kernel(const SchurWork* __restrict__ ws, double rtol, int* dflag) {
  __shared__ double red[4];
  __shared__ int bad;
  const SchurWork w = ws[blockIdx.x];
  const int nv = w.d.nv, k = w.d.k, ng = nv + k, m = nv - k;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double fs = 0.0, fi = 0.0;
  for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) {
    const int i = idx / k, j = idx - i * k;
    const double sv = w.d.M[(size_t)i * w.d.ld + j];
    const double iv = w.G[(size_t)(nv + i) * ng + nv + j];
    fs += sv * sv;
    fi += iv * iv;
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x)
    if (!(w.G[(size_t)i * ng + i] > 0.0)) bad = 1;   // a non-positive pivot: not positive definite
  fs = block_sum256(fs, red);
  __syncthreads();
  fi = block_sum256(fi, red);
  const double prod = sqrt(fs) * sqrt(fi);
  const bool ok = !bad && isfinite(prod) && prod * rtol < 1.0;
  if (threadIdx.x == 0) {
    *w.flag = ok ? 0 : 1;
    if (!ok && k > 128) atomicOr(dflag, 1);
  }
  if (!ok) return;
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
    const int i = idx / m, j = idx - i * m;
    w.d.M[(size_t)(k + i) * w.d.ld + k + j] = w.G[(size_t)(k + i) * ng + k + j];
  }
}

// X <- (L L^T)^{-1} X for the Cholesky factor L (LDS, lower triangle) and
// X (k x m, LDS or global, leading dimension ldx): blocked forward and backward
// substitution, one thread per column inside a 16-row block, all threads
// on the update of the remaining rows.
template <int NM>
__device__ __forceinline__ void chol_solve(const double (*Lm)[NM + 1], int k, double* X, int ldx, int m) {
  const int tid = threadIdx.x;
  for (int r0 = 0; r0 < k; r0 += 16) {
    const int rw = min(16, k - r0);
    for (int c = tid; c < m; c += blockDim.x) {
      double x[16], rl[16];   // rl: reciprocal pivots, off the substitution chain
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        x[i] = i < rw ? X[(size_t)(r0 + i) * ldx + c] : 0.0;
        rl[i] = i < rw ? 1.0 / Lm[r0 + i][r0 + i] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i < rw) {
          double v = x[i];
#pragma unroll
          for (int q = 0; q < i; ++q) v -= Lm[r0 + i][r0 + q] * x[q];
          x[i] = v * rl[i];
        }
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i < rw) X[(size_t)(r0 + i) * ldx + c] = x[i];
    }
    __syncthreads();
    const int r1 = r0 + rw, mr = k - r1;
    for (int idx = tid; idx < mr * m; idx += blockDim.x) {
      const int r = r1 + idx / m, c = idx % m;
      double acc = 0.0;
      for (int q = 0; q < rw; ++q) acc += Lm[r][r0 + q] * X[(size_t)(r0 + q) * ldx + c];
      X[(size_t)r * ldx + c] -= acc;
    }
    __syncthreads();
  }
  for (int r0 = ((k - 1) / 16) * 16; r0 >= 0; r0 -= 16) {
    const int rw = min(16, k - r0);
    for (int c = tid; c < m; c += blockDim.x) {
      double x[16], rl[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        x[i] = i < rw ? X[(size_t)(r0 + i) * ldx + c] : 0.0;
        rl[i] = i < rw ? 1.0 / Lm[r0 + i][r0 + i] : 0.0;
      }
#pragma unroll
      for (int i = 15; i >= 0; --i)
        if (i < rw) {
          double v = x[i];
#pragma unroll
          for (int q = i + 1; q < 16; ++q)
            if (q < rw) v -= Lm[r0 + q][r0 + i] * x[q];
          x[i] = v * rl[i];
        }
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i < rw) X[(size_t)(r0 + i) * ldx + c] = x[i];
    }
    __syncthreads();
    for (int idx = tid; idx < r0 * m; idx += blockDim.x) {
      const int r = idx / m, c = idx % m;
      double acc = 0.0;
      for (int q = 0; q < rw; ++q) acc += Lm[r0 + q][r] * X[(size_t)(r0 + q) * ldx + c];
      X[(size_t)r * ldx + c] -= acc;
    }
    __syncthreads();
  }
}

// Second half of the fallback: X = M12 (k x m, leading dimension ldx),
// projected off V_d (rows of Vd, each staged in the LDS array vs of NM
// doubles), solved with M' = L L^T (L in Am), then M22 -= M21 X, with M21
// staged in Am when it fits.
template <int NM>
__device__ __forceinline__ void spinv_fallback_apply(double (*Am)[NM + 1], double* M, int ld, int k, int m,
                                                     const double* Vd, int pd, double* X, int ldx, double* vs) {
  const int tid = threadIdx.x, tj = tid & 63, ti = tid >> 6, nstep = blockDim.x >> 6;
  for (int idx = tid; idx < k * m; idx += blockDim.x) {
    const int r = idx / m, c = idx - r * m;
    X[(size_t)r * ldx + c] = M[(size_t)r * ld + k + c];
  }
  __syncthreads();
  for (int q = 0; q < pd; ++q) {
    for (int i = tid; i < k; i += blockDim.x) vs[i] = Vd[(size_t)q * k + i];
    __syncthreads();
    for (int c = tid; c < m; c += blockDim.x) {
      double t = 0.0;
      for (int i = 0; i < k; ++i) t += vs[i] * X[(size_t)i * ldx + c];
      for (int i = 0; i < k; ++i) X[(size_t)i * ldx + c] -= vs[i] * t;
    }
    __syncthreads();
  }
  chol_solve<NM>(Am, k, X, ldx, m);
  const bool stage = m <= NM;
  if (stage) {
    for (int r = ti; r < m; r += nstep)
      for (int j = tj; j < k; j += 64) Am[r][j] = M[(size_t)(k + r) * ld + j];
    __syncthreads();
  }
  for (int idx = tid; idx < m * m; idx += blockDim.x) {
    const int r = idx / m, c = idx - r * m;
    double acc = 0.0;
    if (stage)
      for (int q = 0; q < k; ++q) acc += Am[r][q] * X[(size_t)q * ldx + c];
    else
      for (int q = 0; q < k; ++q) acc += M[(size_t)(k + r) * ld + q] * X[(size_t)q * ldx + c];
    M[(size_t)(k + r) * ld + k + c] -= acc;
  }
}

// Fallback for flagged matrices, by deflation: sym(M11) has the
// eigenvalues lambda and the dropped ones (<= rtol lambda_max) span V_d.
// With sigma = lambda_max, M' = sym(M11) + V_d (sigma - Lambda_d) V_d^T is
// positive definite with M'^{-1} V_d = V_d / sigma, so
//   (sym M11)^+ M12 = M'^{-1} M12 - V_d V_d^T M12 / sigma
//                   = M'^{-1} (I - V_d V_d^T) M12:
// M12 is projected off V_d and solved with the Cholesky factor of M'.  Of
// the spectrum only lambda_max, the number of dropped eigenvalues (a Sturm
// count at the cut) and the dropped eigenvalues are computed, V_d by
// inverse iteration on the tridiagonal form.  For NM = 64 the right-hand
// side lives in LDS.
template <int NM, int NT>
__global__ void __launch_bounds__(NT) spinv_fallback_kernel(const SchurWork* __restrict__ ws, double rtol,
                                                            int* dflag) {
  constexpr bool XL = NM <= 64;
  __shared__ double Am[NM][NM + 1];
  __shared__ double Xs[XL ? NM : 1][XL ? NM + 1 : 1];
  TRI_SHARED(NM, NT)
  __shared__ int pd_s;
  const SchurWork w = ws[blockIdx.x];
  const int nv = w.d.nv, k = w.d.k, m = nv - k, ld = w.d.ld, tid = threadIdx.x;
  if (k <= 0 || *w.flag == 0) return;
  double* M = w.d.M;
  double* Vd = w.work;   // dropped eigenvectors, rows, ld k
  const int tj = tid & 63, ti = tid >> 6, nstep = blockDim.x >> 6;
  for (int r = ti; r < k; r += nstep)
    for (int j = tj; j < k; j += 64) Am[r][j] = 0.5 * (M[(size_t)r * ld + j] + M[(size_t)j * ld + r]);
  __syncthreads();
  tridiagonalize<NM>(Am, k, tw.dg, tw.od, tw.tau, tw.q1, tw.lam);
  tri_prepare_sturm(tw.dg, tw.od, tw.e2, k);
  __syncthreads();
  bisect_range(tw.dg, tw.od, tw.e2, k, k - 1, k, tw.lam);
  __syncthreads();
  const double lmax = tw.lam[k - 1];
  if (!(lmax > 0.0)) return;   // nothing kept: the pseudo-inverse is 0
  const double cut = rtol * lmax;
  if (tid == 0) pd_s = min(k - 1, sturm_count(tw.dg, tw.e2, k, cut, tri_bounds(tw.dg, tw.od, k).pivmin));
  __syncthreads();
  const int pd = pd_s;
  bisect_range(tw.dg, tw.od, tw.e2, k, 0, pd, tw.q1);
  __syncthreads();
  rank_sort(tw.q1, 0, pd, tw.lam);
  __syncthreads();
  tri_vectors(k, pd, tri_norm_inf(tw.dg, tw.od, k), tw, Vd, k);
  tri_back_transform<NM>(Am, tw.tau, k, pd, Vd, k);
  // M' in Am, then its Cholesky factor
  for (int r = ti; r < k; r += nstep)
    for (int j = tj; j < k; j += 64) {
      double v = 0.5 * (M[(size_t)r * ld + j] + M[(size_t)j * ld + r]);
      for (int q = 0; q < pd; ++q) v += (lmax - tw.lam[q]) * Vd[(size_t)q * k + r] * Vd[(size_t)q * k + j];
      Am[r][j] = v;
    }
  __syncthreads();
  cholesky_panels<NM>(&Am[0][0], NM + 1, k, dflag);
  if (XL && m <= NM)
    spinv_fallback_apply<NM>(Am, M, ld, k, m, Vd, pd, &Xs[0][0], NM + 1, tw.q1);
  else
    spinv_fallback_apply<NM>(Am, M, ld, k, m, Vd, pd, w.work + (size_t)k * k, m, tw.q1);
}

// Parallel sum pieces: [[A + B, B], [-A, 0]] (its pseudo-inverse Schur
// complement is A (A + B)^+ B), and out = sym of that block.
__global__ void __launch_bounds__(256) psum_pack_kernel(const PsumDesc* __restrict__ ds, double* __restrict__ buf,
                                                        const int64_t* __restrict__ off) {
  const PsumDesc d = ds[blockIdx.x];
  const int n = d.n, n2 = 2 * n;
  double* M = buf + off[blockIdx.x];
  for (int idx = threadIdx.x; idx < n2 * n2; idx += blockDim.x) {
    const int r = idx / n2, c = idx - r * n2;
    double v = 0.0;
    if (r < n) v = c < n ? d.A[r * d.lda + c] + d.B[r * d.ldb + c] : d.B[r * d.ldb + c - n];
    else if (c < n) v = -d.A[(r - n) * d.lda + c];
    M[idx] = v;
  }
}

__global__ void __launch_bounds__(256) psum_sym_kernel(const PsumDesc* __restrict__ ds, const double* __restrict__ buf,
                                                       const int64_t* __restrict__ off) {
  const PsumDesc d = ds[blockIdx.x];
  const int n = d.n, n2 = 2 * n;
  const double* T = buf + off[blockIdx.x] + (size_t)n * n2 + n;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx - i * n;
    d.out[idx] = 0.5 * (T[(size_t)i * n2 + j] + T[(size_t)j * n2 + i]);
  }
}

// Householder QR of X (n x p), accumulated into Q = H_0 H_1 ... H_{p-1}
// (X copy and Q in LDS for NM = 64, in global scratch / the output for 128).
template <int NM>
__global__ void __launch_bounds__(256) qr_complete_kernel(const QrDesc* __restrict__ descs,
                                                          double* __restrict__ scratch) {
  constexpr bool SMALL = NM <= 64;
  __shared__ double Xsm[SMALL ? NM : 1][SMALL ? NM + 1 : 1];
  __shared__ double Qsm[SMALL ? NM : 1][SMALL ? NM + 1 : 1];
  __shared__ double v[NM];
  __shared__ double tau_s;
  const QrDesc d = descs[blockIdx.x];
  const int n = d.n, p = d.p, tid = threadIdx.x;
  const int ld = SMALL ? NM + 1 : NM;
  double* X = SMALL ? &Xsm[0][0] : scratch + (size_t)blockIdx.x * NM * NM;
  double* Q = SMALL ? &Qsm[0][0] : d.T;
  const int ldq = SMALL ? NM + 1 : n;
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int r = idx / n, c = idx % n;
    Q[r * ldq + c] = (r == c) ? 1.0 : 0.0;
    if (c < p) X[r * ld + c] = d.X[r * d.ldx + c];
  }
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    if (tid == 0) {
      double nrm2 = 0.0;
      for (int i = j; i < n; ++i) nrm2 += X[i * ld + j] * X[i * ld + j];
      const double x0 = X[j * ld + j];
      const double alpha = (x0 >= 0 ? -1.0 : 1.0) * sqrt(nrm2);
      for (int i = 0; i < n; ++i) v[i] = (i < j) ? 0.0 : X[i * ld + j];
      v[j] = x0 - alpha;
      const double vn2 = nrm2 - x0 * x0 + v[j] * v[j];
      tau_s = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
    }
    __syncthreads();
    const double tau = tau_s;
    for (int c = j + tid; c < p; c += blockDim.x) {
      double dsum = 0.0;
      for (int i = j; i < n; ++i) dsum += v[i] * X[i * ld + c];
      for (int i = j; i < n; ++i) X[i * ld + c] -= tau * dsum * v[i];
    }
    for (int r = tid; r < n; r += blockDim.x) {
      double dsum = 0.0;
      for (int i = j; i < n; ++i) dsum += Q[r * ldq + i] * v[i];
      for (int i = j; i < n; ++i) Q[r * ldq + i] -= tau * dsum * v[i];
    }
    __syncthreads();
  }
  if (SMALL)
    for (int idx = tid; idx < n * n; idx += blockDim.x) d.T[idx] = Q[(idx / n) * ldq + idx % n];
}

// One-sided Jacobi on the rows of G: G = U diag(sigma) W^T, U accumulated.
// RMAX: the largest n_E of the instance.
template <int RMAX>
__global__ void __launch_bounds__(64) svd_left_kernel(const SvdDesc* __restrict__ descs, double rtol) {
  constexpr int CMAX = 256;
  __shared__ double Gm[RMAX][CMAX];
  __shared__ double Um[RMAX][RMAX];
  __shared__ double sig[RMAX];
  const SvdDesc d = descs[blockIdx.x];
  const int n = d.n, nc = d.ncol, lane = threadIdx.x;
  for (int idx = lane; idx < n * n; idx += 64) Um[idx / n][idx % n] = (idx / n == idx % n) ? 1.0 : 0.0;
  for (int idx = lane; idx < n * nc; idx += 64) Gm[idx / nc][idx % nc] = d.G[(idx / nc) * d.ldg + idx % nc];
  __syncthreads();
  for (int sweep = 0; sweep < 40 && nc > 0; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double a = 0.0, b = 0.0, g = 0.0;
        for (int k = lane; k < nc; k += 64) {
          a += Gm[p][k] * Gm[p][k];
          b += Gm[q][k] * Gm[q][k];
          g += Gm[p][k] * Gm[q][k];
        }
        a = wave_sum64(a);
        b = wave_sum64(b);
        g = wave_sum64(g);
        a = __shfl(a, 0, 64);
        b = __shfl(b, 0, 64);
        g = __shfl(g, 0, 64);
        if (fabs(g) <= 1e-15 * sqrt(a * b) || g == 0.0) continue;
        rotated = true;
        const double tau = (b - a) / (2.0 * g);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        for (int k = lane; k < nc; k += 64) {
          const double gp = Gm[p][k], gq = Gm[q][k];
          Gm[p][k] = c * gp - s * gq;
          Gm[q][k] = s * gp + c * gq;
        }
        for (int r = lane; r < n; r += 64) {
          const double up = Um[r][p], uq = Um[r][q];
          Um[r][p] = c * up - s * uq;
          Um[r][q] = s * up + c * uq;
        }
        __syncthreads();
      }
    if (!rotated) break;
  }
  for (int i = 0; i < n; ++i) {
    double a = 0.0;
    for (int k = lane; k < nc; k += 64) a += Gm[i][k] * Gm[i][k];
    a = wave_sum64(a);
    if (lane == 0) sig[i] = sqrt(a);
  }
  __syncthreads();
  double smax = 0.0;
  for (int i = 0; i < n; ++i) smax = fmax(smax, sig[i]);
  // descending order of sigma, ties by index
  for (int i = lane; i < n; i += 64) {
    int r = 0;
    for (int j = 0; j < n; ++j) r += (sig[j] > sig[i]) || (sig[j] == sig[i] && j < i);
    for (int row = 0; row < n; ++row) d.T[row * n + r] = Um[row][i];
  }
  if (lane == 0) {
    int rk = 0;
    if (smax > 0.0)
      for (int i = 0; i < n; ++i) rk += sig[i] > rtol * smax;
    d.rank[0] = rk;
  }
}

}  // namespace

namespace {
// Threads per eigenproblem: small orders have few rotations per round, and
// a round costs two barriers, so fewer waves can be faster; many problems in
// a batch also favour fewer waves each.  The autotuner picks among these
// per (kernel, order bucket, batch bucket); ABDDC_EIG_THREADS forces one.
constexpr int EIG_VARIANTS[3] = {64, 256, 1024};

template <class Launch>
int eig_threads(const char* name, int nmax, size_t batch, Launch launch, hipStream_t s) {
  const char* force = std::getenv("ABDDC_EIG_THREADS");
  if (force)
    for (int v : EIG_VARIANTS)
      if (std::atoi(force) == v) return v;
  int dev = 0;
  ABDDC_HIP(hipGetDevice(&dev));
  const std::string key = device_arch(dev) + "|" + name + "|n" + std::to_string(size_bucket(nmax)) + "|b" +
                          std::to_string(size_bucket((long long)batch));
  const int cached = tune_lookup(key);
  if (cached >= 0 && cached < 3) return EIG_VARIANTS[cached];
  hipEvent_t e0, e1;
  ABDDC_HIP(hipEventCreate(&e0));
  ABDDC_HIP(hipEventCreate(&e1));
  int best = 2;
  float best_ms = 0.f;
  for (int v = 0; v < 3; ++v) {
    launch(EIG_VARIANTS[v]);   // warm-up; every launch recomputes the same outputs
    ABDDC_HIP(hipEventRecord(e0, s));
    launch(EIG_VARIANTS[v]);
    launch(EIG_VARIANTS[v]);
    ABDDC_HIP(hipEventRecord(e1, s));
    ABDDC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    ABDDC_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (v == 0 || ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tune_store(key, best);
  return EIG_VARIANTS[best];
}

// Split a descriptor list by order: n <= 64 (LDS variant), 64 < n <= 128,
// and, where a caller takes them (huge != nullptr), 128 < n <= EIG_HUGE.
template <class D, class F>
void split_launch(const std::vector<D>& descs, F order, hipStream_t s, const char* what,
                  std::vector<D>& small, std::vector<D>& big, std::vector<D>* huge = nullptr) {
  const int limit = huge ? EIG_HUGE : 128;
  for (auto& d : descs) {
    const int n = order(d);
    ABDDC_REQUIRE(n <= limit, ABDDC_EINVAL, std::string(what) + ": matrix order exceeds " + std::to_string(limit));
    (n <= 64 ? small : (n <= 128 ? big : *huge)).push_back(d);
  }
  // largest problems first (ragged batches): they are dispatched first
  auto by_size = [&](const D& a, const D& b) { return order(a) > order(b); };
  std::stable_sort(small.begin(), small.end(), by_size);
  std::stable_sort(big.begin(), big.end(), by_size);
  if (huge) std::stable_sort(huge->begin(), huge->end(), by_size);
  (void)s;
}
}  // namespace

void schur_pinv_batched(const std::vector<SchurPinvDesc>& descs, double rtol, int* dflag, hipStream_t s) {
  if (descs.empty()) return;
  HostTrace ht;
  int64_t gtot = 0, wtot = 0;
  for (auto& d : descs) {
    ABDDC_REQUIRE(d.k >= 0 && d.k <= d.nv && d.ld >= d.nv, ABDDC_EINVAL, "pinv Schur complement: bad shape");
    gtot += (int64_t)(d.nv + d.k) * (d.nv + d.k);
    wtot += (int64_t)d.k * d.nv;   // V_d (k x k) and X (k x (nv - k))
  }
  const int nb = (int)descs.size();
  DevBuf<double> G(std::max<int64_t>(gtot, 1)), work(std::max<int64_t>(wtot, 1));
  DevBuf<int32_t> flags(nb), lu_flag(1);
  lu_flag.zero(s);
  ht.mark("pinv Schur: buffers");
  std::vector<SchurWork> ws(nb);
  std::vector<PluDesc<double>> pd(nb);
  int64_t go = 0, wo = 0;
  for (int b = 0; b < nb; ++b) {
    const int ng = descs[b].nv + descs[b].k;
    ws[b] = {descs[b], G.p + go, work.p + wo, flags.p + b};
    pd[b] = {G.p + go, ng, ng, ng, descs[b].k};
    go += (int64_t)ng * ng;
    wo += (int64_t)descs[b].k * descs[b].nv;
  }
  Arena& ar = Arena::for_stream(s);
  const SchurWork* dw = ar.put(ws);
  spinv_build_kernel<<<nb, 256, 0, s>>>(dw);
  ht.mark("pinv Schur: descriptors, build");
  // a zero or non-finite pivot only sends the matrix to the fallback: the
  // finish kernel sees a non-positive pivot or a non-finite ||M11^{-1}||
  partial_lu<double>(pd, lu_flag.p, s);
  ht.mark("pinv Schur: partial LU queued");
  spinv_finish_kernel<<<nb, 256, 0, s>>>(dw, rtol, dflag);
  // the eigenvalue fallback exists for k <= 128; a larger block that fails
  // the test is reported through dflag by the finish kernel
  std::vector<SchurWork> small_k;
  for (auto& w : ws)
    if (w.d.k <= 128) small_k.push_back(w);
  std::vector<SchurWork> sm, bg;
  split_launch(small_k, [](const SchurWork& w) { return w.d.k; }, s, "pinv Schur complement", sm, bg);
  if (!sm.empty()) {
    const SchurWork* dd = ar.put(sm);
    spinv_fallback_kernel<64, 512><<<sm.size(), 512, 0, s>>>(dd, rtol, dflag);
  }
  if (!bg.empty()) {
    const SchurWork* dd = ar.put(bg);
    spinv_fallback_kernel<128, 1024><<<bg.size(), 1024, 0, s>>>(dd, rtol, dflag);
  }
  ABDDC_HIP(hipGetLastError());
  ht.mark("pinv Schur: finish, fallback queued");
}

void parallel_sum_batched(const std::vector<PsumDesc>& descs, double rtol, hipStream_t s) {
  if (descs.empty()) return;
  const int nb = (int)descs.size();
  std::vector<int64_t> off(nb);
  int64_t tot = 0;
  for (int b = 0; b < nb; ++b) {
    ABDDC_REQUIRE(descs[b].n >= 1 && descs[b].n <= EIG_HUGE, ABDDC_EINVAL, "parallel sum: order outside [1, 512]");
    off[b] = tot;
    tot += (int64_t)4 * descs[b].n * descs[b].n;
  }
  DevBuf<double> M(tot);
  Arena& ar = Arena::for_stream(s);
  const PsumDesc* dd = ar.put(descs);
  const int64_t* doff = ar.put(off);
  psum_pack_kernel<<<nb, 256, 0, s>>>(dd, M.p, doff);
  std::vector<SchurPinvDesc> sd(nb);
  for (int b = 0; b < nb; ++b) sd[b] = {M.p + off[b], 2 * descs[b].n, descs[b].n, 2 * descs[b].n};
  DevBuf<int> unused(1);
  schur_pinv_batched(sd, rtol, unused.p, s);
  psum_sym_kernel<<<nb, 256, 0, s>>>(dd, M.p, doff);
  ABDDC_HIP(hipGetLastError());
}

void sygv_select_batched(const std::vector<SygvDesc>& descs, double sel, int* dflag, hipStream_t s) {
  std::vector<SygvDesc> sm, bg, hg;
  split_launch(descs, [](const SygvDesc& d) { return d.n; }, s, "sygv", sm, bg, &hg);
  if (!hg.empty()) {
    DevBuf<double> scr(hg.size() * EigScratch<EIG_HUGE>::PER);
    const SygvDesc* dd = Arena::for_stream(s).put(hg);
    sygv_sel_kernel<EIG_HUGE, 512><<<hg.size(), 512, 0, s>>>(dd, sel, dflag, scr.p);
  }
  if (!sm.empty()) {
    const SygvDesc* dd = Arena::for_stream(s).put(sm);
    sygv_sel_kernel<64, 512><<<sm.size(), 512, 0, s>>>(dd, sel, dflag, nullptr);
  }
  if (!bg.empty()) {
    DevBuf<double> scr(bg.size() * 2 * 128 * 128);
    const SygvDesc* dd = Arena::for_stream(s).put(bg);
    sygv_sel_kernel<128, 1024><<<bg.size(), 1024, 0, s>>>(dd, sel, dflag, scr.p);
  }
  ABDDC_HIP(hipGetLastError());
}

void qr_complete_batched(const std::vector<QrDesc>& descs, hipStream_t s) {
  std::vector<QrDesc> sm, bg, hg;
  split_launch(descs, [](const QrDesc& d) { return d.n; }, s, "qr", sm, bg, &hg);
  if (!hg.empty()) {
    DevBuf<double> scr(hg.size() * (size_t)EIG_HUGE * EIG_HUGE);
    const QrDesc* dd = Arena::for_stream(s).put(hg);
    qr_complete_kernel<EIG_HUGE><<<hg.size(), 256, 0, s>>>(dd, scr.p);
  }
  if (!sm.empty()) {
    const QrDesc* dd = Arena::for_stream(s).put(sm);
    qr_complete_kernel<64><<<sm.size(), 256, 0, s>>>(dd, nullptr);
  }
  if (!bg.empty()) {
    DevBuf<double> scr(bg.size() * 128 * 128);
    const QrDesc* dd = Arena::for_stream(s).put(bg);
    qr_complete_kernel<128><<<bg.size(), 256, 0, s>>>(dd, scr.p);
  }
  ABDDC_HIP(hipGetLastError());
}

void svd_left_batched(const std::vector<SvdDesc>& descs, double rtol, hipStream_t s) {
  if (descs.empty()) return;
  int nmax = 0;
  for (auto& d : descs) {
    ABDDC_REQUIRE(d.n <= 32 && d.ncol <= 256, ABDDC_EINVAL, "svd: edge block too large");
    nmax = std::max(nmax, d.n);
  }
  const SvdDesc* dd = Arena::for_stream(s).put(descs);
  if (nmax <= 16) svd_left_kernel<16><<<descs.size(), 64, 0, s>>>(dd, rtol);
  else svd_left_kernel<32><<<descs.size(), 64, 0, s>>>(dd, rtol);
  ABDDC_HIP(hipGetLastError());
}

void sygv_batched(const std::vector<SygvDesc>& descs, int* dflag, hipStream_t s) {
  std::vector<SygvDesc> sm, bg;
  split_launch(descs, [](const SygvDesc& d) { return d.n; }, s, "sygv", sm, bg);
  if (!sm.empty()) {
    const SygvDesc* dd = Arena::for_stream(s).put(sm);
    int nmax = 0;
    for (auto& d : sm) nmax = std::max(nmax, d.n);
    auto go = [&](int th) { sygv_kernel<64><<<sm.size(), th, 0, s>>>(dd, dflag, nullptr); };
    go(eig_threads("sygv", nmax, sm.size(), go, s));
  }
  if (!bg.empty()) {
    DevBuf<double> scr(bg.size() * 2 * 128 * 128);
    const SygvDesc* dd = Arena::for_stream(s).put(bg);
    sygv_kernel<128><<<bg.size(), EIG_THREADS, 0, s>>>(dd, dflag, scr.p);
  }
  ABDDC_HIP(hipGetLastError());
}

}  // namespace abddc
