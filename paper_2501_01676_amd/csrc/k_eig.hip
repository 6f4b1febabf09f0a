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
#include "internal.h"
#include "tune.h"

namespace abddc {

namespace {

constexpr int NMAX = 64;
// Threads per eigenproblem: the Jacobi rounds are latency-bound chains of
// LDS accesses, so more waves per problem shorten each round.
constexpr int EIG_THREADS = 1024;
constexpr int LDN = NMAX + 1;

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

// Per-problem global scratch for the large variant: L and Vt (NM x NM each).
template <int NM>
struct EigScratch {
  static __device__ inline double* L(double* base) { return base + (size_t)blockIdx.x * 2 * NM * NM; }
  static __device__ inline double* V(double* base) { return base + (size_t)blockIdx.x * 2 * NM * NM + NM * NM; }
};

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
  for (int r = ti; r < n; r += nstep)
    for (int j = tj; j < n; j += 64) {
      L[r * ldl + j] = 0.5 * (d.B[r * n + j] + d.B[j * n + r]);
      Cm[r][j] = 0.5 * (d.A[r * n + j] + d.A[j * n + r]);
    }
  __syncthreads();
  // right-looking Cholesky, lower triangle
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double djj = L[j * ldl + j];
      if (!(djj > 0.0) || !isfinite(djj)) atomicOr(dflag, 2);
      L[j * ldl + j] = sqrt(fmax(djj, 1e-300));
    }
    __syncthreads();
    const double ljj = L[j * ldl + j];
    for (int i = j + 1 + tid; i < n; i += blockDim.x) L[i * ldl + j] /= ljj;
    __syncthreads();
    for (int c = j + 1 + tj; c < n; c += 64) {
      const double lc = L[c * ldl + j];
      for (int i = j + 1 + ti; i < n; i += nstep)
        if (i >= c) L[i * ldl + c] -= L[i * ldl + j] * lc;
    }
    __syncthreads();
  }
  // W = L^{-1} A (columns in place), then Z = L^{-1} W^T (rows of W in
  // place).  Sixteen lanes share one column (row): lane l sums the terms
  // q = l mod 16 of each substitution step and writes the solved entries
  // r = l mod 16, so every value a lane reads back is one it wrote itself.
  {
    const int g = tid >> 4, l = tid & 15, ng = blockDim.x >> 4;
    for (int c = g; c < n; c += ng)
      for (int r = 0; r < n; ++r) {
        double part = 0.0;
        for (int q = l; q < r; q += 16) part += L[r * ldl + q] * Cm[q][c];
        for (int m = 8; m > 0; m >>= 1) part += __shfl_xor(part, m, 16);
        const double v = (Cm[r][c] - part) / L[r * ldl + r];
        if ((r & 15) == l) Cm[r][c] = v;
      }
    __syncthreads();
    for (int jr = g; jr < n; jr += ng)
      for (int r = 0; r < n; ++r) {
        double part = 0.0;
        for (int q = l; q < r; q += 16) part += L[r * ldl + q] * Cm[jr][q];
        for (int m = 8; m > 0; m >>= 1) part += __shfl_xor(part, m, 16);
        const double v = (Cm[jr][r] - part) / L[r * ldl + r];
        if ((r & 15) == l) Cm[jr][r] = v;
      }
    __syncthreads();
  }
  for (int r = ti; r < n; r += nstep)
    for (int j = tj; j < n; j += 64) {
      if (r < j) {
        const double v = 0.5 * (Cm[r][j] + Cm[j][r]);
        Cm[r][j] = v;
        Cm[j][r] = v;
      }
      if (SMALL && j <= r) d.X[r * n + j] = L[r * ldl + j];   // park L
    }
  __syncthreads();
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

// out = sum over kept eigenpairs of v v^T / lambda (lambda > rtol lambda_max)
template <int NM>
__global__ void __launch_bounds__(EIG_THREADS) pinv_kernel(const PinvDesc* __restrict__ descs, double rtol,
                                                   double* __restrict__ scratch) {
  constexpr bool SMALL = NM <= 64;
  __shared__ double Am[NM][NM + 1];
  __shared__ double Vsm[SMALL ? NM : 1][SMALL ? NM + 1 : 1];
  __shared__ double cs[NM / 2], sn[NM / 2];
  __shared__ int pp[NM / 2], qq[NM / 2];
  __shared__ int nrot;
  __shared__ double lmax;
  const PinvDesc d = descs[blockIdx.x];
  const int n = d.n, tid = threadIdx.x;
  if (n <= 0) return;
  double* Vt = SMALL ? &Vsm[0][0] : EigScratch<NM>::V(scratch);
  const int ldv = SMALL ? NM + 1 : NM;
  const int tj = tid & 63, ti = tid >> 6, nstep = blockDim.x >> 6;
  for (int r = ti; r < n; r += nstep)
    for (int j = tj; j < n; j += 64) Am[r][j] = 0.5 * (d.M[r * d.ld + j] + d.M[j * d.ld + r]);
  __syncthreads();
  jacobi<NM>(Am, Vt, ldv, n, cs, sn, pp, qq, &nrot);
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = fmax(mx, Am[i][i]);
    lmax = mx;
  }
  __syncthreads();
  const double cut = rtol * lmax;
  for (int r = ti; r < n; r += nstep)
    for (int j = tj; j < n; j += 64) {
      double v = 0.0;
      if (lmax > 0.0)
        for (int k = 0; k < n; ++k) {
          const double lam = Am[k][k];
          if (lam > cut) v += Vt[k * ldv + r] * Vt[k * ldv + j] / lam;
        }
      d.out[r * d.ld + j] = v;
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
__global__ void __launch_bounds__(64) svd_left_kernel(const SvdDesc* __restrict__ descs, double rtol) {
  constexpr int RMAX = 16, CMAX = 256;
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

// Split a descriptor list by order: n <= 64 (LDS variant) and 64 < n <= 128.
template <class D, class F>
void split_launch(const std::vector<D>& descs, F order, hipStream_t s, const char* what,
                  std::vector<D>& small, std::vector<D>& big) {
  for (auto& d : descs) {
    const int n = order(d);
    ABDDC_REQUIRE(n <= 128, ABDDC_EINVAL, std::string(what) + ": matrix order exceeds 128");
    (n <= 64 ? small : big).push_back(d);
  }
  // largest problems first (ragged batches): they are dispatched first
  auto by_size = [&](const D& a, const D& b) { return order(a) > order(b); };
  std::stable_sort(small.begin(), small.end(), by_size);
  std::stable_sort(big.begin(), big.end(), by_size);
  (void)s;
}
}  // namespace

void pinv_batched(const std::vector<PinvDesc>& descs, double rtol, hipStream_t s) {
  std::vector<PinvDesc> sm, bg;
  split_launch(descs, [](const PinvDesc& d) { return d.n; }, s, "pinv", sm, bg);
  if (!sm.empty()) {
    const PinvDesc* dd = Arena::for_stream(s).put(sm);
    int nmax = 0;
    for (auto& d : sm) nmax = std::max(nmax, d.n);
    auto go = [&](int th) { pinv_kernel<64><<<sm.size(), th, 0, s>>>(dd, rtol, nullptr); };
    go(eig_threads("pinv", nmax, sm.size(), go, s));
  }
  if (!bg.empty()) {
    DevBuf<double> scr(bg.size() * 2 * 128 * 128);
    const PinvDesc* dd = Arena::for_stream(s).put(bg);
    pinv_kernel<128><<<bg.size(), EIG_THREADS, 0, s>>>(dd, rtol, scr.p);
  }
  ABDDC_HIP(hipGetLastError());
}

void qr_complete_batched(const std::vector<QrDesc>& descs, hipStream_t s) {
  std::vector<QrDesc> sm, bg;
  split_launch(descs, [](const QrDesc& d) { return d.n; }, s, "qr", sm, bg);
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
  for (auto& d : descs) ABDDC_REQUIRE(d.n <= 16 && d.ncol <= 256, ABDDC_EINVAL, "svd: edge block too large");
  const SvdDesc* dd = Arena::for_stream(s).put(descs);
  svd_left_kernel<<<descs.size(), 64, 0, s>>>(dd, rtol);
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
