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

#include "arena.h"
#include "internal.h"

namespace abddc {

namespace {

constexpr int NMAX = 64;
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

// Jacobi on the symmetric n x n matrix in A (LDS), accumulating V (LDS,
// starts as identity).  Index n (when n is odd) is a dummy that never
// rotates.  Returns after convergence or 40 sweeps.
__device__ void jacobi_lds(double (*A)[LDN], double (*V)[LDN], int n, double* cs, double* sn,
                           int* pp, int* qq, int* nrot) {
  const int tid = threadIdx.x;
  const int m = (n + 1) & ~1;
  const int half = m / 2;
  const int tj = tid & 63, ti = tid >> 6, nstep = blockDim.x >> 6;
  if (tj < n)
    for (int r = ti; r < n; r += nstep) V[r][tj] = (r == tj) ? 1.0 : 0.0;
  if (tid == 0) *nrot = 0;
  __syncthreads();
  // Cyclic sweeps; a rotation is skipped when |a_pq| is negligible against
  // sqrt(|a_pp a_qq|) (relative threshold 1e-18 below double precision), and
  // the iteration stops after a sweep without rotations.
  for (int sweep = 0; sweep < 60; ++sweep) {
    for (int r = 0; r < m - 1; ++r) {
      if (tid < half) {
        int a = rr_slot(tid, r, m), b = rr_slot(m - 1 - tid, r, m);
        int p = min(a, b), q = max(a, b);
        double c = 1.0, s = 0.0;
        int active = 0;
        if (q < n) {
          const double apq = A[p][q];
          const double app = A[p][p], aqq = A[q][q];
          if (apq != 0.0 && fabs(apq) > 1e-18 * sqrt(fabs(app) * fabs(aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            active = 1;
            atomicAdd(nrot, 1);
          }
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = p;
        qq[tid] = active ? q : n;   // inactive pairs are skipped below
      }
      __syncthreads();
      // rows: A <- J^T A   (pair i = ti, ti + nstep, ...; element j = tj)
      for (int i = ti; i < half && tj < n; i += nstep) {
        const int p = pp[i], q = qq[i], j = tj;
        if (q >= n) continue;
        const double c = cs[i], s = sn[i];
        const double ap = A[p][j], aq = A[q][j];
        A[p][j] = c * ap - s * aq;
        A[q][j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int i = ti; i < half && tj < n; i += nstep) {
        const int p = pp[i], q = qq[i], j = tj;
        if (q >= n) continue;
        const double c = cs[i], s = sn[i];
        const double ap = A[j][p], aq = A[j][q];
        A[j][p] = c * ap - s * aq;
        A[j][q] = s * ap + c * aq;
        const double vp = V[j][p], vq = V[j][q];
        V[j][p] = c * vp - s * vq;
        V[j][q] = s * vp + c * vq;
      }
      __syncthreads();
      // the rotation annihilates a_pq
      if (tid < half && qq[tid] < n) {
        A[pp[tid]][qq[tid]] = 0.0;
        A[qq[tid]][pp[tid]] = 0.0;
      }
      __syncthreads();
    }
    const int done = (*nrot == 0);
    __syncthreads();
    if (done) break;
    if (tid == 0) *nrot = 0;
    __syncthreads();
  }
}

// Position of eigenvalue i in ascending order (ties by index).
__device__ inline int rank_of(const double (*A)[LDN], int n, int i) {
  const double v = A[i][i];
  int r = 0;
  for (int j = 0; j < n; ++j) {
    const double u = A[j][j];
    r += (u < v) || (u == v && j < i);
  }
  return r;
}

// A y = mu B y, B SPD: B = L L^T (Cholesky in LDS), C = L^{-1} A L^{-T},
// Jacobi C = Y diag(mu) Y^T, output mu ascending and X = L Y.
__global__ void __launch_bounds__(256) sygv_kernel(const SygvDesc* __restrict__ descs, int* dflag) {
  __shared__ double Lm[NMAX][LDN];
  __shared__ double Cm[NMAX][LDN];
  __shared__ double Vm[NMAX][LDN];
  __shared__ double cs[NMAX / 2], sn[NMAX / 2];
  __shared__ int pp[NMAX / 2], qq[NMAX / 2];
  __shared__ int nrot;
  const SygvDesc d = descs[blockIdx.x];
  const int n = d.n, tid = threadIdx.x;
  if (n <= 0) return;
  const int tj = tid & 63, ti = tid >> 6, nstep = blockDim.x >> 6;
  if (tj < n)
    for (int r = ti; r < n; r += nstep) {
      Lm[r][tj] = 0.5 * (d.B[r * n + tj] + d.B[tj * n + r]);
      Cm[r][tj] = 0.5 * (d.A[r * n + tj] + d.A[tj * n + r]);
    }
  __syncthreads();
  // right-looking Cholesky, lower triangle
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double djj = Lm[j][j];
      if (!(djj > 0.0) || !isfinite(djj)) atomicOr(dflag, 2);
      Lm[j][j] = sqrt(fmax(djj, 1e-300));
    }
    __syncthreads();
    const double ljj = Lm[j][j];
    for (int i = j + 1 + tid; i < n; i += blockDim.x) Lm[i][j] /= ljj;
    __syncthreads();
    if (tj > j && tj < n) {
      const double lc = Lm[tj][j];
      for (int i = j + 1 + ti; i < n; i += nstep)
        if (tj <= i) Lm[i][tj] -= Lm[i][j] * lc;
    }
    __syncthreads();
  }
  // W = L^{-1} A (columns in place), then Z = L^{-1} W^T (rows of W in place)
  if (tid < n) {
    const int c = tid;
    for (int r = 0; r < n; ++r) {
      double v = Cm[r][c];
      for (int q = 0; q < r; ++q) v -= Lm[r][q] * Cm[q][c];
      Cm[r][c] = v / Lm[r][r];
    }
  }
  __syncthreads();
  if (tid < n) {
    const int j = tid;
    for (int r = 0; r < n; ++r) {
      double v = Cm[j][r];
      for (int q = 0; q < r; ++q) v -= Lm[r][q] * Cm[j][q];
      Cm[j][r] = v / Lm[r][r];
    }
  }
  __syncthreads();
  if (tj < n)
    for (int r = ti; r < tj; r += nstep) {
      const double v = 0.5 * (Cm[r][tj] + Cm[tj][r]);
      Cm[r][tj] = v;
      Cm[tj][r] = v;
    }
  __syncthreads();
  jacobi_lds(Cm, Vm, n, cs, sn, pp, qq, &nrot);
  // outputs: mu ascending, X[:, rank] = L Y[:, i]
  for (int i = tid; i < n; i += blockDim.x) d.w[rank_of(Cm, n, i)] = Cm[i][i];
  if (tj < n) {
    const int col = rank_of(Cm, n, tj);
    for (int r = ti; r < n; r += nstep) {
      double v = 0.0;
      for (int q = 0; q <= r; ++q) v += Lm[r][q] * Vm[q][tj];
      d.X[r * n + col] = v;
    }
  }
}

// out = sum over kept eigenpairs of v v^T / lambda (lambda > rtol lambda_max)
__global__ void __launch_bounds__(256) pinv_kernel(const PinvDesc* __restrict__ descs, double rtol) {
  __shared__ double Am[NMAX][LDN];
  __shared__ double Vm[NMAX][LDN];
  __shared__ double cs[NMAX / 2], sn[NMAX / 2];
  __shared__ int pp[NMAX / 2], qq[NMAX / 2];
  __shared__ int nrot;
  __shared__ double lmax;
  const PinvDesc d = descs[blockIdx.x];
  const int n = d.n, tid = threadIdx.x;
  if (n <= 0) return;
  const int tj = tid & 63, ti = tid >> 6, nstep = blockDim.x >> 6;
  if (tj < n)
    for (int r = ti; r < n; r += nstep) Am[r][tj] = 0.5 * (d.M[r * d.ld + tj] + d.M[tj * d.ld + r]);
  __syncthreads();
  jacobi_lds(Am, Vm, n, cs, sn, pp, qq, &nrot);
  if (tid == 0) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fmax(m, Am[i][i]);
    lmax = m;
  }
  __syncthreads();
  const double cut = rtol * lmax;
  if (tj < n)
    for (int r = ti; r < n; r += nstep) {
      double v = 0.0;
      if (lmax > 0.0)
        for (int k = 0; k < n; ++k) {
          const double lam = Am[k][k];
          if (lam > cut) v += Vm[r][k] * Vm[tj][k] / lam;
        }
      d.out[r * d.ld + tj] = v;
    }
}

// Householder QR of X (n x p), accumulated into Q = H_0 H_1 ... H_{p-1}.
__global__ void __launch_bounds__(256) qr_complete_kernel(const QrDesc* __restrict__ descs) {
  __shared__ double Xm[NMAX][LDN];
  __shared__ double Qm[NMAX][LDN];
  __shared__ double v[NMAX];
  __shared__ double tau_s;
  const QrDesc d = descs[blockIdx.x];
  const int n = d.n, p = d.p, tid = threadIdx.x;
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int r = idx / n, c = idx % n;
    Qm[r][c] = (r == c) ? 1.0 : 0.0;
    if (c < p) Xm[r][c] = d.X[r * d.ldx + c];
  }
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    if (tid == 0) {
      double nrm2 = 0.0;
      for (int i = j; i < n; ++i) nrm2 += Xm[i][j] * Xm[i][j];
      const double x0 = Xm[j][j];
      const double alpha = (x0 >= 0 ? -1.0 : 1.0) * sqrt(nrm2);
      for (int i = 0; i < n; ++i) v[i] = (i < j) ? 0.0 : Xm[i][j];
      v[j] = x0 - alpha;
      const double vn2 = nrm2 - x0 * x0 + v[j] * v[j];
      tau_s = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
    }
    __syncthreads();
    const double tau = tau_s;
    for (int c = j + tid; c < p; c += blockDim.x) {
      double dsum = 0.0;
      for (int i = j; i < n; ++i) dsum += v[i] * Xm[i][c];
      for (int i = j; i < n; ++i) Xm[i][c] -= tau * dsum * v[i];
    }
    for (int r = tid; r < n; r += blockDim.x) {
      double dsum = 0.0;
      for (int i = j; i < n; ++i) dsum += Qm[r][i] * v[i];
      for (int i = j; i < n; ++i) Qm[r][i] -= tau * dsum * v[i];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < n * n; idx += blockDim.x) d.T[idx] = Qm[idx / n][idx % n];
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

void pinv_batched(const std::vector<PinvDesc>& descs, double rtol, hipStream_t s) {
  if (descs.empty()) return;
  for (auto& d : descs) ABDDC_REQUIRE(d.n <= NMAX, ABDDC_EINVAL, "pinv: matrix order exceeds 64");
  const PinvDesc* dd = Arena::for_stream(s).put(descs);
  pinv_kernel<<<descs.size(), 256, 0, s>>>(dd, rtol);
  ABDDC_HIP(hipGetLastError());
}

void qr_complete_batched(const std::vector<QrDesc>& descs, hipStream_t s) {
  if (descs.empty()) return;
  for (auto& d : descs) ABDDC_REQUIRE(d.n <= NMAX && d.p <= d.n, ABDDC_EINVAL, "qr: order exceeds 64");
  const QrDesc* dd = Arena::for_stream(s).put(descs);
  qr_complete_kernel<<<descs.size(), 256, 0, s>>>(dd);
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
  if (descs.empty()) return;
  for (auto& d : descs)
    ABDDC_REQUIRE(d.n <= NMAX, ABDDC_EINVAL, "sygv: matrix order exceeds 64");
  Arena& ar = Arena::for_stream(s);
  const SygvDesc* dd = ar.put(descs);
  sygv_kernel<<<descs.size(), 256, 0, s>>>(dd, dflag);
  ABDDC_HIP(hipGetLastError());
}

}  // namespace abddc
