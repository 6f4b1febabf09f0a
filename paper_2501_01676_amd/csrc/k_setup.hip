// Setup-only helper kernels: deluxe systems, edge operator assembly,
// coarse-matrix assembly and elementwise combinations.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "arena.h"
#include "internal.h"
#include "setup_k.h"

namespace abddc {

namespace {

// [[sum_k S_k, S_1, ..., S_m], [-I, 0, ..., 0]]: its Schur complement onto
// the trailing block is [(sum S)^{-1} S_1, ..., (sum S)^{-1} S_m].
__global__ void deluxe_build_kernel(const DeluxeDesc* __restrict__ descs) {
  // the descriptor (indexed by member) staged in LDS once per workgroup
  __shared__ DeluxeDesc sd;
  if (threadIdx.x == 0) sd = descs[blockIdx.y];
  __syncthreads();
  const DeluxeDesc& d = sd;
  const int n = d.n, cols = (d.m + 1) * n;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < 2 * n * cols; idx += gridDim.x * blockDim.x) {
    const int r = idx / cols, c = idx % cols;
    double v = 0.0;
    if (r < n) {
      if (c < n) {
        for (int k = 0; k < d.m; ++k) v += d.src[k][(size_t)r * d.lds[k] + c];
      } else {
        const int k = c / n - 1, cc = c % n;
        v = d.src[k][(size_t)r * d.lds[k] + cc];
      }
    } else if (c < n && r - n == c) {
      v = -1.0;
    }
    d.dst[(size_t)r * cols + c] = v;
  }
}

// Aug = [[Sbar_r, W_r^T], [-W_r, 0]] (AugDesc), one wave per row (rows
// strided over the grid's waves), lanes along the row.  Eliminating its
// n_Delta leading pivots leaves [[S_PiPi - S_PiD X S_DPi, V], [-U, L]] with
// X = S_DD^{-1}: L = W_D X W_D^T, V = W_Pi^T - S_PiD X W_D^T and
// U = W_Pi - W_D X S_DPi, the averaged local solve operators.
template <class TO>
__global__ void __launch_bounds__(256) aug_build_kernel(const AugDesc* __restrict__ descs) {
  __shared__ AugDesc sd;
  if (threadIdx.x == 0) sd = descs[blockIdx.y];
  __syncthreads();
  const AugDesc& d = sd;
  const int nB = d.nB, na = 2 * nB, lane = threadIdx.x & 63;
  const int nwv = gridDim.x * (blockDim.x >> 6);
  // four columns per lane at a time, every load of a group issued before
  // its stores (the stores could alias the maps as far as the compiler knows)
  for (int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < na; i += nwv) {
    TO* row = static_cast<TO*>(d.aug) + (size_t)i * na;
    if (i < nB) {
      // row of rotated coordinate ci: Sbar(ci, am(j)), then W(m, ci) =
      // W_X(m - off, ci - off) for the m of the object of ci
      const int ci = d.am[i], q = d.slot[ci], off = d.obj_off[q], n = d.obj_n[q];
      const double* srow = d.sbar + (size_t)ci * nB;
      const double* wcol = d.wx + d.obj_w[q] + (ci - off);
      for (int j0 = lane; j0 < nB; j0 += 256) {
        int sc[4];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) sc[u] = j0 + 64 * u < nB ? d.am[j0 + 64 * u] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = sc[u] >= 0 ? srow[sc[u]] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (sc[u] >= 0) row[j0 + 64 * u] = (TO)v[u];
      }
      for (int m = lane; m < nB; m += 64)
        row[nB + m] = (TO)((m >= off && m < off + n) ? wcol[(size_t)(m - off) * n] : 0.0);
    } else {
      // row of original coordinate m: -W(m, am(j)) inside its object, then zeros
      const int m = i - nB, q = d.slot[m], off = d.obj_off[q], n = d.obj_n[q];
      const double* wrow = d.wx + d.obj_w[q] + (size_t)(m - off) * n;
      for (int j0 = lane; j0 < nB; j0 += 256) {
        int cc[4];
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) cc[u] = j0 + 64 * u < nB ? d.am[j0 + 64 * u] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (cc[u] >= off && cc[u] < off + n) ? -wrow[cc[u] - off] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (cc[u] >= 0) row[j0 + 64 * u] = (TO)v[u];
      }
      for (int j = nB + lane; j < na; j += 64) row[j] = TO(0);
    }
  }
}

// AugOutDesc: one wave per output row (the rows of M, then those of U),
// lanes along the row.
template <class T>
__global__ void __launch_bounds__(256) aug_extract_kernel(const AugOutDesc* __restrict__ descs) {
  const AugOutDesc d = descs[blockIdx.y];
  const int nB = d.nB, nD = d.nD, nP = nB - nD, na = 2 * nB, lane = threadIdx.x & 63;
  const T* A = static_cast<const T*>(d.aug);
  const int nwv = gridDim.x * (blockDim.x >> 6);
  for (int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < 2 * nB + nP; r += nwv) {
    if (r < nB + nP) {
      const T* src = A + (size_t)(r < nB ? nB + r : nD + r - nB) * na + nB;
      T* dst = static_cast<T*>(d.M) + (size_t)r * nB;
      for (int c = lane; c < nB; c += 64) dst[c] = src[c];
    } else {
      const int m = r - nB - nP;
      const T* src = A + (size_t)(nB + m) * na + nD;
      T* dst = static_cast<T*>(d.U) + (size_t)m * nP;
      for (int c = lane; c < nP; c += 64) dst[c] = -src[c];
    }
  }
}

// LinesDesc: one wave per copied row (rows = 1, lanes along the row) or per
// matrix row (rows = 0, lanes over the copied columns of that row).
__global__ void __launch_bounds__(256) copy_lines_kernel(const LinesDesc* __restrict__ descs) {
  const LinesDesc d = descs[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int nwv = gridDim.x * (blockDim.x >> 6);
  const int nr = d.rows ? d.nidx : d.n;
  for (int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < nr; r += nwv) {
    if (d.rows) {
      const size_t o = (size_t)d.idx[r] * d.n;
      for (int c = lane; c < d.n; c += 64) d.dst[o + c] = d.src[o + c];
    } else {
      const size_t o = (size_t)r * d.n;
      for (int q = lane; q < d.nidx; q += 64) {
        const int c = d.idx[q];
        d.dst[o + c] = d.src[o + c];
      }
    }
  }
}

// Metric of the earlier edge eigenproblem, regrouped by the weight index:
// B_E = sum_k D^(k)^T (sum_{i != k} B_E^(i)) D^(k), written symmetrised.
template <int NE>
__global__ void __launch_bounds__(256) edge_old_metric_kernel(const EdgeOldDesc* __restrict__ descs) {
  __shared__ double G[NE][NE + 1], Z[NE][NE + 1], A[NE][NE + 1];
  __shared__ EdgeOldDesc sd;   // the descriptor (indexed by member) staged in LDS once
  if (threadIdx.x == 0) sd = descs[blockIdx.x];
  __syncthreads();
  const EdgeOldDesc& d = sd;
  const int n = d.nE, m = d.m, tid = threadIdx.x;
  for (int idx = tid; idx < n * n; idx += blockDim.x) A[idx / n][idx % n] = 0.0;
  for (int k = 0; k < m; ++k) {
    for (int idx = tid; idx < n * n; idx += blockDim.x) {
      const int r = idx / n, c = idx % n;
      double v = 0.0;
      for (int i = 0; i < m; ++i)
        if (i != k) v += d.BE[i][(size_t)r * d.ldBE[i] + c];
      G[r][c] = v;
    }
    __syncthreads();
    const double* Dk = d.D[k];
    for (int idx = tid; idx < n * n; idx += blockDim.x) {
      const int r = idx / n, c = idx % n;
      double v = 0.0;
      for (int q = 0; q < n; ++q) v += G[r][q] * Dk[q * n + c];
      Z[r][c] = v;
    }
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += blockDim.x) {
      const int r = idx / n, c = idx % n;
      double v = 0.0;
      for (int p = 0; p < n; ++p) v += Dk[p * n + r] * Z[p][c];
      A[r][c] += v;
    }
    __syncthreads();
  }
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int r = idx / n, c = idx % n;
    d.out[idx] = 0.5 * (A[r][c] + A[c][r]);
  }
}

// Edge operators for one edge shared by m subdomains (reference = member 0):
//   That_k = [-D_2 ... -D_m] + (I in slot k for k >= 2)      (n_E x (m-1) n_E)
//   M_E    = sum_k That_k^T B_E^(k) That_k
//   Q      = sum_k P_k^T Btilde^(k) P_k in the variable order
//            [what (n_E), w_H (n_H), wcheck ((m-1) n_E)], where P_k maps
//            (wcheck, what, w_H) to (w_k,E = That_k wcheck + what, w_k,H = R_k w_H).
// NE, NW: the largest n_E and (m - 1) n_E of the instance (LDS arrays).
template <int NE, int NW>
__global__ void __launch_bounds__(256) edge_assemble_kernel(const EdgeAsmDesc* __restrict__ descs) {
  // Tb[p][a] = -D_slot[p][q] for a = (slot - 1) n_E + q; That_k = Tb + the
  // identity in slot k (k >= 1), added where That_k is read
  __shared__ double Tb[NE][NW];
  __shared__ double Z[NE][NW + NE];
  __shared__ EdgeAsmDesc sd;   // the descriptor (indexed by member) staged in LDS once
  if (threadIdx.x == 0) sd = descs[blockIdx.x];
  __syncthreads();
  const EdgeAsmDesc& d = sd;
  const int nE = d.nE, m = d.m, nw = (m - 1) * nE, nv = d.nv, nH = d.nH, tid = threadIdx.x;
  const int nt = nw + nE;  // [wcheck, what] width of T_E^(k) = [That_k | I]
  // variable position in Q of paper-order index a (wcheck, what)
  auto qpos = [&](int a) { return a < nw ? nE + nH + a : a - nw; };
  for (int idx = tid; idx < nE * nw; idx += blockDim.x) {
    const int p = idx / nw, a = idx % nw, slot = a / nE + 1, q = a % nE;
    Tb[p][a] = -d.D[slot][p * nE + q];
  }
  auto th = [&](int k, int p, int a) { return Tb[p][a] + ((a / nE + 1 == k && p == a % nE) ? 1.0 : 0.0); };
  for (int idx = tid; idx < nw * nw; idx += blockDim.x) d.ME[idx] = 0.0;
  for (int idx = tid; idx < nv * nv; idx += blockDim.x) d.Q[idx] = 0.0;
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    // M_E += That^T (B_E That)
    for (int idx = tid; idx < nE * nw; idx += blockDim.x) {
      const int p = idx / nw, a = idx % nw;
      double v = 0.0;
      for (int q = 0; q < nE; ++q) v += d.BE[k][(size_t)p * d.ldBE[k] + q] * th(k, q, a);
      Z[p][a] = v;
    }
    __syncthreads();
    for (int idx = tid; idx < nw * nw; idx += blockDim.x) {
      const int a = idx / nw, b = idx % nw;
      double v = 0.0;
      for (int p = 0; p < nE; ++p) v += th(k, p, a) * Z[p][b];
      d.ME[idx] += v;
    }
    __syncthreads();
    // Z = Btilde_EE T_E  (n_E x nt), T_E = [That | I]
    const double* Bt = d.Bt[k];
    const int ldb = d.ldBt[k], nHk = d.nHk[k];
    for (int idx = tid; idx < nE * nt; idx += blockDim.x) {
      const int p = idx / nt, a = idx % nt;
      double v = 0.0;
      if (a < nw)
        for (int q = 0; q < nE; ++q) v += Bt[(size_t)p * ldb + q] * th(k, q, a);
      else
        v = Bt[(size_t)p * ldb + (a - nw)];
      Z[p][a] = v;
    }
    __syncthreads();
    // (wcheck what, wcheck what) block: T_E^T Z
    for (int idx = tid; idx < nt * nt; idx += blockDim.x) {
      const int a = idx / nt, b = idx % nt;
      double v = 0.0;
      if (a < nw)
        for (int p = 0; p < nE; ++p) v += th(k, p, a) * Z[p][b];
      else
        v = Z[a - nw][b];
      d.Q[(size_t)qpos(a) * nv + qpos(b)] += v;
    }
    // (wcheck what, H) and (H, wcheck what): T_E^T Btilde_EH R_k and transpose side
    for (int idx = tid; idx < nt * nHk; idx += blockDim.x) {
      const int a = idx / nHk, h = idx % nHk;
      double v1 = 0.0, v2 = 0.0;
      for (int p = 0; p < nE; ++p) {
        const double t = a < nw ? th(k, p, a) : (p == a - nw ? 1.0 : 0.0);
        v1 += t * Bt[(size_t)p * ldb + nE + h];
        v2 += Bt[(size_t)(nE + h) * ldb + p] * t;
      }
      const int hq = nE + d.R[k][h];
      d.Q[(size_t)qpos(a) * nv + hq] += v1;
      d.Q[(size_t)hq * nv + qpos(a)] += v2;
    }
    // (H, H)
    for (int idx = tid; idx < nHk * nHk; idx += blockDim.x) {
      const int h1 = idx / nHk, h2 = idx % nHk;
      d.Q[(size_t)(nE + d.R[k][h1]) * nv + nE + d.R[k][h2]] += Bt[(size_t)(nE + h1) * ldb + nE + h2];
    }
    __syncthreads();
  }
}

__global__ void coarse_add_kernel(const CoarseAddDesc* __restrict__ descs, double* __restrict__ SPi, int64_t ldc) {
  const CoarseAddDesc d = descs[blockIdx.y];
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < d.n * d.n; idx += gridDim.x * blockDim.x) {
    const int a = idx / d.n, b = idx % d.n;
    SPi[(int64_t)d.gid[a] * ldc + d.gid[b]] += d.src32 ? (double)d.src32[(size_t)a * d.ld + b] : d.src[(size_t)a * d.ld + b];
  }
}

__global__ void axpby_kernel(const AxpbyDesc* __restrict__ descs) {
  const AxpbyDesc d = descs[blockIdx.y];
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < d.nr * d.nc; idx += gridDim.x * blockDim.x) {
    const int r = idx / d.nc, c = idx % d.nc;
    d.dst[(size_t)r * d.ldd + c] = d.alpha * d.X[(size_t)r * d.ldx + c] + d.beta * d.Y[(size_t)r * d.ldy + c];
  }
}

}  // namespace

void deluxe_build_batched(const std::vector<DeluxeDesc>& descs, hipStream_t s) {
  if (descs.empty()) return;
  int maxe = 0;
  for (auto& d : descs) maxe = std::max(maxe, 2 * d.n * (d.m + 1) * d.n);
  const DeluxeDesc* dd = Arena::for_stream(s).put(descs);
  deluxe_build_kernel<<<dim3(std::min(256, (maxe + 255) / 256), descs.size()), 256, 0, s>>>(dd);
  ABDDC_HIP(hipGetLastError());
}

void aug_build_batched(const std::vector<AugDesc>& descs, bool f32, hipStream_t s) {
  if (descs.empty()) return;
  int maxr = 0;
  for (auto& d : descs) maxr = std::max(maxr, 2 * d.nB);
  if (maxr == 0) return;
  const AugDesc* dd = Arena::for_stream(s).put(descs);
  const int gx = std::min((maxr + 3) / 4, 1024);   // four rows (waves) per workgroup
  if (f32) aug_build_kernel<float><<<dim3(gx, descs.size()), 256, 0, s>>>(dd);
  else aug_build_kernel<double><<<dim3(gx, descs.size()), 256, 0, s>>>(dd);
  ABDDC_HIP(hipGetLastError());
}

void aug_extract_batched(const std::vector<AugOutDesc>& descs, bool f32, hipStream_t s) {
  if (descs.empty()) return;
  int maxr = 0;
  for (auto& d : descs) maxr = std::max(maxr, 3 * d.nB - d.nD);
  if (maxr == 0) return;
  const AugOutDesc* dd = Arena::for_stream(s).put(descs);
  const int gx = std::min((maxr + 3) / 4, 1024);
  if (f32) aug_extract_kernel<float><<<dim3(gx, descs.size()), 256, 0, s>>>(dd);
  else aug_extract_kernel<double><<<dim3(gx, descs.size()), 256, 0, s>>>(dd);
  ABDDC_HIP(hipGetLastError());
}

void copy_lines_batched(const std::vector<LinesDesc>& descs, hipStream_t s) {
  if (descs.empty()) return;
  int maxr = 0;
  for (auto& d : descs) maxr = std::max(maxr, d.rows ? d.nidx : d.n);
  if (maxr == 0) return;
  const LinesDesc* dd = Arena::for_stream(s).put(descs);
  const int gx = std::min((maxr + 3) / 4, 1024);   // four lines (waves) per workgroup
  copy_lines_kernel<<<dim3(gx, descs.size()), 256, 0, s>>>(dd);
  ABDDC_HIP(hipGetLastError());
}

void edge_old_metric_batched(const std::vector<EdgeOldDesc>& descs, hipStream_t s) {
  if (descs.empty()) return;
  int nmax = 0;
  for (auto& d : descs) {
    ABDDC_REQUIRE(d.nE >= 1 && d.nE <= 32 && d.m >= 2 && d.m <= MAX_EDGE_MEMBERS, ABDDC_EINVAL,
                  "earlier edge eigenproblem: edges need 2..8 members and at most 32 dofs");
    nmax = std::max(nmax, d.nE);
  }
  const EdgeOldDesc* dd = Arena::for_stream(s).put(descs);
  if (nmax <= 16) edge_old_metric_kernel<16><<<(unsigned)descs.size(), 256, 0, s>>>(dd);
  else edge_old_metric_kernel<32><<<(unsigned)descs.size(), 256, 0, s>>>(dd);
  ABDDC_HIP(hipGetLastError());
}

void edge_assemble_batched(const std::vector<EdgeAsmDesc>& descs, hipStream_t s) {
  if (descs.empty()) return;
  bool small = true;
  for (auto& d : descs) {
    ABDDC_REQUIRE(d.nE <= 32 && (d.m - 1) * d.nE <= 128 && d.m <= MAX_EDGE_MEMBERS, ABDDC_EINVAL,
                  "edge too large: at most 32 dofs, 8 members and 128 jump unknowns");
    small = small && d.nE <= 16 && (d.m - 1) * d.nE <= 48;
  }
  const EdgeAsmDesc* dd = Arena::for_stream(s).put(descs);
  if (small) edge_assemble_kernel<16, 48><<<descs.size(), 256, 0, s>>>(dd);
  else edge_assemble_kernel<32, 128><<<descs.size(), 256, 0, s>>>(dd);
  ABDDC_HIP(hipGetLastError());
}

void coarse_add_batched(const std::vector<CoarseAddDesc>& descs, double* SPi, int64_t ldc, hipStream_t s) {
  if (descs.empty()) return;
  int maxe = 0;
  for (auto& d : descs) maxe = std::max(maxe, d.n * d.n);
  if (maxe == 0) return;
  const CoarseAddDesc* dd = Arena::for_stream(s).put(descs);
  coarse_add_kernel<<<dim3(std::min(64, (maxe + 255) / 256), descs.size()), 256, 0, s>>>(dd, SPi, ldc);
  ABDDC_HIP(hipGetLastError());
}

void axpby_batched(const std::vector<AxpbyDesc>& descs, hipStream_t s) {
  if (descs.empty()) return;
  int maxe = 0;
  for (auto& d : descs) maxe = std::max(maxe, d.nr * d.nc);
  if (maxe == 0) return;
  const AxpbyDesc* dd = Arena::for_stream(s).put(descs);
  axpby_kernel<<<dim3(std::min(256, (maxe + 255) / 256), descs.size()), 256, 0, s>>>(dd);
  ABDDC_HIP(hipGetLastError());
}

}  // namespace abddc
