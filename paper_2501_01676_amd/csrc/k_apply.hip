// Per-iteration kernels: batched ragged GEMV with gathered input (the local
// and coarse pieces of M^{-1} and the local Schur complements of Shat), the
// deterministic interface gather-sum R^T (sum over the subdomains sharing a
// dof, fixed order), and the GMRES vector kernels (multi-dot with wavefront
// reductions, multi-axpy, Givens update of the Hessenberg column).
//
// These kernels move O(bytes) with O(1) flops per byte: they are bound by
// HBM bandwidth, so the design goal is coalesced 512-byte wave loads of
// matrix rows and no re-reads.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>

#include "apply.h"
#include "buffer.h"
#include "internal.h"
#include "htrace.h"
#include "kstats.h"
#include "tune.h"

namespace abddc {

namespace {

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// A workgroup = 4 waves x R rows of one matrix.  The gathered input vector
// is staged in LDS once per workgroup; each wave streams its R rows with
// 64-lane coalesced loads and reduces them with wavefront shuffles.
template <class TM, int R>
__global__ void __launch_bounds__(256) gemv_kernel(const GemvBlock* __restrict__ blocks,
                                                   const GemvMat* __restrict__ mats, const TM* __restrict__ M,
                                                   const double* __restrict__ x, const int32_t* __restrict__ xidx,
                                                   double* __restrict__ y, int accumulate) {
  extern __shared__ double xs[];
  const GemvBlock blk = blocks[blockIdx.x];
  const GemvMat d = mats[blk.mat];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = blk.row0 + w * R;
  // matrix rows through a buffer descriptor at the matrix's start: a row
  // past the last one has offset BUF_OUT and reads zero, and so does a
  // column past the last one in the final partial block
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(M + d.moff);
  const int nr = min(R, d.nrows - r0), cl = lane * (int)sizeof(TM);
  int ro[R];
#pragma unroll
  for (int q = 0; q < R; ++q) ro[q] = q < nr ? (r0 + q) * d.ld * (int)sizeof(TM) + cl : BUF_OUT;
  // the rows' first 64 columns are requested before the input gather, so
  // the two latencies overlap
  TM pre[R];
#pragma unroll
  for (int q = 0; q < R; ++q) pre[q] = buf_load<TM>(rs, lane < d.ncols ? ro[q] : BUF_OUT, 0);
  for (int c = threadIdx.x; c < d.ncols; c += blockDim.x)
    xs[c] = xidx ? x[xidx[d.xoff + c]] : x[d.xoff + c];
  __syncthreads();
  double acc[R];
  {
    const double xv = d.ncols > 0 ? xs[min(lane, d.ncols - 1)] : 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = (double)pre[q] * xv;
  }
  int c0 = 64;
#pragma unroll 2
  for (; c0 + 64 <= d.ncols; c0 += 64) {   // whole blocks of 64 columns
    const double xv = xs[c0 + lane];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] += (double)buf_load<TM>(rs, ro[q], c0 * (int)sizeof(TM)) * xv;
  }
  if (c0 < d.ncols) {
    const bool ok = c0 + lane < d.ncols;
    const double xv = xs[ok ? c0 + lane : d.ncols - 1];
#pragma unroll
    for (int q = 0; q < R; ++q)
      acc[q] += (double)buf_load<TM>(rs, ok ? ro[q] : BUF_OUT, c0 * (int)sizeof(TM)) * xv;
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0 && q < nr) {
      double* yp = y + d.yoff + r0 + q;
      *yp = accumulate ? *yp + v : v;
    }
  }
}

// Operators of at most 64 columns (the tall and thin U): one lane per row,
// the workgroup's 256 rows of one matrix.  A lane forms the 64 products the
// 64 lanes of gemv_kernel would hold and adds them in the same tree as its
// wavefront reduction, so every variant gives the same bits.
template <class TM>
__global__ void __launch_bounds__(256) gemv_narrow_kernel(const GemvBlock* __restrict__ blocks,
                                                          const GemvMat* __restrict__ mats,
                                                          const TM* __restrict__ M, const double* __restrict__ x,
                                                          const int32_t* __restrict__ xidx, double* __restrict__ y,
                                                          int accumulate) {
  extern __shared__ double xs[];
  const GemvBlock blk = blocks[blockIdx.x];
  const GemvMat d = mats[blk.mat];
  for (int c = threadIdx.x; c < d.ncols; c += blockDim.x)
    xs[c] = xidx ? x[xidx[d.xoff + c]] : x[d.xoff + c];
  __syncthreads();
  const int r = blk.row0 + (int)threadIdx.x;
  if (r >= d.nrows) return;
  // loads through a buffer descriptor: a column past the last one reads zero
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(M + d.moff);
  const int ro = r * d.ld * (int)sizeof(TM);
  const double xlast = d.ncols > 0 ? xs[d.ncols - 1] : 0.0;
  double a[64];
#pragma unroll
  for (int l = 0; l < 64; ++l)
    a[l] = (double)buf_load<TM>(rs, l < d.ncols ? ro : BUF_OUT, l * (int)sizeof(TM)) * (l < d.ncols ? xs[l] : xlast);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int l = 0; l < off; ++l) a[l] += a[l + off];
  double* yp = y + d.yoff + r;
  *yp = accumulate ? *yp + a[0] : a[0];
}

__global__ void gather_sum_kernel(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                                  const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  for (int j = ptr[i]; j < ptr[i + 1]; ++j) v += src[idx[j]];
  dst[i] = v;
}

// dst[i] = sum of src over the positions of i; the same into Z[:, st->j]
__global__ void gather_sum_col_kernel(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                                      const double* __restrict__ src, double* __restrict__ dst, double* __restrict__ Z,
                                      int64_t ldz, const GmresState* __restrict__ st, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  for (int j = ptr[i]; j < ptr[i + 1]; ++j) v += src[idx[j]];
  dst[i] = v;
  Z[(int64_t)st->j * ldz + i] = v;
}

// partial[b * DOT_STRIDE + j] = sum over block b's chunk of V[j][i] w[i]
__global__ void __launch_bounds__(256) dots_partial_kernel(const double* __restrict__ V, int64_t ldv, int nv,
                                                           const GmresState* __restrict__ st,
                                                           const double* __restrict__ w, int64_t n,
                                                           double* __restrict__ partial) {
  __shared__ double red[4];
  if (st) nv = st->j + 1;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = 0; j < nv; ++j) {
    double a = 0.0;
    const double* vj = V + (int64_t)j * ldv;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) a += vj[i] * w[i];
    a = wave_sum(a);
    if (lane == 0) red[wv] = a;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x * DOT_STRIDE + j] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
}

// w -= V[:, 0..nv) coef (nv = st->j + 1), then the partial dot products of
// the updated w over the same chunks as dots_partial_kernel: with V[j] for
// j < nv, or with itself (norm) -- each workgroup updates exactly the
// entries it then reads, so one launch does both.
__global__ void __launch_bounds__(256) axpy_dots_partial_kernel(const double* __restrict__ V, int64_t ldv,
                                                                const GmresState* __restrict__ st,
                                                                const double* __restrict__ coef, double* __restrict__ w,
                                                                int64_t n, int norm, double* __restrict__ partial) {
  __shared__ double red[4];
  const int nv = st->j + 1;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    double sacc = 0.0;
    for (int j = 0; j < nv; ++j) sacc += coef[j] * V[(int64_t)j * ldv + i];
    w[i] -= sacc;
  }
  const int nd = norm ? 1 : nv;
  for (int j = 0; j < nd; ++j) {
    double a = 0.0;
    const double* vj = norm ? w : V + (int64_t)j * ldv;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) a += vj[i] * w[i];
    a = wave_sum(a);
    if (lane == 0) red[wv] = a;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x * DOT_STRIDE + j] = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
  }
}

// one workgroup per vector j: fixed-order tree over the block partials
__global__ void __launch_bounds__(256) dots_final_kernel(const double* __restrict__ partial, int nblk,
                                                         const GmresState* __restrict__ st,
                                                         double* __restrict__ out) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  if (st && j > st->j) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += partial[b * DOT_STRIDE + j];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[j] = (red[0] + red[1]) + (red[2] + red[3]);
}

// w[i] += sign * sum_j coef[j] V[j][i]
__global__ void axpy_multi_kernel(const double* __restrict__ V, int64_t ldv, int nv,
                                  const GmresState* __restrict__ st, const double* __restrict__ coef,
                                  double sign, double* __restrict__ w, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (st) nv = st->j + 1;
  double s = 0.0;
  for (int j = 0; j < nv; ++j) s += coef[j] * V[(int64_t)j * ldv + i];
  w[i] += sign * s;
}

// Hessenberg column j from the two Gram-Schmidt passes and the norm, the
// previous Givens rotations, a new rotation, the rotated rhs g and the
// residual estimate |g[j+1]|.
__device__ void arnoldi_column(GmresState* st, int j, const double* __restrict__ h1, const double* __restrict__ h2,
                               const double* __restrict__ nrm2) {
  double col[GMRES_MAXR + 1];
  for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
  const double hn = sqrt(fmax(nrm2[0], 0.0));
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double t = st->cs[i] * col[i] + st->sn[i] * col[i + 1];
    col[i + 1] = -st->sn[i] * col[i] + st->cs[i] * col[i + 1];
    col[i] = t;
  }
  const double a = col[j], b = col[j + 1];
  const double r = hypot(a, b);
  double c = 1.0, s = 0.0;
  if (r != 0.0) {
    c = a / r;
    s = b / r;
  }
  st->cs[j] = c;
  st->sn[j] = s;
  col[j] = r;
  col[j + 1] = 0.0;
  st->g[j + 1] = -s * st->g[j];
  st->g[j] = c * st->g[j];
  for (int i = 0; i <= j + 1; ++i) st->H[i * GMRES_MAXR + j] = col[i];
  st->hn = hn;
  st->inv_hn = hn > 0.0 ? 1.0 / hn : 0.0;
  st->res = fabs(st->g[j + 1]);
  st->j = j + 1;
}


// beta, hn, inv_hn, res into pinned host memory (device-coherent), visible
// to the host once the kernel has completed.
__device__ inline void publish_scalars(const GmresState* st, double* host) {
  host[0] = st->beta;
  host[1] = st->hn;
  host[2] = st->inv_hn;
  host[3] = st->res;
  __threadfence_system();
}

// host_out (optional): two slots of four scalars; step jj writes slot jj % 2.
__global__ void arnoldi_finish_kernel(GmresState* st, int j, const double* __restrict__ h1,
                                      const double* __restrict__ h2, const double* __restrict__ nrm2,
                                      double* host_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const bool dev_j = j < 0;
  const int jj = dev_j ? st->j : j;
  const int keep = st->j;
  arnoldi_column(st, jj, h1, h2, nrm2);
  if (!dev_j) st->j = keep;
  if (host_out) publish_scalars(st, host_out + 4 * (jj & 1));
}

// y = H(0:m, 0:m)^{-1} g(0:m) (upper triangular)
__global__ void gmres_trisolve_kernel(GmresState* st, int m) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = m - 1; i >= 0; --i) {
    double v = st->g[i];
    for (int q = i + 1; q < m; ++q) v -= st->H[i * GMRES_MAXR + q] * st->y[q];
    st->y[i] = v / st->H[i * GMRES_MAXR + i];
  }
}

__global__ void gmres_start_kernel(GmresState* st, const double* __restrict__ nrm2, double* host_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double b = sqrt(fmax(nrm2[0], 0.0));
  for (int i = 0; i <= GMRES_MAXR; ++i) st->g[i] = 0.0;
  st->g[0] = b;
  st->beta = b;
  st->inv_hn = b > 0.0 ? 1.0 / b : 0.0;
  st->res = b;
  st->j = 0;
  if (host_out) publish_scalars(st, host_out);
}

__global__ void scale_to_col_kernel(const double* __restrict__ src, const GmresState* __restrict__ st,
                                    double* __restrict__ V, int64_t ldv, double* __restrict__ cur, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = src[i] * st->inv_hn;
  V[(int64_t)st->j * ldv + i] = v;
  cur[i] = v;
}

__global__ void scale_copy_kernel(const double* __restrict__ src, const double* __restrict__ factor,
                                  double* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i] * factor[0];
}

__global__ void sub_kernel(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out,
                           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

inline unsigned nblocks(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

}  // namespace

namespace {
template <class TM, int R>
void gemv_launch(const GemvOp& op, int v, const TM* M, const double* x, const int32_t* xidx, double* y,
                 bool accumulate, hipStream_t s) {
  hipEvent_t ea, eb;
  tracked_events(KC_GEMV, op.bytes, &ea, &eb);
  const uint32_t lds = (uint32_t)(op.maxc * sizeof(double));
  if (ea)
    hipExtLaunchKernelGGL(gemv_kernel<TM, R>, dim3(op.nblk[v]), dim3(256), lds, s, ea, eb, 0, op.blocks[v].p,
                          op.mats.p, M, x, xidx, y, accumulate ? 1 : 0);
  else
    gemv_kernel<TM, R><<<op.nblk[v], 256, lds, s>>>(op.blocks[v].p, op.mats.p, M, x, xidx, y, accumulate ? 1 : 0);
}

template <class TM>
void gemv_narrow_launch(const GemvOp& op, const TM* M, const double* x, const int32_t* xidx, double* y,
                        bool accumulate, hipStream_t s) {
  hipEvent_t ea, eb;
  tracked_events(KC_GEMV, op.bytes, &ea, &eb);
  const uint32_t lds = (uint32_t)(op.maxc * sizeof(double));
  const int v = GEMV_NARROW;
  if (ea)
    hipExtLaunchKernelGGL(gemv_narrow_kernel<TM>, dim3(op.nblk[v]), dim3(256), lds, s, ea, eb, 0, op.blocks[v].p,
                          op.mats.p, M, x, xidx, y, accumulate ? 1 : 0);
  else
    gemv_narrow_kernel<TM><<<op.nblk[v], 256, lds, s>>>(op.blocks[v].p, op.mats.p, M, x, xidx, y,
                                                        accumulate ? 1 : 0);
}

template <class TM>
void gemv_variant(const GemvOp& op, int v, const TM* M, const double* x, const int32_t* xidx, double* y,
                  bool accumulate, hipStream_t s) {
  if (op.nblk[v] == 0) return;
  switch (v) {
    case 0: gemv_launch<TM, 2>(op, v, M, x, xidx, y, accumulate, s); break;
    case 1: gemv_launch<TM, 4>(op, v, M, x, xidx, y, accumulate, s); break;
    case 2: gemv_launch<TM, 8>(op, v, M, x, xidx, y, accumulate, s); break;
    default: gemv_narrow_launch<TM>(op, M, x, xidx, y, accumulate, s); break;
  }
  ABDDC_HIP(hipGetLastError());
}
}  // namespace

void gemv_build(GemvOp& op, const std::vector<GemvMat>& mats, const std::vector<char>* active, double bytes,
                hipStream_t s) {
  op.maxc = 1;
  op.rows = 0;
  for (const GemvMat& m : mats) {
    op.maxc = std::max(op.maxc, (int)m.ncols);
    ABDDC_REQUIRE((int64_t)m.nrows * m.ld * (int64_t)sizeof(double) < BUF_LIMIT, ABDDC_EINVAL,
                  "gemv: matrix spans 2 GiB or more");
  }
  HostTrace ht;
  for (int v = 0; v < GEMV_NVAR; ++v) {
    std::vector<GemvBlock> b;
    const int rpb = v == GEMV_NARROW ? 256 : 4 * GEMV_ROWS[v];
    for (size_t i = 0; i < mats.size() && (v != GEMV_NARROW || op.maxc <= 64); ++i) {
      if (active && !(*active)[i]) continue;
      for (int r = 0; r < mats[i].nrows; r += rpb) b.push_back({(int32_t)i, r});
    }
    op.blocks[v] = to_device(b, s);
    op.nblk[v] = (int)b.size();
  }
  for (size_t i = 0; i < mats.size(); ++i)
    if (!active || (*active)[i]) op.rows += mats[i].nrows;
  ht.mark("gemv_build: block lists");
  op.mats = to_device(mats, s);
  op.bytes = bytes;
  ht.mark("gemv_build: matrices");
}

template <class TM>
void gemv_run(const GemvOp& op, const TM* M, const double* x, const int32_t* xidx, double* y, bool accumulate,
              hipStream_t s) {
  gemv_variant<TM>(op, op.var, M, x, xidx, y, accumulate, s);
}

template <class TM>
void gemv_tune(GemvOp& op, const char* name, int device, const TM* M, const double* x, const int32_t* xidx,
               double* y, hipStream_t s) {
  if (op.nblk[0] == 0) return;
  const char* force = std::getenv("ABDDC_GEMV_VARIANT");   // fixed variant, no timing (tests, experiments)
  if (force && *force >= '0' && *force < '0' + GEMV_NVAR && force[1] == 0) {
    op.var = op.nblk[*force - '0'] > 0 ? *force - '0' : 1;   // the narrow form only where it applies
    return;
  }
  const std::string key = device_arch(device) + "|gemv|" + name + "|" + (sizeof(TM) == 8 ? "f64" : "f32") + "|c" +
                          std::to_string(size_bucket(op.maxc)) + "|r" + std::to_string(size_bucket(op.rows));
  const int cached = tune_lookup(key);
  if (cached >= 0 && cached < GEMV_NVAR && op.nblk[cached] > 0) {
    op.var = cached;
    return;
  }
  KStatsScope none(nullptr);
  HostTrace ht;
  hipEvent_t e0, e1;
  ABDDC_HIP(hipEventCreate(&e0));
  ABDDC_HIP(hipEventCreate(&e1));
  float best = 0.f;
  int bestv = 1;
  for (int v = 0; v < GEMV_NVAR; ++v) {
    if (op.nblk[v] == 0) continue;
    gemv_variant<TM>(op, v, M, x, xidx, y, false, s);   // warm-up
    ABDDC_HIP(hipEventRecord(e0, s));
    for (int rep = 0; rep < 3; ++rep) gemv_variant<TM>(op, v, M, x, xidx, y, false, s);
    ABDDC_HIP(hipEventRecord(e1, s));
    ABDDC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    ABDDC_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (v == 0 || ms < best) {
      best = ms;
      bestv = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  op.var = bestv;
  tune_store(key, bestv);
  ht.mark(("autotuner: timed " + key).c_str());
}

template void gemv_run<double>(const GemvOp&, const double*, const double*, const int32_t*, double*, bool,
                               hipStream_t);
template void gemv_run<float>(const GemvOp&, const float*, const double*, const int32_t*, double*, bool, hipStream_t);
template void gemv_tune<double>(GemvOp&, const char*, int, const double*, const double*, const int32_t*, double*,
                                hipStream_t);
template void gemv_tune<float>(GemvOp&, const char*, int, const float*, const double*, const int32_t*, double*,
                               hipStream_t);

void launch_gather_sum(const int32_t* ptr, const int32_t* idx, const double* src, double* dst, int64_t n,
                       hipStream_t s) {
  if (n == 0) return;
  gather_sum_kernel<<<nblocks(n), 256, 0, s>>>(ptr, idx, src, dst, n);
  ABDDC_HIP(hipGetLastError());
}

void launch_gather_sum_col(const int32_t* ptr, const int32_t* idx, const double* src, double* dst, double* Z,
                           int64_t ldz, const GmresState* st, int64_t n, hipStream_t s) {
  if (n == 0) return;
  gather_sum_col_kernel<<<nblocks(n), 256, 0, s>>>(ptr, idx, src, dst, Z, ldz, st, n);
  ABDDC_HIP(hipGetLastError());
}

void launch_dots(const double* V, int64_t ldv, int nv, const double* w, int64_t n, double* partial, double* out,
                 hipStream_t s) {
  dots_partial_kernel<<<DOT_BLOCKS, 256, 0, s>>>(V, ldv, nv, nullptr, w, n, partial);
  dots_final_kernel<<<nv, 256, 0, s>>>(partial, DOT_BLOCKS, nullptr, out);
  ABDDC_HIP(hipGetLastError());
}

void launch_dots_dev(const double* V, int64_t ldv, const GmresState* st, int max_nv, const double* w, int64_t n,
                     double* partial, double* out, hipStream_t s) {
  dots_partial_kernel<<<DOT_BLOCKS, 256, 0, s>>>(V, ldv, 0, st, w, n, partial);
  dots_final_kernel<<<max_nv, 256, 0, s>>>(partial, DOT_BLOCKS, st, out);
  ABDDC_HIP(hipGetLastError());
}

void launch_axpy_dots_dev(const double* V, int64_t ldv, const GmresState* st, int max_nv, const double* coef,
                          double* w, int64_t n, bool norm, double* partial, double* out, hipStream_t s) {
  axpy_dots_partial_kernel<<<DOT_BLOCKS, 256, 0, s>>>(V, ldv, st, coef, w, n, norm ? 1 : 0, partial);
  if (norm)
    dots_final_kernel<<<1, 256, 0, s>>>(partial, DOT_BLOCKS, nullptr, out);
  else
    dots_final_kernel<<<max_nv, 256, 0, s>>>(partial, DOT_BLOCKS, st, out);
  ABDDC_HIP(hipGetLastError());
}

void launch_axpy_multi_dev(const double* V, int64_t ldv, const GmresState* st, const double* coef, double sign,
                           double* w, int64_t n, hipStream_t s) {
  axpy_multi_kernel<<<nblocks(n), 256, 0, s>>>(V, ldv, 0, st, coef, sign, w, n);
  ABDDC_HIP(hipGetLastError());
}

void launch_scale_to_col(const double* src, const GmresState* st, double* V, int64_t ldv, double* cur, int64_t n,
                         hipStream_t s) {
  scale_to_col_kernel<<<nblocks(n), 256, 0, s>>>(src, st, V, ldv, cur, n);
  ABDDC_HIP(hipGetLastError());
}

void launch_arnoldi_finish_dev(GmresState* st, const double* h1, const double* h2, const double* nrm2,
                               double* host_out, hipStream_t s) {
  arnoldi_finish_kernel<<<1, 64, 0, s>>>(st, -1, h1, h2, nrm2, host_out);
  ABDDC_HIP(hipGetLastError());
}

void launch_axpy_multi(const double* V, int64_t ldv, int nv, const double* coef, double sign, double* w, int64_t n,
                       hipStream_t s) {
  axpy_multi_kernel<<<nblocks(n), 256, 0, s>>>(V, ldv, nv, nullptr, coef, sign, w, n);
  ABDDC_HIP(hipGetLastError());
}

void launch_arnoldi_finish(GmresState* st, int j, const double* h1, const double* h2, const double* nrm2,
                           hipStream_t s) {
  arnoldi_finish_kernel<<<1, 64, 0, s>>>(st, j, h1, h2, nrm2, nullptr);
  ABDDC_HIP(hipGetLastError());
}

void launch_gmres_trisolve(GmresState* st, int m, hipStream_t s) {
  gmres_trisolve_kernel<<<1, 64, 0, s>>>(st, m);
  ABDDC_HIP(hipGetLastError());
}

void launch_gmres_start(GmresState* st, const double* nrm2, double* host_out, hipStream_t s) {
  gmres_start_kernel<<<1, 64, 0, s>>>(st, nrm2, host_out);
  ABDDC_HIP(hipGetLastError());
}

void launch_scale_copy(const double* src, const double* factor, double* dst, int64_t n, hipStream_t s) {
  scale_copy_kernel<<<nblocks(n), 256, 0, s>>>(src, factor, dst, n);
  ABDDC_HIP(hipGetLastError());
}

void launch_sub(const double* a, const double* b, double* out, int64_t n, hipStream_t s) {
  sub_kernel<<<nblocks(n), 256, 0, s>>>(a, b, out, n);
  ABDDC_HIP(hipGetLastError());
}

}  // namespace abddc
