// Learned edge constraints on gfx950: edge features, a 133-128-128-28 MLP
// with bfloat16 weights and activations on MFMA (FP32 accumulation), its
// backward pass, Adam, and the small kernels of the gate.
//
// Every product of the network, forward and backward, is one launch of
// bf16_gemm_kernel: C (M x N, FP32) = A (M x K) B (K x N) with arbitrary
// element strides for A and B, so transposed operands need no copies.  One
// wave computes a 16 x 16 tile with v_mfma_f32_16x16x16_bf16 (lane l holds
// A row l % 16, k = 4 (l / 16) .. + 3 and B column l % 16, same k; output
// register j is row 4 (l / 16) + j, column l % 16).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "arena.h"
#include "internal.h"
#include "mlp.h"

namespace abddc {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest, ties to even
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

struct BfGemm {
  const uint16_t* A;
  const uint16_t* B;
  float* C;             // FP32 result (may be null)
  uint16_t* Cb;         // bfloat16 copy of the (activated) result (may be null)
  const float* bias;    // per column (may be null)
  int64_t sam, sak, sbk, sbn, ldc, ldcb;
  int M, N, K, relu, accumulate;
};

__global__ void __launch_bounds__(256) bf16_gemm_kernel(BfGemm d) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.x * 32 + (wave >> 1) * 16, col0 = blockIdx.y * 32 + (wave & 1) * 16;
  const int li = lane & 15, kq = (lane >> 4) * 4;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  const int ar = row0 + li, bc = col0 + li;
  for (int k0 = 0; k0 < d.K; k0 += 16) {
    v4s a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + kq + j;
      a[j] = (ar < d.M && k < d.K) ? (short)d.A[ar * d.sam + k * d.sak] : (short)0;
      b[j] = (bc < d.N && k < d.K) ? (short)d.B[k * d.sbk + bc * d.sbn] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = row0 + kq + j, cidx = col0 + li;
    if (r >= d.M || cidx >= d.N) continue;
    float v = acc[j];
    if (d.accumulate && d.C) v += d.C[(int64_t)r * d.ldc + cidx];
    if (d.bias) v += d.bias[cidx];
    if (d.C) d.C[(int64_t)r * d.ldc + cidx] = v;
    if (d.Cb) d.Cb[(int64_t)r * d.ldcb + cidx] = to_bf16(d.relu ? fmaxf(v, 0.f) : v);
  }
}

void gemm(const BfGemm& d, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0) return;
  bf16_gemm_kernel<<<dim3((d.M + 31) / 32, (d.N + 31) / 32), 256, 0, s>>>(d);
  ABDDC_HIP(hipGetLastError());
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = to_bf16(x[i]);
}

void to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  to_bf16_kernel<<<(unsigned)std::min<int64_t>((n + 255) / 256, 4096), 256, 0, s>>>(x, y, n);
  ABDDC_HIP(hipGetLastError());
}

// dY = 2 w (Y - T) / n, its bfloat16 copy, and loss += sum w (Y - T)^2 / n
__global__ void loss_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T, int n, float* __restrict__ dY,
                                 uint16_t* __restrict__ dYb, float* __restrict__ loss) {
  __shared__ float red[4];
  const int64_t total = (int64_t)n * MLP_OUT;
  float part = 0.f;
  const float inv = 1.f / (float)n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(i % MLP_OUT);
    // upper-triangle entry e of a 7 x 7 matrix is diagonal iff it starts a row
    int r = 0, start = 0;
    while (start + (MLP_NE - r) <= e) {
      start += MLP_NE - r;
      ++r;
    }
    const float w = (e == start) ? 1.f : 2.f;
    const float df = Y[i] - T[i];
    const float g = 2.f * w * df * inv;
    dY[i] = g;
    dYb[i] = to_bf16(g);
    part += w * df * df * inv;
  }
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, red[0] + red[1] + red[2] + red[3]);
}

// dZ = dH * (Z > 0) and its bfloat16 copy
__global__ void relu_back_kernel(const float* __restrict__ dH, const float* __restrict__ Z, int64_t n, float* __restrict__ dZ,
                                 uint16_t* __restrict__ dZb) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float v = Z[i] > 0.f ? dH[i] : 0.f;
    dZ[i] = v;
    dZb[i] = to_bf16(v);
  }
}

// out[c] = sum over rows of X[r][c] (one block per column)
__global__ void colsum_kernel(const float* __restrict__ X, int rows, int cols, float* __restrict__ out) {
  __shared__ float red[4];
  const int c = blockIdx.x;
  float part = 0.f;
  for (int r = threadIdx.x; r < rows; r += blockDim.x) part += X[(int64_t)r * cols + c];
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) out[c] = red[0] + red[1] + red[2] + red[3];
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                            int64_t n, float lr, float c1, float c2) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void weights_bf16_kernel(const float* __restrict__ p, uint16_t* __restrict__ w) {
  const int64_t n1 = (int64_t)MLP_HID * MLP_IN, n2 = (int64_t)MLP_HID * MLP_HID, n3 = (int64_t)MLP_OUT * MLP_HID;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n1 + n2 + n3; i += (int64_t)gridDim.x * blockDim.x) {
    float x;
    if (i < n1) x = p[MLP_OFF_W1 + i];
    else if (i < n1 + n2) x = p[MLP_OFF_W2 + (i - n1)];
    else x = p[MLP_OFF_W3 + (i - n1 - n2)];
    w[i] = to_bf16(x);
  }
}

__global__ void ranges_kernel(const float* __restrict__ X, int n, float* __restrict__ fmin, float* __restrict__ fmax) {
  const int f = blockIdx.x;
  __shared__ float lo[256], hi[256];
  float a = INFINITY, b = -INFINITY;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    const float x = X[(int64_t)r * MLP_IN + f];
    a = fminf(a, x);
    b = fmaxf(b, x);
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      lo[threadIdx.x] = fminf(lo[threadIdx.x], lo[threadIdx.x + st]);
      hi[threadIdx.x] = fmaxf(hi[threadIdx.x], hi[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    fmin[f] = lo[0];
    fmax[f] = hi[0];
  }
}

// ------------------------------------------------------------ edge side
// one block of 128 threads per edge: thread t owns tube element t
__global__ void __launch_bounds__(128) edge_features_kernel(const EdgeGeom* __restrict__ geom, FeatParams P,
                                                            const double* __restrict__ nu, float* __restrict__ X) {
  __shared__ double ssum[2], smax[2];
  const EdgeGeom g = geom[blockIdx.x];
  float* out = X + (int64_t)blockIdx.x * MLP_IN;
  const int t = threadIdx.x;
  const int a = g.axis, b = (a + 1) % 3, c = (a + 2) % 3;
  const int tt = t >> 4, u = (t >> 2) & 3, v = t & 3;
  int e3[3];
  e3[a] = g.ilo + (2 * tt + 1) * (g.ihi - g.ilo) / 16;
  e3[b] = min(max(g.tb - 2 + u, 0), P.ne[b] - 1);
  e3[c] = min(max(g.tc - 2 + v, 0), P.ne[c] - 1);
  const int64_t eid = e3[0] + (int64_t)P.ne[0] * (e3[1] + (int64_t)P.ne[1] * e3[2]);
  const double nue = nu[eid];
  out[t] = (float)log10(nue);
  double vel[3];
  for (int i = 0; i < 3; ++i) {
    double x = P.beta0[i];
    for (int j = 0; j < 3; ++j) x += P.beta1[i * 3 + j] * (e3[j] + 0.5) * P.h[j];
    vel[i] = x;
  }
  const double pe = P.hmax * sqrt(vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]) / nue;
  double s = pe, mx = pe;
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_down(s, off, 64);
    mx = fmax(mx, __shfl_down(mx, off, 64));
  }
  if ((t & 63) == 0) {
    ssum[t >> 6] = s;
    smax[t >> 6] = mx;
  }
  __syncthreads();
  if (t == 0) {
    double mid[3];
    mid[a] = 0.5 * (g.ilo + g.ihi) * P.h[a];
    mid[b] = g.tb * P.h[b];
    mid[c] = g.tc * P.h[c];
    double w[3];
    for (int i = 0; i < 3; ++i) {
      double x = P.beta0[i];
      for (int j = 0; j < 3; ++j) x += P.beta1[i * 3 + j] * mid[j];
      w[i] = x;
    }
    out[128] = (float)asinh(w[b]);
    out[129] = (float)asinh(w[c]);
    out[130] = (float)asinh(w[a]);
    out[131] = (float)log10((ssum[0] + ssum[1]) / 128.0 + 1e-30);
    out[132] = (float)log10(fmax(smax[0], smax[1]) + 1e-30);
  }
}

__global__ void edge_projectors_kernel(const EdgeGeom* __restrict__ geom, int n_edge, const double* __restrict__ TE,
                                       const int64_t* __restrict__ teoff, const int32_t* __restrict__ r,
                                       float* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_edge * MLP_OUT) return;
  const int e = (int)(i / MLP_OUT), q = (int)(i % MLP_OUT);
  int row = 0, start = 0;
  while (start + (MLP_NE - row) <= q) {
    start += MLP_NE - row;
    ++row;
  }
  const int col = row + (q - start);
  float val = 0.f;
  if (geom[e].eligible) {
    const double* T = TE + teoff[e];
    double acc = 0.0;
    for (int k = 0; k < r[e]; ++k) acc += T[row * MLP_NE + k] * T[col * MLP_NE + k];
    val = (float)acc;
  }
  Y[i] = val;
}

__global__ void phat_kernel(const float* __restrict__ Y, int n_edge, double* __restrict__ P, double* __restrict__ I) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_edge * MLP_NE * MLP_NE) return;
  const int e = (int)(i / (MLP_NE * MLP_NE)), rc = (int)(i % (MLP_NE * MLP_NE));
  const int r = rc / MLP_NE, c = rc % MLP_NE;
  const int lo = min(r, c), hi = max(r, c);
  const int q = lo * MLP_NE - lo * (lo - 1) / 2 + (hi - lo);
  P[i] = (double)Y[(int64_t)e * MLP_OUT + q];
  I[i] = (r == c) ? 1.0 : 0.0;
}

__global__ void range_flags_kernel(const float* __restrict__ X, int n_edge, const float* __restrict__ fmin,
                                   const float* __restrict__ fmax, float slack, int32_t* __restrict__ flag) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_edge) return;
  int out = 0;
  for (int f = 0; f < MLP_IN; ++f) {
    const float span = fmax[f] - fmin[f];
    const float x = X[(int64_t)e * MLP_IN + f];
    if (x < fmin[f] - slack * span || x > fmax[f] + slack * span) out = 1;
  }
  flag[e] = out;
}

}  // namespace

void mlp_reserve(abddc_mlp* w, int n) {
  if (n <= w->cap) return;
  const int c = std::max(n, 256);
  w->X0.alloc((size_t)c * MLP_IN);
  w->H1.alloc((size_t)c * MLP_HID);
  w->H2.alloc((size_t)c * MLP_HID);
  w->G.alloc((size_t)c * MLP_HID);
  w->Z1.alloc((size_t)c * MLP_HID);
  w->Z2.alloc((size_t)c * MLP_HID);
  w->Y.alloc((size_t)c * MLP_OUT);
  w->dY.alloc((size_t)c * MLP_OUT);
  w->dZ.alloc((size_t)c * MLP_HID);
  w->dH.alloc((size_t)c * MLP_HID);
  w->cap = c;
}

void mlp_refresh_bf16(abddc_mlp* w, hipStream_t s) {
  weights_bf16_kernel<<<256, 256, 0, s>>>(w->params.p, w->wbf.p);
  ABDDC_HIP(hipGetLastError());
}

namespace {
const uint16_t* W1b(const abddc_mlp* w) { return w->wbf.p; }
const uint16_t* W2b(const abddc_mlp* w) { return w->wbf.p + (int64_t)MLP_HID * MLP_IN; }
const uint16_t* W3b(const abddc_mlp* w) { return w->wbf.p + (int64_t)MLP_HID * MLP_IN + (int64_t)MLP_HID * MLP_HID; }

// forward into the workspace; Y (fp32) written to Yout
void forward_ws(abddc_mlp* w, const float* X, int n, float* Yout, hipStream_t s) {
  to_bf16(X, w->X0.p, (int64_t)n * MLP_IN, s);
  const float* p = w->params.p;
  gemm({w->X0.p, W1b(w), w->Z1.p, w->H1.p, p + MLP_OFF_B1, MLP_IN, 1, 1, MLP_IN, MLP_HID, MLP_HID, n, MLP_HID, MLP_IN,
        1, 0},
       s);
  gemm({w->H1.p, W2b(w), w->Z2.p, w->H2.p, p + MLP_OFF_B2, MLP_HID, 1, 1, MLP_HID, MLP_HID, MLP_HID, n, MLP_HID,
        MLP_HID, 1, 0},
       s);
  gemm({w->H2.p, W3b(w), Yout, nullptr, p + MLP_OFF_B3, MLP_HID, 1, 1, MLP_HID, MLP_OUT, 0, n, MLP_OUT, MLP_HID, 0, 0},
       s);
}
}  // namespace

void mlp_forward_dev(abddc_mlp* w, const float* X, int n, float* Y, hipStream_t s) {
  if (n <= 0) return;
  mlp_reserve(w, n);
  forward_ws(w, X, n, Y, s);
}

void mlp_loss_grad_dev(abddc_mlp* w, const float* X, const float* T, int n, hipStream_t s) {
  ABDDC_REQUIRE(n > 0, ABDDC_EINVAL, "empty batch");
  mlp_reserve(w, n);
  forward_ws(w, X, n, w->Y.p, s);
  ABDDC_HIP(hipMemsetAsync(w->loss.p, 0, sizeof(float), s));
  const int64_t no = (int64_t)n * MLP_OUT, nh = (int64_t)n * MLP_HID;
  uint16_t* G3 = w->G.p;  // bf16 dY (n x OUT) in the front of G
  loss_grad_kernel<<<(unsigned)std::min<int64_t>((no + 255) / 256, 1024), 256, 0, s>>>(w->Y.p, T, n, w->dY.p, G3,
                                                                                       w->loss.p);
  ABDDC_HIP(hipGetLastError());
  float* g = w->grad.p;
  // layer 3: dW3 = G3^T H2, db3 = colsum dY, dH2 = G3 W3
  gemm({G3, w->H2.p, g + MLP_OFF_W3, nullptr, nullptr, 1, MLP_OUT, MLP_HID, 1, MLP_HID, 0, MLP_OUT, MLP_HID, n, 0, 0}, s);
  colsum_kernel<<<MLP_OUT, 256, 0, s>>>(w->dY.p, n, MLP_OUT, g + MLP_OFF_B3);
  gemm({G3, W3b(w), w->dH.p, nullptr, nullptr, MLP_OUT, 1, MLP_HID, 1, MLP_HID, 0, n, MLP_HID, MLP_OUT, 0, 0}, s);
  // layer 2 (G now holds bf16 dZ2, after dH2 has been formed from G3)
  relu_back_kernel<<<(unsigned)std::min<int64_t>((nh + 255) / 256, 4096), 256, 0, s>>>(w->dH.p, w->Z2.p, nh, w->dZ.p,
                                                                                       w->G.p);
  gemm({w->G.p, w->H1.p, g + MLP_OFF_W2, nullptr, nullptr, 1, MLP_HID, MLP_HID, 1, MLP_HID, 0, MLP_HID, MLP_HID, n, 0, 0},
       s);
  colsum_kernel<<<MLP_HID, 256, 0, s>>>(w->dZ.p, n, MLP_HID, g + MLP_OFF_B2);
  gemm({w->G.p, W2b(w), w->dH.p, nullptr, nullptr, MLP_HID, 1, MLP_HID, 1, MLP_HID, 0, n, MLP_HID, MLP_HID, 0, 0}, s);
  // layer 1
  relu_back_kernel<<<(unsigned)std::min<int64_t>((nh + 255) / 256, 4096), 256, 0, s>>>(w->dH.p, w->Z1.p, nh, w->dZ.p,
                                                                                       w->G.p);
  gemm({w->G.p, w->X0.p, g + MLP_OFF_W1, nullptr, nullptr, 1, MLP_HID, MLP_IN, 1, MLP_IN, 0, MLP_HID, MLP_IN, n, 0, 0},
       s);
  colsum_kernel<<<MLP_HID, 256, 0, s>>>(w->dZ.p, n, MLP_HID, g + MLP_OFF_B1);
  ABDDC_HIP(hipGetLastError());
}

void mlp_adam_dev(abddc_mlp* w, float lr, hipStream_t s) {
  w->step += 1;
  const float c1 = 1.f - std::pow(0.9f, (float)w->step), c2 = 1.f - std::pow(0.999f, (float)w->step);
  adam_kernel<<<256, 256, 0, s>>>(w->params.p, w->grad.p, w->m.p, w->v.p, MLP_NPARAM, lr, c1, c2);
  ABDDC_HIP(hipGetLastError());
  mlp_refresh_bf16(w, s);
}

void mlp_ranges_dev(abddc_mlp* w, const float* X, int n, hipStream_t s) {
  ABDDC_REQUIRE(n > 0, ABDDC_EINVAL, "empty feature set");
  ranges_kernel<<<MLP_IN, 256, 0, s>>>(X, n, w->fmin.p, w->fmax.p);
  ABDDC_HIP(hipGetLastError());
  w->have_ranges = true;
}

void launch_edge_features(const EdgeGeom* geom, int n_edge, const FeatParams& P, const double* nu, float* X,
                          hipStream_t s) {
  if (n_edge <= 0) return;
  edge_features_kernel<<<n_edge, 128, 0, s>>>(geom, P, nu, X);
  ABDDC_HIP(hipGetLastError());
}

void launch_edge_projectors(const EdgeGeom* geom, int n_edge, const double* TE, const int64_t* teoff,
                            const int32_t* r, float* Y, hipStream_t s) {
  const int64_t n = (int64_t)n_edge * MLP_OUT;
  if (n <= 0) return;
  edge_projectors_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(geom, n_edge, TE, teoff, r, Y);
  ABDDC_HIP(hipGetLastError());
}

void launch_phat(const float* Y, int n_edge, double* P, double* I, hipStream_t s) {
  const int64_t n = (int64_t)n_edge * MLP_NE * MLP_NE;
  if (n <= 0) return;
  phat_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(Y, n_edge, P, I);
  ABDDC_HIP(hipGetLastError());
}

void launch_range_flags(const float* X, int n_edge, const float* fmin, const float* fmax, float slack,
                        int32_t* flag, hipStream_t s) {
  if (n_edge <= 0) return;
  range_flags_kernel<<<(n_edge + 255) / 256, 256, 0, s>>>(X, n_edge, fmin, fmax, slack, flag);
  ABDDC_HIP(hipGetLastError());
}

}  // namespace abddc
