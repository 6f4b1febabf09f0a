// Learned edge constraints: the network object, edge features and the
// device kernels around them (k_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "internal.h"

namespace abddc {

constexpr int MLP_IN = 133, MLP_HID = 128, MLP_OUT = 28, MLP_NE = 7;
// parameter layout: W1 (HID x IN), b1, W2 (HID x HID), b2, W3 (OUT x HID), b3
constexpr int64_t MLP_OFF_W1 = 0;
constexpr int64_t MLP_OFF_B1 = MLP_OFF_W1 + (int64_t)MLP_HID * MLP_IN;
constexpr int64_t MLP_OFF_W2 = MLP_OFF_B1 + MLP_HID;
constexpr int64_t MLP_OFF_B2 = MLP_OFF_W2 + (int64_t)MLP_HID * MLP_HID;
constexpr int64_t MLP_OFF_W3 = MLP_OFF_B2 + MLP_HID;
constexpr int64_t MLP_OFF_B3 = MLP_OFF_W3 + (int64_t)MLP_OUT * MLP_HID;
constexpr int64_t MLP_NPARAM = MLP_OFF_B3 + MLP_OUT;

// Per-edge geometry for the feature kernel (edge frame: axis a along the
// edge, b = a + 1, c = a + 2 mod 3).
struct EdgeGeom {
  int32_t axis, tb, tc, ilo, ihi, eligible;
};

struct FeatParams {
  int32_t ne[3];
  double h[3], hmax, beta0[3], beta1[9];
};

}  // namespace abddc

struct abddc_ctx;

struct abddc_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  abddc::DevAlloc dalloc;          // caller's device allocation hooks
  abddc::DevBuf<float> params, m, v, grad, fmin, fmax, loss;
  abddc::DevBuf<uint16_t> wbf;     // bfloat16 W1 | W2 | W3
  int64_t step = 0;
  bool have_ranges = false;
  int cap = 0;                     // workspace rows
  abddc::DevBuf<uint16_t> X0, H1, H2, G;
  abddc::DevBuf<float> Z1, Z2, Y, dY, dZ, dH;
};

namespace abddc {

void mlp_reserve(abddc_mlp* w, int n);
void mlp_refresh_bf16(abddc_mlp* w, hipStream_t s);
// Y (n x OUT, fp32) = network(X (n x IN, fp32)); X, Y device pointers.
void mlp_forward_dev(abddc_mlp* w, const float* X, int n, float* Y, hipStream_t s);
// loss (device scalar) and grad (device, parameter layout) of the batch.
void mlp_loss_grad_dev(abddc_mlp* w, const float* X, const float* T, int n, hipStream_t s);
void mlp_adam_dev(abddc_mlp* w, float lr, hipStream_t s);
void mlp_ranges_dev(abddc_mlp* w, const float* X, int n, hipStream_t s);

// per-edge frame of a context (built once) and the feature constants
void build_edge_geometry(abddc_ctx* c);
FeatParams feature_params(const abddc_ctx* c);

void launch_edge_features(const EdgeGeom* geom, int n_edge, const FeatParams& P, const double* nu, float* X,
                          hipStream_t s);
// projector upper triangles of the first r columns of each edge basis
void launch_edge_projectors(const EdgeGeom* geom, int n_edge, const double* TE, const int64_t* teoff,
                            const int32_t* r, float* Y, hipStream_t s);
// symmetric P-hat (double, 7 x 7 per edge, consecutive) and identity metric
void launch_phat(const float* Y, int n_edge, double* P, double* I, hipStream_t s);
// flag[e] = 1 when a feature of edge e is outside [fmin, fmax] widened by slack
void launch_range_flags(const float* X, int n_edge, const float* fmin, const float* fmax, float slack,
                        int32_t* flag, hipStream_t s);

}  // namespace abddc
