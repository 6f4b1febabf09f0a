// C ABI of the learned edge constraints: network object, training step,
// edge features and training targets.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <memory>

#include "../../include/abddc.h"
#include "ctx.h"
#include "guard.h"
#include "internal.h"
#include "mlp.h"

using namespace abddc;

namespace abddc {

// Edge frame of every edge: the edge axis is the one whose coordinate is
// not a subdomain cut; the element range along it runs from the vertex
// before the first edge node to the vertex after the last.
void build_edge_geometry(abddc_ctx* c) {
  if (!c->egeom.empty() || c->topo.edges.empty()) return;
  const Topology& T = c->topo;
  for (int k : T.edges) {
    const Object& o = T.objects[k];
    int64_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = INT64_MAX;
      hi[a] = -1;
    }
    for (int64_t nid : o.nodes) {
      const int64_t x[3] = {nid % T.nn[0], (nid / T.nn[0]) % T.nn[1], nid / ((int64_t)T.nn[0] * T.nn[1])};
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], x[a]);
        hi[a] = std::max(hi[a], x[a]);
      }
    }
    int axis = 0;
    for (int a = 0; a < 3; ++a) {
      bool on_cut = false;
      for (int cpos : T.cuts[a]) on_cut |= (cpos == lo[a]);
      if (!on_cut) axis = a;
    }
    const int b = (axis + 1) % 3, cc = (axis + 2) % 3;
    EdgeGeom g{axis, (int32_t)lo[b], (int32_t)lo[cc], (int32_t)(lo[axis] - 1), (int32_t)(hi[axis] + 1),
               o.n == MLP_NE ? 1 : 0};
    c->egeom.push_back(g);
  }
  c->d_egeom = to_device(c->egeom, c->stream);
}

FeatParams feature_params(const abddc_ctx* c) {
  FeatParams P{};
  P.hmax = 0;
  for (int a = 0; a < 3; ++a) {
    P.ne[a] = c->topo.ne[a];
    P.h[a] = c->length[a] / c->topo.ne[a];
    P.hmax = std::max(P.hmax, P.h[a]);
    P.beta0[a] = c->beta0[a];
  }
  for (int i = 0; i < 9; ++i) P.beta1[i] = c->beta1[i];
  return P;
}

}  // namespace abddc

namespace {
abddc_mlp* checked(abddc_mlp* w) {
  ABDDC_REQUIRE(w, ABDDC_EINVAL, "null network");
  ABDDC_HIP(hipSetDevice(w->device));
  return w;
}

__global__ void eligible_kernel(const EdgeGeom* g, int n, int32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = g[i].eligible;
}
}  // namespace

extern "C" int abddc_mlp_create(const float* params, int32_t n_params, const abddc_device* dev, abddc_mlp** out) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(params && dev && out, ABDDC_EINVAL, "null argument");
    ABDDC_REQUIRE(n_params == MLP_NPARAM, ABDDC_EINVAL, "parameter count must be ABDDC_MLP_PARAMS");
    *out = nullptr;
    ABDDC_HIP(hipSetDevice(dev->device));
    ABDDC_REQUIRE((dev->alloc == nullptr) == (dev->free == nullptr), ABDDC_EINVAL,
                  "device allocation hooks: alloc and free must both be set or both be null");
    std::unique_ptr<abddc_mlp> w(new abddc_mlp());
    w->device = dev->device;
    w->stream = (hipStream_t)dev->stream;
    w->dalloc = DevAlloc{dev->alloc, dev->free, dev->user};
    AllocScope as(&w->dalloc);
    StreamScope ss(w->stream);
    std::vector<float> h(params, params + MLP_NPARAM), z(MLP_NPARAM, 0.f);
    w->params = to_device(h, w->stream);
    w->m = to_device(z, w->stream);
    w->v = to_device(z, w->stream);
    w->grad.alloc(MLP_NPARAM);
    w->fmin.alloc(MLP_IN);
    w->fmax.alloc(MLP_IN);
    w->loss.alloc(1);
    w->wbf.alloc((size_t)MLP_HID * MLP_IN + (size_t)MLP_HID * MLP_HID + (size_t)MLP_OUT * MLP_HID);
    mlp_refresh_bf16(w.get(), w->stream);
    ABDDC_HIP(hipStreamSynchronize(w->stream));
    *out = w.release();
    return ABDDC_OK;
  });
}

extern "C" int abddc_mlp_get_params(abddc_mlp* mlp, float* params, int32_t n_params) {
  return guarded([&]() -> int {
    abddc_mlp* w = checked(mlp);
    AllocScope as(&w->dalloc);
    ABDDC_REQUIRE(params && n_params == MLP_NPARAM, ABDDC_EINVAL, "bad parameter buffer");
    StreamScope ss(w->stream);
    std::vector<float> h = to_host(w->params.p, MLP_NPARAM, w->stream);
    std::copy(h.begin(), h.end(), params);
    return ABDDC_OK;
  });
}

extern "C" int abddc_mlp_forward(abddc_mlp* mlp, const float* X, int32_t n, float* Y) {
  return guarded([&]() -> int {
    abddc_mlp* w = checked(mlp);
    AllocScope as(&w->dalloc);
    ABDDC_REQUIRE(n >= 0 && (n == 0 || (X && Y)), ABDDC_EINVAL, "bad batch");
    StreamScope ss(w->stream);
    mlp_forward_dev(w, X, n, Y, w->stream);
    return ABDDC_OK;
  });
}

extern "C" int abddc_mlp_loss_grad(abddc_mlp* mlp, const float* X, const float* T, int32_t n, float* grad,
                                   float* loss) {
  return guarded([&]() -> int {
    abddc_mlp* w = checked(mlp);
    AllocScope as(&w->dalloc);
    ABDDC_REQUIRE(n > 0 && X && T && grad && loss, ABDDC_EINVAL, "bad batch");
    StreamScope ss(w->stream);
    mlp_loss_grad_dev(w, X, T, n, w->stream);
    ABDDC_HIP(hipMemcpyAsync(grad, w->grad.p, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToDevice, w->stream));
    std::vector<float> l = to_host(w->loss.p, 1, w->stream);
    *loss = l[0];
    return ABDDC_OK;
  });
}

extern "C" int abddc_mlp_train_step(abddc_mlp* mlp, const float* X, const float* T, int32_t n, float lr,
                                    float* loss) {
  return guarded([&]() -> int {
    abddc_mlp* w = checked(mlp);
    AllocScope as(&w->dalloc);
    ABDDC_REQUIRE(n > 0 && X && T, ABDDC_EINVAL, "bad batch");
    ABDDC_REQUIRE(lr > 0 && std::isfinite(lr), ABDDC_EINVAL, "learning rate must be > 0");
    StreamScope ss(w->stream);
    mlp_loss_grad_dev(w, X, T, n, w->stream);
    mlp_adam_dev(w, lr, w->stream);
    if (loss) {
      std::vector<float> l = to_host(w->loss.p, 1, w->stream);
      *loss = l[0];
    }
    return ABDDC_OK;
  });
}

extern "C" int abddc_mlp_set_ranges(abddc_mlp* mlp, const float* X, int32_t n) {
  return guarded([&]() -> int {
    abddc_mlp* w = checked(mlp);
    AllocScope as(&w->dalloc);
    ABDDC_REQUIRE(n > 0 && X, ABDDC_EINVAL, "bad feature set");
    StreamScope ss(w->stream);
    mlp_ranges_dev(w, X, n, w->stream);
    ABDDC_HIP(hipStreamSynchronize(w->stream));
    return ABDDC_OK;
  });
}

extern "C" void abddc_mlp_destroy(abddc_mlp* mlp) {
  if (!mlp) return;
  (void)hipSetDevice(mlp->device);
  (void)hipStreamSynchronize(mlp->stream);
  StreamScope ss(mlp->stream);
  delete mlp;
}

extern "C" int abddc_edge_features(abddc_ctx* c, float* X, int32_t* eligible) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(c, ABDDC_EINVAL, "null context");
    ABDDC_HIP(hipSetDevice(c->device));
    AllocScope as(&c->dalloc);
    StreamScope ss(c->stream);
    ABDDC_REQUIRE(c->element == ABDDC_ELEM_Q1 && !c->topo.general, ABDDC_EINVAL,
                  "edge features read one viscosity per box around straight edges: trilinear boxes on box "
                  "partitions only");
    const int ne = (int)c->topo.edges.size();
    if (ne == 0) return ABDDC_OK;
    ABDDC_REQUIRE(X, ABDDC_EINVAL, "null feature buffer");
    build_edge_geometry(c);
    launch_edge_features(c->d_egeom.p, ne, feature_params(c), c->d_nu.p, X, c->stream);
    if (eligible) {
      eligible_kernel<<<(ne + 255) / 256, 256, 0, c->stream>>>(c->d_egeom.p, ne, eligible);
      ABDDC_HIP(hipGetLastError());
    }
    ABDDC_HIP(hipStreamSynchronize(c->stream));
    return ABDDC_OK;
  });
}

extern "C" int abddc_edge_projectors(abddc_ctx* c, float* Y) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(c, ABDDC_EINVAL, "null context");
    ABDDC_REQUIRE(c->state >= 2, ABDDC_ESTATE, "setup_coarse_space has not run");
    ABDDC_HIP(hipSetDevice(c->device));
    AllocScope as(&c->dalloc);
    StreamScope ss(c->stream);
    const int ne = (int)c->topo.edges.size();
    if (ne == 0) return ABDDC_OK;
    ABDDC_REQUIRE(Y, ABDDC_EINVAL, "null output");
    build_edge_geometry(c);
    std::vector<int32_t> r(c->rE.begin(), c->rE.end());
    DevBuf<int32_t> dr = to_device(r, c->stream);
    DevBuf<int64_t> doff = to_device(c->teoff, c->stream);
    launch_edge_projectors(c->d_egeom.p, ne, c->dTE.p, doff.p, dr.p, Y, c->stream);
    ABDDC_HIP(hipStreamSynchronize(c->stream));
    return ABDDC_OK;
  });
}

extern "C" int abddc_learned_stats(const abddc_ctx* c, int32_t* n_predicted, int32_t* n_exact) {
  if (!c) return fail(ABDDC_EINVAL, "null context");
  if (n_predicted) *n_predicted = c->n_pred_edges;
  if (n_exact) *n_exact = c->n_exact_edges;
  return ABDDC_OK;
}
