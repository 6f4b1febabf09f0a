// C ABI entry points: assemble, setup_coarse_space, apply_bddc, apply_schur,
// gmres_solve and the query / parity hooks (include/abddc.h).
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstddef>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "apply.h"
#include "arena.h"
#include "assemble.h"
#include "ctx.h"
#include "guard.h"
#include "htrace.h"
#include "host_pool.h"
#include "internal.h"
#include "setup_k.h"

namespace abddc {
void run_setup(abddc_ctx* c);
void setup_final_check(abddc_ctx* c);
void plan_face_elimination(abddc_ctx* c, hipStream_t s);
}

using namespace abddc;

namespace {

double ev_ms(abddc_ctx* c, int a, int b) {
  float ms = 0.f;
  if (c->events && hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) == hipSuccess) return ms * 1e-3;
  return 0.0;
}

void record(abddc_ctx* c, int i) {
  if (c->events) ABDDC_HIP(hipEventRecord(c->ev[i], c->stream));
}

// Work vectors of one M^{-1} application: the local outputs [L; V] r_i and
// U x_Pi (length sum_i (n_B,i + n_Pi,i)), the coarse right-hand side and
// the coarse solution (length n_Pi each).  Every entry is written before it
// is read, so they need no clearing.
struct ApplyWork {
  double* out;
  double* bpi;
  double* xpi;
};

ApplyWork ctx_work(abddc_ctx* c) { return {c->d_out.p, c->d_bpi.p, c->d_xpi.p}; }

// z = M^{-1} r (device vectors of length n_gamma); with Z and st also
// Z[:, st->j] = z
void apply_bddc_dev(abddc_ctx* c, const double* r, double* z, hipStream_t s, const ApplyWork& w,
                    double* Z = nullptr, int64_t ldz = 0, const GmresState* st = nullptr) {
  const int np = c->n_primal;
  const bool mixed = c->dM32.p != nullptr;
  if (mixed)
    gemv_run<float>(c->opM, c->dM32.p, r, c->d_gam.p, w.out, false, s);
  else
    gemv_run<double>(c->opM, c->dM.p, r, c->d_gam.p, w.out, false, s);
  if (np > 0) {
    launch_gather_sum(c->d_pown_ptr.p, c->d_pown_idx.p, w.out, w.bpi, np, s);
    gemv_run<double>(c->opC, c->dSPinv.p, w.bpi, nullptr, w.xpi, false, s);
    if (mixed)
      gemv_run<float>(c->opU, c->dU32.p, w.xpi, c->d_pid.p, w.out, true, s);
    else
      gemv_run<double>(c->opU, c->dU.p, w.xpi, c->d_pid.p, w.out, true, s);
  }
  if (Z)
    launch_gather_sum_col(c->d_aown_ptr.p, c->d_aown_idx.p, w.out, z, Z, ldz, st, c->topo.n_gamma, s);
  else
    launch_gather_sum(c->d_aown_ptr.p, c->d_aown_idx.p, w.out, z, c->topo.n_gamma, s);
}

void apply_schur_dev(abddc_ctx* c, const double* x, double* y, hipStream_t s) {
  gemv_run<double>(c->opS, c->dS.p, x, c->d_gam.p, c->d_wS.p, false, s);
  launch_gather_sum(c->d_own_ptr.p, c->d_own_idx.p, c->d_wS.p, y, c->topo.n_gamma, s);
}

// Runtime objects of a context (timing events, the pinned scalar slots and
// their events, the capture stream), kept per device after a context is
// destroyed and handed to the next one: creating them costs more than a
// small solve.
struct CtxResources {
  hipEvent_t ev[20];
  double* h_step;
  double* dh_step;
  hipEvent_t ev_step[2];
  hipStream_t cap_stream;
};
std::mutex g_res_mu;
std::map<int, std::vector<CtxResources>> g_res_pool;

void acquire_resources(abddc_ctx* c) {
  CtxResources r{};
  bool have = false;
  {
    std::lock_guard<std::mutex> g(g_res_mu);
    std::vector<CtxResources>& v = g_res_pool[c->device];
    if (!v.empty()) {
      r = v.back();
      v.pop_back();
      have = true;
    }
  }
  if (!have) {
    for (int i = 0; i < 20; ++i) ABDDC_HIP(hipEventCreate(&r.ev[i]));
    // scalars the kernels publish straight to the host: two step slots and
    // the restart slot (pinned, device-coherent)
    ABDDC_HIP(hipHostMalloc(&r.h_step, 12 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
    ABDDC_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&r.dh_step), r.h_step, 0));
    for (int i = 0; i < 2; ++i) ABDDC_HIP(hipEventCreateWithFlags(&r.ev_step[i], hipEventDisableTiming));
    ABDDC_HIP(hipStreamCreateWithFlags(&r.cap_stream, hipStreamNonBlocking));
  }
  for (int i = 0; i < 20; ++i) c->ev[i] = r.ev[i];
  c->h_step = r.h_step;
  c->dh_step = r.dh_step;
  c->ev_step[0] = r.ev_step[0];
  c->ev_step[1] = r.ev_step[1];
  c->cap_stream = r.cap_stream;
  c->events = true;
}

// A destroyed context's topology (per-object and per-subdomain index lists,
// thousands of small allocations: ~0.5 ms to free on config3) is freed by one
// background thread, so that abddc_destroy returns without waiting for it.
// Host memory only; the thread and its queue live until the process ends.
void reap_topology(Topology&& t) {
  struct Reaper {
    std::mutex mu;
    std::condition_variable cv;
    std::vector<Topology> q;
    Reaper() {
      std::thread([this] {
        std::unique_lock<std::mutex> g(mu);
        for (;;) {
          cv.wait(g, [&] { return !q.empty(); });
          std::vector<Topology> batch;
          batch.swap(q);
          g.unlock();
          batch.clear();
          g.lock();
        }
      }).detach();
    }
  };
  static Reaper* r = new Reaper();   // never destroyed: its thread runs until exit
  {
    std::lock_guard<std::mutex> g(r->mu);
    r->q.push_back(std::move(t));
  }
  r->cv.notify_one();
}

void release_resources(abddc_ctx* c) {
  if (!c->events) return;
  CtxResources r{};
  for (int i = 0; i < 20; ++i) r.ev[i] = c->ev[i];
  r.h_step = c->h_step;
  r.dh_step = c->dh_step;
  r.ev_step[0] = c->ev_step[0];
  r.ev_step[1] = c->ev_step[1];
  r.cap_stream = c->cap_stream;
  std::lock_guard<std::mutex> g(g_res_mu);
  g_res_pool[c->device].push_back(r);
  c->events = false;
}

// One Arnoldi step of right-preconditioned FGMRES on stream s, every kernel
// taking the step index from the device state: z_j = M^{-1} v_j, Z[:, j] =
// z_j, w = Shat z_j, two classical Gram-Schmidt passes over V[:, 0..j], the
// norm, the Hessenberg column with Givens rotations, and v_{j+1} = w / h.
void arnoldi_step(abddc_ctx* c, int restart, hipStream_t s) {
  const int64_t n = c->topo.n_gamma;
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  GmresState* st = c->d_gst.p;
  apply_bddc_dev(c, c->d_vcur.p, c->d_zcur.p, s, ctx_work(c), c->d_Z.p, nn, st);   // also Z[:, j] = z_j
  apply_schur_dev(c, c->d_zcur.p, c->d_w.p, s);
  launch_dots_dev(c->d_V.p, nn, st, restart, c->d_w.p, n, c->d_partial.p, c->d_h1.p, s);
  // w -= V h1 with the second pass's products, w -= V h2 with the norm
  launch_axpy_dots_dev(c->d_V.p, nn, st, restart, c->d_h1.p, c->d_w.p, n, false, c->d_partial.p, c->d_h2.p, s);
  launch_axpy_dots_dev(c->d_V.p, nn, st, restart, c->d_h2.p, c->d_w.p, n, true, c->d_partial.p, c->d_nrm.p, s);
  launch_arnoldi_finish_dev(st, c->d_h1.p, c->d_h2.p, c->d_nrm.p, c->dh_step, s);
  launch_scale_to_col(c->d_w.p, st, c->d_V.p, nn, c->d_vcur.p, n, s);
}

// The Arnoldi step captured once per context (and restart length) into a
// HIP graph on a private capture stream; replays go to the context stream.
// Returns false (and the caller launches eagerly) when capture fails.
bool ensure_step_graph(abddc_ctx* c, int restart) {
  if (c->step_exec && c->step_restart == restart) return true;
  if (c->graph_failed) return false;
  if (c->step_exec) {
    (void)hipGraphExecDestroy(c->step_exec);
    (void)hipGraphDestroy(c->step_graph);
    c->step_exec = nullptr;
    c->step_graph = nullptr;
  }
  KStatsScope none(nullptr);   // no timing events inside the graph
  if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    c->graph_failed = true;
    return false;
  }
  bool ok = true;
  try {
    arnoldi_step(c, restart, c->cap_stream);
  } catch (const Error&) {
    ok = false;
  }
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(c->cap_stream, &g) != hipSuccess || !ok || !g) {
    (void)hipGetLastError();
    if (g) (void)hipGraphDestroy(g);
    c->graph_failed = true;
    return false;
  }
  hipGraphExec_t e = nullptr;
  if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g);
    c->graph_failed = true;
    return false;
  }
  c->step_graph = g;
  c->step_exec = e;
  c->step_restart = restart;
  return true;
}

// Coarse-space setup with validated options (the caller has set the scopes).
void setup_with(abddc_ctx* c, const abddc_options& o) {
  c->opt = o;
  c->n_ties = 0;
  c->state = 1;
  if (c->step_exec) {   // the captured Arnoldi step points at the previous setup's buffers
    ABDDC_HIP(hipStreamSynchronize(c->stream));
    (void)hipGraphExecDestroy(c->step_exec);
    (void)hipGraphDestroy(c->step_graph);
    c->step_exec = nullptr;
    c->step_graph = nullptr;
    c->step_restart = 0;
  }
  HostTrace ht;
  run_setup(c);
  ht.mark("setup: queued, stage buffers released");
  setup_final_check(c);
  c->kstats.resolve();
  ht.mark("setup: kernel statistics resolved");
  c->phase[2] = ev_ms(c, 2, 3);
  c->phase[3] = ev_ms(c, 3, 4);
  c->phase[4] = ev_ms(c, 4, 5);
  c->phase[5] = ev_ms(c, 5, 6);
  c->phase[6] = ev_ms(c, 6, 8);
  c->state = 2;
}

}  // namespace

extern "C" int abddc_assemble(const abddc_problem* prob, const abddc_device* dev, abddc_ctx** out) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(prob && dev && out, ABDDC_EINVAL, "null argument");
    *out = nullptr;
    for (int a = 0; a < 3; ++a) {
      ABDDC_REQUIRE(prob->nsub[a] >= 1 && prob->width[a], ABDDC_EINVAL, "bad nsub / width");
      ABDDC_REQUIRE(prob->length[a] > 0 && std::isfinite(prob->length[a]), ABDDC_EINVAL, "length must be > 0");
    }
    ABDDC_REQUIRE(prob->tau > 0 && std::isfinite(prob->tau), ABDDC_EINVAL, "tau must be > 0");
    ABDDC_REQUIRE(prob->nu, ABDDC_EINVAL, "nu is null");
    ABDDC_REQUIRE(prob->element == ABDDC_ELEM_Q1 || prob->element == ABDDC_ELEM_P1, ABDDC_EINVAL,
                  "element must be ABDDC_ELEM_Q1 or ABDDC_ELEM_P1");
    ABDDC_REQUIRE(!prob->a_nodal || prob->element == ABDDC_ELEM_P1, ABDDC_EINVAL,
                  "a_nodal needs element = ABDDC_ELEM_P1");
    ABDDC_REQUIRE(!prob->part || (prob->nsub[0] == 1 && prob->nsub[1] == 1 && prob->nsub[2] == 1), ABDDC_EINVAL,
                  "part needs nsub = {1, 1, 1} (width gives the grid)");
    ABDDC_REQUIRE(!prob->part || prob->n_parts >= 1, ABDDC_EINVAL, "part needs n_parts >= 1");
    for (int a = 0; a < 3; ++a)
      ABDDC_REQUIRE(std::isfinite(prob->origin[a]), ABDDC_EINVAL, "origin must be finite");
    ABDDC_REQUIRE((dev->alloc == nullptr) == (dev->free == nullptr), ABDDC_EINVAL,
                  "device allocation hooks: alloc and free must both be set or both be null");
    std::unique_ptr<abddc_ctx> c(new abddc_ctx());
    c->dalloc = DevAlloc{dev->alloc, dev->free, dev->user};
    AllocScope as(&c->dalloc);
    KStatsScope ks(&c->kstats);
    c->device = dev->device;
    ABDDC_HIP(hipSetDevice(dev->device));
    c->stream = (hipStream_t)dev->stream;
    hipStream_t s = c->stream;
    StreamScope ss(s);
    Topology& T = c->topo;
    int nsub_in[3] = {prob->nsub[0], prob->nsub[1], prob->nsub[2]};
    const int* w_in[3] = {prob->width[0], prob->width[1], prob->width[2]};
    HostTrace ht;
    T.build_grid(nsub_in, w_in);   // the interface objects follow once the element kernel is queued
    const bool on_dev = prob->arrays_on_device != 0;
    const int64_t n_nu = T.n_elem * (prob->element == ABDDC_ELEM_P1 ? 6 : 1);
    if (!on_dev) {
      for (int64_t e = 0; e < n_nu; ++e)
        ABDDC_REQUIRE(prob->nu[e] > 0 && std::isfinite(prob->nu[e]), ABDDC_EINVAL, "nu must be positive and finite");
      if (prob->a_nodal)
        for (int64_t q = 0; q < 3 * T.n_nodes; ++q)
          ABDDC_REQUIRE(std::isfinite(prob->a_nodal[q]), ABDDC_EINVAL, "a_nodal must be finite");
      if (prob->u_dirichlet)
        for (int64_t q = 0; q < T.n_nodes; ++q)
          ABDDC_REQUIRE(std::isfinite(prob->u_dirichlet[q]), ABDDC_EINVAL, "u_dirichlet must be finite");
    }
    c->element = prob->element;
    for (int a = 0; a < 3; ++a) {
      c->length[a] = prob->length[a];
      c->beta0[a] = prob->beta0[a];
    }
    for (int i = 0; i < 9; ++i) c->beta1[i] = prob->beta1[i];
    c->c = prob->c;
    c->f_const = prob->f_const;
    c->tau = prob->tau;
    acquire_resources(c.get());
    struct ResGuard {   // back to the pool if assembly fails
      abddc_ctx* c;
      ~ResGuard() {
        if (c) release_resources(c);
      }
    } res_guard{c.get()};
    c->d_flag.alloc(1);
    c->d_flag.zero(s);
    record(c.get(), 10);
    // coefficients, then the element matrices: they need no layout, so the
    // GPU computes them while the host builds the local maps below
    DevBuf<double> d_anodal, d_udir;
    if (on_dev) {
      c->d_nu.alloc(n_nu);
      ABDDC_HIP(hipMemcpyAsync(c->d_nu.p, prob->nu, n_nu * sizeof(double), hipMemcpyDeviceToDevice, s));
      launch_check_positive(c->d_nu.p, n_nu, c->d_flag.p, s);
      if (prob->f_nodal) {
        c->d_fnodal.alloc(T.n_nodes);
        ABDDC_HIP(hipMemcpyAsync(c->d_fnodal.p, prob->f_nodal, T.n_nodes * sizeof(double), hipMemcpyDeviceToDevice, s));
        c->have_fnodal = true;
      }
      if (prob->a_nodal) {
        d_anodal.alloc(3 * T.n_nodes);
        ABDDC_HIP(hipMemcpyAsync(d_anodal.p, prob->a_nodal, 3 * T.n_nodes * sizeof(double), hipMemcpyDeviceToDevice, s));
      }
      if (prob->u_dirichlet) {
        d_udir.alloc(T.n_nodes);
        ABDDC_HIP(hipMemcpyAsync(d_udir.p, prob->u_dirichlet, T.n_nodes * sizeof(double), hipMemcpyDeviceToDevice, s));
      }
    } else {
      std::vector<double> nu(prob->nu, prob->nu + n_nu);
      c->d_nu = to_device(nu, s);
      if (prob->f_nodal) {
        std::vector<double> fn(prob->f_nodal, prob->f_nodal + T.n_nodes);
        c->d_fnodal = to_device(fn, s);
        c->have_fnodal = true;
      }
      if (prob->a_nodal) d_anodal = to_device(std::vector<double>(prob->a_nodal, prob->a_nodal + 3 * T.n_nodes), s);
      if (prob->u_dirichlet)
        d_udir = to_device(std::vector<double>(prob->u_dirichlet, prob->u_dirichlet + T.n_nodes), s);
    }

    DevBuf<double> Ae(T.n_elem * 64), Fe(T.n_elem * 8);
    {
      ElemParams P{};
      P.n_elem = T.n_elem;
      for (int a = 0; a < 3; ++a) {
        P.ne[a] = T.ne[a];
        P.nn[a] = T.nn[a];
        P.h[a] = c->length[a] / T.ne[a];
        P.origin[a] = prob->origin[a];
        P.b0[a] = c->beta0[a];
      }
      for (int i = 0; i < 9; ++i) P.b1[i] = c->beta1[i];
      P.c = c->c;
      P.tau = c->tau;
      P.f_const = c->f_const;
      P.element = prob->element;
      const ElemFields F{c->have_fnodal ? c->d_fnodal.p : nullptr, d_anodal.p, d_udir.p};
      launch_elem(P, c->d_nu.p, F, Ae.p, Fe.p, s);
    }

    // box partitions: the dense local matrices (order n_loc = the free nodes
    // of the subdomain's box, one extra column) are sized from the cuts
    // alone, so their zero fill runs beside the host's topology and maps
    int64_t at_early = -1;
    if (!prob->part) {
      at_early = 0;
      for (int sz = 0; sz < T.nsub[2]; ++sz)
        for (int sy = 0; sy < T.nsub[1]; ++sy)
          for (int sx = 0; sx < T.nsub[0]; ++sx) {
            const int sc[3] = {sx, sy, sz};
            int64_t nl = 1;
            for (int a = 0; a < 3; ++a) {
              const int lo = std::max(T.cuts[a][sc[a]], 1), hi = std::min(T.cuts[a][sc[a] + 1], T.nn[a] - 2);
              nl *= std::max(0, hi - lo + 1);
            }
            at_early += nl * (nl + 1);
          }
      c->dA.alloc(std::max<int64_t>(at_early, 1));
      c->dA.zero(s);
    }
    ht.mark("assemble: coefficients, element kernel queued");
    if (prob->part) {
      T.build_partition(prob->part, prob->n_parts);
      for (int f : T.faces)
        ABDDC_REQUIRE(T.objects[f].n <= 512, ABDDC_EINVAL,
                      "partition: a face has more than 512 dofs (the eigensolvers' limit)");
      for (int e : T.edges)
        ABDDC_REQUIRE((int)T.objects[e].subs.size() <= MAX_EDGE_MEMBERS && T.objects[e].n <= 32, ABDDC_EINVAL,
                      "partition: an edge has more than 8 subdomains or more than 32 dofs");
    } else {
      T.build_objects();
    }
    ht.mark("assemble: topology");
    // ---------------------------------------------------- local layout
    const int nsub = T.n_sub;
    c->nI.resize(nsub);
    c->nB.resize(nsub);
    c->nloc.resize(nsub);
    c->aoff.resize(nsub);
    c->soff.resize(nsub);
    c->goff.resize(nsub);
    c->ioff.resize(nsub);
    int64_t at = 0, st = 0, gt = 0, it = 0, rows = 0, lmt = 0;
    std::vector<SubAsm> sa(nsub);
    // offsets of every subdomain in each array, serially; the maps are then
    // filled per subdomain in parallel
    for (int sub = 0; sub < nsub; ++sub) {
      const SubInfo& si = T.sub[sub];
      c->nI[sub] = si.nI;
      c->nB[sub] = si.nB;
      c->nloc[sub] = si.nI + si.nB;
      const int ld = c->nloc[sub] + 1;
      c->aoff[sub] = at;
      c->soff[sub] = st;
      c->goff[sub] = gt;
      c->ioff[sub] = it;
      SubAsm& a = sa[sub];
      a.aoff = at;
      a.soff = st;
      a.goff = gt;
      a.ioff = it;
      a.loff = rows;
      a.lmoff = (int32_t)lmt;
      a.nloc = c->nloc[sub];
      a.nI = si.nI;
      a.ld = ld;
      for (int ax = 0; ax < 3; ++ax) {
        a.ebox[2 * ax] = si.ebox[ax][0];
        a.ebox[2 * ax + 1] = si.ebox[ax][1];
      }
      at += (int64_t)c->nloc[sub] * ld;
      st += (int64_t)si.nB * si.nB;
      gt += si.nB;
      it += si.nI;
      lmt += (int64_t)(si.ebox[0][1] - si.ebox[0][0] + 1) * (si.ebox[1][1] - si.ebox[1][0] + 1) *
             (si.ebox[2][1] - si.ebox[2][0] + 1);
      rows += c->nloc[sub];
    }
    ABDDC_REQUIRE(T.n_nodes < (int64_t)1 << 31 && lmt < (int64_t)1 << 31, ABDDC_EINVAL, "mesh too large");
    // host arrays left uninitialised (a serial zero fill of these ~5 MB
    // would cost more than the parallel loop that writes every entry; each
    // subdomain clears its own range of the box map first)
    auto uninit = [](int64_t n) { return std::unique_ptr<int32_t[]>(new int32_t[std::max<int64_t>(n, 1)]); };
    auto lnode = uninit(rows), rowsub = uninit(rows), lmap = uninit(lmt), gam = uninit(gt), int_dof = uninit(it);
    host_parallel_for(nsub, 4, [&](int64_t sb, int64_t se) {
      for (int sub = (int)sb; sub < (int)se; ++sub) {
        const SubInfo& si = T.sub[sub];
        const SubAsm& a = sa[sub];
        // local node list [interior; Gamma_i] (interior nodes by node id,
        // then the nodes of every interface object) and the map from the
        // subdomain's bounding box of nodes to local positions
        const int e0[3] = {si.ebox[0][0], si.ebox[1][0], si.ebox[2][0]};
        const int bx = si.ebox[0][1] - e0[0] + 1, by = si.ebox[1][1] - e0[1] + 1;
        const int bz = si.ebox[2][1] - e0[2] + 1;
        const size_t b0 = (size_t)a.lmoff;
        std::fill(lmap.get() + b0, lmap.get() + b0 + (size_t)bx * by * bz, -1);
        int32_t* ln = lnode.get() + a.loff;
        int32_t* idof = int_dof.get() + a.ioff;
        int loc = 0;
        auto place = [&](int64_t v, bool interior) {
          const int ix = (int)(v % T.nn[0]), iy = (int)((v / T.nn[0]) % T.nn[1]);
          const int iz = (int)(v / ((int64_t)T.nn[0] * T.nn[1]));
          if (interior) idof[loc] = (int32_t)T.dof_of(v);
          ln[loc] = (int32_t)v;
          lmap[b0 + (ix - e0[0]) + (size_t)bx * ((iy - e0[1]) + (size_t)by * (iz - e0[2]))] = loc++;
        };
        for (int64_t v : si.interior) place(v, true);
        for (int k : si.objs)
          for (int64_t v : T.objects[k].nodes) place(v, false);
        ABDDC_REQUIRE(loc == a.nloc && (int)si.interior.size() == a.nI, ABDDC_EINVAL,
                      "local layout: node lists do not match the subdomain sizes");
        std::fill(rowsub.get() + a.loff, rowsub.get() + a.loff + loc, sub);
        for (int l = 0; l < si.nB; ++l) gam[a.goff + l] = (int32_t)si.gamma[l];
      }
    });
    ht.mark("assemble: local layout maps");
    c->d_subs = to_device(sa, s);
    DevBuf<int32_t> d_lnode = to_device(lnode.get(), rows, s), d_rowsub = to_device(rowsub.get(), rows, s),
                    d_lmap = to_device(lmap.get(), lmt, s);
    c->d_gam = to_device(gam.get(), gt, s);
    c->d_int_dof = to_device(int_dof.get(), it, s);
    std::vector<int32_t> iface_dof(T.n_gamma);
    host_parallel_for((int64_t)T.objects.size(), 64, [&](int64_t b, int64_t e) {
      for (int64_t k = b; k < e; ++k) {
        const Object& o = T.objects[k];
        for (int q = 0; q < o.n; ++q) iface_dof[o.gstart + q] = (int32_t)T.dof_of(o.nodes[q]);
      }
    });
    c->d_iface_dof = to_device(iface_dof, s);
    ht.mark("assemble: uploads");
    // -------------------------------------------- element matrices + scatter
    if (at_early < 0) {
      c->dA.alloc(std::max<int64_t>(at, 1));
      c->dA.zero(s);
    }
    ABDDC_REQUIRE(at_early < 0 || at_early == at, ABDDC_EINVAL, "internal: local matrix sizes from the cuts disagree");
    {
      DevBuf<int32_t> d_part;
      if (prob->part) d_part = to_device(std::vector<int32_t>(prob->part, prob->part + T.n_elem), s);
      launch_scatter(c->d_subs.p, d_rowsub.p, d_lnode.p, d_lmap.p, rows, T.nn, T.ne, Ae.p, Fe.p, d_part.p, c->dA.p, s);
      record(c.get(), 11);
      // interior elimination: S^(i), g^(i) in the trailing block / column
      std::vector<PluDesc<double>> pd;
      for (int sub = 0; sub < nsub; ++sub)
        pd.push_back({c->dA.p + c->aoff[sub], c->nloc[sub], c->nloc[sub] + 1, c->nloc[sub] + 1, c->nI[sub]});
      partial_lu<double>(pd, c->d_flag.p, s);
    }
    c->dS.alloc(std::max<int64_t>(st, 1));
    c->dB.alloc(std::max<int64_t>(st, 1));
    c->dg.alloc(std::max<int64_t>(gt, 1));
    int maxnB = 1;
    for (int sub = 0; sub < nsub; ++sub) maxnB = std::max(maxnB, c->nB[sub]);
    ht.mark("assemble: element kernels + interior elimination queued");
    launch_extract(c->d_subs.p, nsub, maxnB, c->dA.p, c->dS.p, c->dB.p, c->dg.p, s);

    // interface owners (goff space) and ghat = sum R_i^T g^(i)
    std::vector<int32_t> okey, oval, optr, oidx;
    for (int sub = 0; sub < nsub; ++sub)
      for (int l = 0; l < c->nB[sub]; ++l) {
        okey.push_back((int32_t)T.sub[sub].gamma[l]);
        oval.push_back((int32_t)(c->goff[sub] + l));
      }
    csr_group(T.n_gamma, okey, oval, optr, oidx);
    c->d_own_ptr = to_device(optr, s);
    c->d_own_idx = to_device(oidx, s);
    c->d_ghat.alloc(std::max<int64_t>(T.n_gamma, 1));
    launch_gather_sum(c->d_own_ptr.p, c->d_own_idx.p, c->dg.p, c->d_ghat.p, T.n_gamma, s);

    // Schur operator GEMV metadata
    std::vector<GemvMat> mS;
    double bytesS = 0.0;   // matrix + gathered input (value and index) + output
    for (int sub = 0; sub < nsub; ++sub) {
      const int nB = c->nB[sub];
      mS.push_back({c->soff[sub], c->goff[sub], c->goff[sub], nB, nB, std::max(nB, 1), 0});
      bytesS += (double)nB * nB * 8.0 + nB * 12.0 + nB * 8.0;
    }
    gemv_build(c->opS, mS, nullptr, bytesS, s);
    c->d_wS.alloc(std::max<int64_t>(gt, 1));
    gemv_tune<double>(c->opS, "schur", c->device, c->dS.p, c->d_ghat.p, c->d_gam.p, c->d_wS.p, s);
    ht.mark("assemble: owners, Schur GEMV metadata");
    record(c.get(), 12);
    // host work of the coarse-space setup that needs only the topology,
    // done while the device finishes the assembly
    plan_face_elimination(c.get(), s);
    ht.mark("assemble: face elimination plan");
    int h = 0;
    ABDDC_HIP(hipMemcpyAsync(&h, c->d_flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    ABDDC_HIP(hipStreamSynchronize(s));
    ht.mark("assemble: wait for the device");
    c->kstats.resolve();
    ABDDC_REQUIRE(!(h & 4), ABDDC_EINVAL, "nu must be positive and finite");
    ABDDC_REQUIRE(!(h & 1), ABDDC_ESINGULAR, "interior elimination: zero or non-finite pivot");
    c->phase[0] = ev_ms(c.get(), 10, 11);
    c->phase[1] = ev_ms(c.get(), 11, 12);
    c->state = 1;
    res_guard.c = nullptr;
    *out = c.release();
    return ABDDC_OK;
  });
}

extern "C" int abddc_setup_coarse_space(abddc_ctx* c, const abddc_options* opts, abddc_counts* counts) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(c, ABDDC_EINVAL, "null context");
    ABDDC_REQUIRE(c->state >= 1, ABDDC_ESTATE, "setup before assemble");
    ABDDC_HIP(hipSetDevice(c->device));
    abddc_options o{};
    o.theta_face = 10.0;
    o.theta_edge = 10.0;
    o.pinv_rtol = 1e-10;
    o.svd_rtol = 1e-8;
    o.tie_rtol = 1e-9;
    if (opts) o = *opts;
    ABDDC_REQUIRE(o.theta_face >= 0 && o.theta_edge >= 0, ABDDC_EINVAL, "thresholds must be >= 0");
    ABDDC_REQUIRE(o.edge_variant == ABDDC_EDGE_NEW || o.edge_variant == ABDDC_EDGE_OLD, ABDDC_EINVAL,
                  "bad edge_variant");
    ABDDC_REQUIRE(o.edge_variant == ABDDC_EDGE_NEW || o.constraint_source == ABDDC_CONSTRAINTS_EXACT, ABDDC_EINVAL,
                  "learned edge constraints predict the new edge eigenproblem's basis only");
    ABDDC_REQUIRE(o.edge_h_mode == ABDDC_H_SHARED || o.edge_h_mode == ABDDC_H_SEPARATE, ABDDC_EINVAL, "bad edge_h_mode");
    ABDDC_REQUIRE(o.deluxe_source == ABDDC_DELUXE_S || o.deluxe_source == ABDDC_DELUXE_B, ABDDC_EINVAL,
                  "bad deluxe_source");
    ABDDC_REQUIRE(o.precision == ABDDC_PREC_FP64 || o.precision == ABDDC_PREC_MIXED, ABDDC_EINVAL,
                  "bad precision mode");
    ABDDC_REQUIRE(o.constraint_source == ABDDC_CONSTRAINTS_EXACT || o.constraint_source == ABDDC_CONSTRAINTS_MLP,
                  ABDDC_EINVAL, "bad constraint source");
    ABDDC_REQUIRE(o.constraint_source != ABDDC_CONSTRAINTS_MLP || (o.mlp && o.mlp->device == c->device), ABDDC_EINVAL,
                  "learned constraints need a network on the context's device");
    ABDDC_REQUIRE(o.constraint_source != ABDDC_CONSTRAINTS_MLP || (c->element == ABDDC_ELEM_Q1 && !c->topo.general),
                  ABDDC_EINVAL,
                  "learned edge constraints read one viscosity per box around straight edges: trilinear boxes on box "
                  "partitions only");
    ABDDC_REQUIRE(o.pinv_rtol >= 0 && o.svd_rtol >= 0 && o.tie_rtol >= 0, ABDDC_EINVAL, "negative tolerance");
    ABDDC_REQUIRE(o.judge_iters >= 0 && o.judge_ratio >= 0 && std::isfinite(o.judge_ratio), ABDDC_EINVAL,
                  "bad judge settings");
    AllocScope as(&c->dalloc);
    KStatsScope ks(&c->kstats);
    StreamScope ss(c->stream);
    HostTrace().mark("setup: entry (since the last library mark)");
    setup_with(c, o);
    if (counts) *counts = {c->n_vertex, c->pnum_face, c->pnum_edge, c->n_primal, c->n_ties};
    return ABDDC_OK;
  });
}

extern "C" int abddc_apply_bddc(abddc_ctx* c, const double* r, double* z) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(c && r && z, ABDDC_EINVAL, "null argument");
    ABDDC_REQUIRE(c->state >= 2, ABDDC_ESTATE, "apply before setup");
    AllocScope as(&c->dalloc);
    KStatsScope ks(&c->kstats);
    apply_bddc_dev(c, r, z, c->stream, ctx_work(c));
    return ABDDC_OK;
  });
}

// ------------------------------------------- M^{-1} r without allocation
// Work vectors of abddc_apply_bddc_noalloc: one array per GPU, resident for
// the life of the process.  Host code never passes the array's name to a
// kernel (on the host it does not denote device memory); it uses the device
// address that hipGetSymbolAddress returns for the current device.
namespace {
static __device__ __align__(256) double scratch[ABDDC_NOALLOC_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (looked up once per device,
// with that device current).
double* scratch_for(int device) {
  ABDDC_REQUIRE(device >= 0 && device < MAX_DEVICES, ABDDC_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    ABDDC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    ABDDC_REQUIRE(ptr != nullptr, ABDDC_EDEVICE, "scratch array has no device address");
    g_scratch_ptr[device] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[device];
}
}  // namespace

extern "C" int abddc_apply_bddc_noalloc(abddc_ctx* c, const double* r, double* z) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(c && r && z, ABDDC_EINVAL, "null argument");
    ABDDC_REQUIRE(c->state >= 2, ABDDC_ESTATE, "apply before setup");
    const int64_t nout = (int64_t)c->d_out.n, np = std::max(c->n_primal, 1);
    const int64_t need = ((nout + 31) / 32) * 32 + 2 * ((np + 31) / 32) * 32;
    ABDDC_REQUIRE(need <= ABDDC_NOALLOC_SCRATCH_DOUBLES, ABDDC_EINVAL,
                  "abddc_apply_bddc_noalloc: the problem needs " + std::to_string(need) +
                      " doubles of work space, more than the fixed " +
                      std::to_string((long long)ABDDC_NOALLOC_SCRATCH_DOUBLES));
    ABDDC_HIP(hipSetDevice(c->device));
    double* base = scratch_for(c->device);
    ApplyWork w;
    w.out = base;
    w.bpi = base + ((nout + 31) / 32) * 32;
    w.xpi = w.bpi + ((np + 31) / 32) * 32;
    KStatsScope none(nullptr);   // no timing events (no event creation)
    apply_bddc_dev(c, r, z, c->stream, w);
    return ABDDC_OK;
  });
}

extern "C" int abddc_apply_schur(abddc_ctx* c, const double* x, double* y) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(c && x && y, ABDDC_EINVAL, "null argument");
    ABDDC_REQUIRE(c->state >= 1, ABDDC_ESTATE, "apply before assemble");
    AllocScope as(&c->dalloc);
    KStatsScope ks(&c->kstats);
    apply_schur_dev(c, x, y, c->stream);
    return ABDDC_OK;
  });
}

extern "C" int abddc_get_rhs(abddc_ctx* c, double* g) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(c && g, ABDDC_EINVAL, "null argument");
    ABDDC_REQUIRE(c->state >= 1, ABDDC_ESTATE, "rhs before assemble");
    if (c->topo.n_gamma)
      ABDDC_HIP(hipMemcpyAsync(g, c->d_ghat.p, c->topo.n_gamma * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return ABDDC_OK;
  });
}

namespace {
// One GMRES solve and the interior recovery (the caller has validated the
// arguments and set the scopes); fills info (may be null) and returns
// whether the true residual met rtol.
bool gmres_core(abddc_ctx* c, int32_t restart, double rtol, int32_t maxit, double* u, abddc_solve_info* info) {
    HostTrace ht;
    hipStream_t s = c->stream;
    const int64_t n = c->topo.n_gamma;
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    if (c->gm_restart < restart) {
      c->d_V.alloc((restart + 1) * nn);
      c->d_Z.alloc(restart * nn);
      c->gm_restart = restart;
    }
    if (!c->d_w.p) {
      c->d_w.alloc(nn);
      c->d_vcur.alloc(nn);
      c->d_zcur.alloc(nn);
      c->d_r.alloc(nn);
      c->d_x.alloc(nn);
      c->d_h1.alloc(GMRES_MAXR + 1);
      c->d_h2.alloc(GMRES_MAXR + 1);
      c->d_nrm.alloc(1);
      c->d_partial.alloc((size_t)DOT_BLOCKS * DOT_STRIDE);
      c->d_gst.alloc(1);
      // scalars the kernels publish straight to the host: two step slots and
      // the restart slot (pinned, device-coherent)
    }
    ht.mark("gmres: work vectors");
    const auto t0 = std::chrono::steady_clock::now();
    record(c, 13);
    double* V = c->d_V.p;
    double* Z = c->d_Z.p;
    const double* h_start = c->h_step + 8;   // beta, hn, inv_hn, res of the last restart
    auto read_scalars = [&]() { ABDDC_HIP(hipStreamSynchronize(s)); };
    int iters = 0, restarts = 0;
    double relres = 0.0;
    bool converged = false;
    ABDDC_HIP(hipMemsetAsync(c->d_x.p, 0, nn * sizeof(double), s));
    if (n > 0) {
      ABDDC_HIP(hipMemcpyAsync(c->d_r.p, c->d_ghat.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      launch_dots(c->d_r.p, n, 1, c->d_r.p, n, c->d_partial.p, c->d_nrm.p, s);
      launch_gmres_start(c->d_gst.p, c->d_nrm.p, c->dh_step + 8, s);
      ht.mark("gmres: initial residual queued");
      read_scalars();
      ht.mark("gmres: initial residual norm (sync)");
      const double bnorm = h_start[0];
      if (bnorm == 0.0) converged = true;
      const char* genv = std::getenv("ABDDC_GRAPH");
      const bool use_graph = !(genv && genv[0] == '0');
      bool eager_done = false;   // one eager step per call keeps the live kernel statistics
      while (!converged) {
        // cycle start: V[0] = v_cur = r / ||r|| (r, its norm and j = 0 in place)
        launch_scale_to_col(c->d_r.p, c->d_gst.p, V, nn, c->d_vcur.p, n, s);
        // Steps run one ahead of the convergence test: step j + 1 is queued
        // before the host waits for the scalars of step j (copied to a
        // pinned slot of their own), so the device does not idle during
        // the round trip.  A step queued past the exit is harmless: it
        // writes only column j + 1 of H, Z and V, its own rotation and
        // g[j + 1], g[j + 2], none of which the solution of the first
        // j + 1 columns reads, and the next cycle resets the state.
        auto launch_step = [&](int j) {
          if (use_graph && eager_done && ensure_step_graph(c, restart))
            ABDDC_HIP(hipGraphLaunch(c->step_exec, s));
          else
            arnoldi_step(c, restart, s);
          eager_done = true;   // the step's last kernel publishes its scalars to h_step[4 (j % 2) ..]
          ABDDC_HIP(hipEventRecord(c->ev_step[j & 1], s));
        };
        int jend = 0;
        launch_step(0);
        for (int j = 0; j < restart; ++j) {
          if (j + 1 < restart && iters + 1 < maxit) launch_step(j + 1);
          ABDDC_HIP(hipEventSynchronize(c->ev_step[j & 1]));
          ++iters;
          const double* sc = c->h_step + 4 * (j & 1);   // beta, hn, inv_hn, res
          const double res = sc[3];
          if (info && info->resid_history && iters <= info->resid_cap) info->resid_history[iters - 1] = res / bnorm;
          jend = j + 1;
          if (sc[1] == 0.0 || res <= rtol * bnorm || iters >= maxit) break;
        }
        launch_gmres_trisolve(c->d_gst.p, jend, s);
        launch_axpy_multi(Z, nn, jend, c->d_gst.p->y, 1.0, c->d_x.p, n, s);
        // true residual
        apply_schur_dev(c, c->d_x.p, c->d_w.p, s);
        launch_sub(c->d_ghat.p, c->d_w.p, c->d_r.p, n, s);
        launch_dots(c->d_r.p, n, 1, c->d_r.p, n, c->d_partial.p, c->d_nrm.p, s);
        launch_gmres_start(c->d_gst.p, c->d_nrm.p, c->dh_step + 8, s);
        read_scalars();
        const double beta = h_start[0];
        relres = beta / bnorm;
        if (beta <= rtol * bnorm) {
          converged = true;
          break;
        }
        if (iters >= maxit) break;
        ++restarts;
      }
    }
    record(c, 14);
    int max_nloc = 1;
    for (int sub = 0; sub < c->topo.n_sub; ++sub) max_nloc = std::max(max_nloc, c->nloc[sub]);
    launch_recover(c->d_subs.p, c->topo.n_sub, max_nloc, c->dA.p, c->d_gam.p, c->d_x.p, c->d_int_dof.p,
                   c->d_iface_dof.p, n, u, s);
    record(c, 15);
    ABDDC_HIP(hipStreamSynchronize(s));
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    c->kstats.resolve();
    c->phase[7] = ev_ms(c, 13, 14);
    c->phase[8] = ev_ms(c, 14, 15);
    if (info) {
      info->iters = iters;
      info->restarts = restarts;
      info->relres_true = relres;
      double ts = 0;
      for (int i = 0; i < 7; ++i) ts += c->phase[i];
      info->t_setup_s = ts;
      info->t_iter_s = wall;
      info->redone = 0;
      info->first_iters = iters;
    }
    return converged;
}
}  // namespace

extern "C" int abddc_gmres_solve(abddc_ctx* c, int32_t restart, double rtol, int32_t maxit, double* u,
                                 abddc_solve_info* info) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(c && u, ABDDC_EINVAL, "null argument");
    ABDDC_REQUIRE(c->state >= 2, ABDDC_ESTATE, "solve before setup");
    ABDDC_REQUIRE(restart >= 1 && restart <= GMRES_MAXR, ABDDC_EINVAL, "restart must be in [1, 63]");
    ABDDC_REQUIRE(rtol > 0 && rtol < 1, ABDDC_EINVAL, "rtol must be in (0, 1)");
    ABDDC_REQUIRE(maxit >= 1, ABDDC_EINVAL, "maxit must be >= 1");
    ABDDC_HIP(hipSetDevice(c->device));
    AllocScope as(&c->dalloc);
    KStatsScope ks(&c->kstats);
    StreamScope ss(c->stream);
    abddc_solve_info local{};
    abddc_solve_info* inf = info ? info : &local;
    bool converged = gmres_core(c, restart, rtol, maxit, u, inf);
    // Judge of the learned edge constraints: a solve that fails or needs
    // more than judge_ratio times the reference iteration count is redone
    // with every edge's constraints from the exact eigenproblem.
    const abddc_options& o = c->opt;
    const double ratio = o.judge_ratio > 0 ? o.judge_ratio : 1.2;
    if (o.constraint_source == ABDDC_CONSTRAINTS_MLP && c->n_pred_edges > 0 && o.judge_iters > 0 &&
        (!converged || inf->iters > ratio * o.judge_iters)) {
      const int first = inf->iters;
      const double t_first = inf->t_iter_s;
      abddc_options ex = o;
      ex.constraint_source = ABDDC_CONSTRAINTS_EXACT;
      const auto t0 = std::chrono::steady_clock::now();
      setup_with(c, ex);
      c->opt = o;   // the context keeps the caller's options; the constraints are now exact
      const double t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      converged = gmres_core(c, restart, rtol, maxit, u, inf);
      inf->redone = 1;
      inf->first_iters = first;
      inf->t_iter_s += t_first + t_setup;   // the whole call: first solve, exact setup, second solve
    }
    return converged ? ABDDC_OK : ABDDC_NOT_CONVERGED;
  });
}

extern "C" int abddc_query(const abddc_ctx* c, int64_t* n_dof, int64_t* n_gamma, int32_t* n_sub, int32_t* n_face,
                           int32_t* n_edge) {
  if (!c) return fail(ABDDC_EINVAL, "null context");
  if (n_dof) *n_dof = c->topo.n_dof;
  if (n_gamma) *n_gamma = c->topo.n_gamma;
  if (n_sub) *n_sub = c->topo.n_sub;
  if (n_face) *n_face = (int32_t)c->topo.faces.size();
  if (n_edge) *n_edge = (int32_t)c->topo.edges.size();
  return ABDDC_OK;
}

extern "C" int64_t abddc_get_stage(abddc_ctx* c, int32_t stage, int32_t index, double* buf, int64_t cap) {
  int64_t result = 0;
  int rc = guarded([&]() -> int {
    ABDDC_REQUIRE(c, ABDDC_EINVAL, "null context");
    ABDDC_REQUIRE(c->state >= 1, ABDDC_ESTATE, "stage before assemble");
    const Topology& T = c->topo;
    const double* src = nullptr;
    int64_t n = 0;
    std::vector<double> host;
    auto need_setup = [&]() { ABDDC_REQUIRE(c->state >= 2, ABDDC_ESTATE, "stage needs setup"); };
    switch (stage) {
      case ABDDC_STAGE_SCHUR:
        ABDDC_REQUIRE(index >= 0 && index < T.n_sub, ABDDC_EINVAL, "bad subdomain index");
        src = c->dS.p + c->soff[index];
        n = (int64_t)c->nB[index] * c->nB[index];
        break;
      case ABDDC_STAGE_LOCAL_RHS:
        ABDDC_REQUIRE(index >= 0 && index < T.n_sub, ABDDC_EINVAL, "bad subdomain index");
        src = c->dg.p + c->goff[index];
        n = c->nB[index];
        break;
      case ABDDC_STAGE_FACE_EIG:
      case ABDDC_STAGE_FACE_BASIS: {
        need_setup();
        ABDDC_REQUIRE(index >= 0 && index < (int)T.faces.size(), ABDDC_EINVAL, "bad face index");
        const int nF = T.objects[T.faces[index]].n;
        src = stage == ABDDC_STAGE_FACE_EIG ? c->dWF.p + c->wfoff[index] : c->dTF.p + c->tfoff[index];
        n = stage == ABDDC_STAGE_FACE_EIG ? nF : (int64_t)nF * nF;
        break;
      }
      case ABDDC_STAGE_EDGE_EIG:
      case ABDDC_STAGE_EDGE_BASIS: {
        need_setup();
        ABDDC_REQUIRE(index >= 0 && index < (int)T.edges.size(), ABDDC_EINVAL, "bad edge index");
        const Object& o = T.objects[T.edges[index]];
        src = stage == ABDDC_STAGE_EDGE_EIG ? c->dWE.p + c->weoff[index] : c->dTE.p + c->teoff[index];
        const int64_t neig = (c->opt.edge_variant == ABDDC_EDGE_OLD ? 1 : (int64_t)o.subs.size() - 1) * o.n;
        n = stage == ABDDC_STAGE_EDGE_EIG ? neig : (int64_t)o.n * o.n;
        break;
      }
      case ABDDC_STAGE_COUNTS:
        need_setup();
        for (int v : c->pF) host.push_back(v);
        for (int v : c->rE) host.push_back(v);
        n = (int64_t)host.size();
        break;
      case ABDDC_STAGE_SUB_SIZES:
        ABDDC_REQUIRE(index >= 0 && index < T.n_sub, ABDDC_EINVAL, "bad subdomain index");
        host = {(double)c->nI[index], (double)c->nB[index],
                c->state >= 2 && (size_t)index < c->nPi.size() ? (double)c->nPi[index] : 0.0};
        n = 3;
        break;
      case ABDDC_STAGE_DELUXE: {
        need_setup();
        const int obj = index / 8, mem = index % 8;
        ABDDC_REQUIRE(obj >= 0 && obj < (int)T.objects.size() && c->dxoff[(size_t)index] >= 0, ABDDC_EINVAL,
                      "bad deluxe index");
        src = c->dD.p + c->dxoff[(size_t)obj * 8 + mem];
        n = (int64_t)T.objects[obj].n * T.objects[obj].n;
        break;
      }
      default:
        throw Error(ABDDC_EINVAL, "unknown stage");
    }
    result = n;
    if (buf && cap >= n && n > 0) {
      if (src) {
        ABDDC_HIP(hipMemcpyAsync(buf, src, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        ABDDC_HIP(hipStreamSynchronize(c->stream));
      } else {
        std::copy(host.begin(), host.end(), buf);
      }
    }
    return ABDDC_OK;
  });
  return rc < 0 ? rc : result;
}

extern "C" int abddc_kernel_stats(abddc_ctx* c, int32_t kernel, double* seconds, int64_t* launches,
                                  double* work) {
  return guarded([&]() -> int {
    ABDDC_REQUIRE(c, ABDDC_EINVAL, "null context");
    ABDDC_REQUIRE(kernel >= 0 && kernel < KC_COUNT, ABDDC_EINVAL, "unknown kernel class");
    ABDDC_HIP(hipStreamSynchronize(c->stream));
    c->kstats.resolve();
    if (seconds) *seconds = c->kstats.seconds[kernel];
    if (launches) *launches = c->kstats.launches[kernel];
    if (work) *work = c->kstats.work[kernel];
    return ABDDC_OK;
  });
}

extern "C" int abddc_phase_times(const abddc_ctx* c, double* t, int32_t n) {
  if (!c || !t || n < 0) return fail(ABDDC_EINVAL, "null argument");
  for (int i = 0; i < n && i < 16; ++i) t[i] = c->phase[i];
  return ABDDC_OK;
}

extern "C" void abddc_destroy(abddc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  StreamScope ss(c->stream);
  HostTrace ht;
  (void)hipStreamSynchronize(c->stream);
  ht.mark("destroy: stream drained");
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  if (c->step_graph) (void)hipGraphDestroy(c->step_graph);
  ht.mark("destroy: Arnoldi-step graph");
  release_resources(c);
  reap_topology(std::move(c->topo));
  delete c;
  ht.mark("destroy: buffers released");
}
