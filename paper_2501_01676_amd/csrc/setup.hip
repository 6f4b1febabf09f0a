// Host orchestration of the adaptive coarse-space setup (Section 3):
// deluxe weights, face eigenproblems (eq. equ-4-8), new edge eigenproblems
// (eq. equ-5-21) with the SVD/QR edge basis, change of basis, the local
// constrained factorisations, the coarse matrix, and the per-iteration
// operators of M^{-1}.  Each stage is a few batched launches over all
// faces / edges / subdomains; the host only builds index maps and
// descriptors and reads back the primal counts.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <cstdlib>
#include <cmath>

#include "apply.h"
#include "arena.h"
#include "ctx.h"
#include "host_pool.h"
#include "htrace.h"
#include "internal.h"
#include "mlp.h"
#include "setup_k.h"

namespace abddc {

namespace {

struct IntPool {
  // Concatenated host int arrays uploaded once (stream-ordered, through the
  // pinned staging ring); device pointers handed out by offset.
  std::vector<int32_t> h;
  DevBuf<int32_t> d;
  size_t add(const std::vector<int32_t>& v) {
    size_t off = h.size();
    h.insert(h.end(), v.begin(), v.end());
    return off;
  }
  // n uninitialised entries at the end, filled later through h.data() + off
  // (after every block is reserved, so the storage no longer moves)
  size_t reserve(size_t n) {
    size_t off = h.size();
    h.resize(off + n);
    return off;
  }
  void upload(hipStream_t s) {
    d.alloc(std::max<size_t>(h.size(), 1));
    if (!h.empty()) staged_upload(d.p, h.data(), h.size() * sizeof(int32_t), s);
  }
  const int32_t* ptr(size_t off) const { return d.p + off; }
};

// Generalized eigenproblems of the face / edge constraints: every mu, and
// the eigenvectors of mu <= sel (the only ones the constraints use).
// ABDDC_SYGV_JACOBI=1 takes the full Jacobi solver instead (all vectors).
void eig_selected(const std::vector<SygvDesc>& gv, double sel, int* dflag, hipStream_t s) {
  static const bool jacobi = [] {
    const char* e = std::getenv("ABDDC_SYGV_JACOBI");
    return e && *e == '1';
  }();
  if (jacobi) sygv_batched(gv, dflag, s);
  else sygv_select_batched(gv, sel, dflag, s);
}

void record(abddc_ctx* c, int i) {
  if (c->events) ABDDC_HIP(hipEventRecord(c->ev[i], c->stream));
}

int check_flag(abddc_ctx* c) {
  int h = 0;
  ABDDC_HIP(hipMemcpyAsync(&h, c->d_flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  ABDDC_HIP(hipStreamSynchronize(c->stream));
  return h;
}

void throw_on_flag(int h, const char* stage) {
  if (h & 1) throw Error(ABDDC_ESINGULAR, std::string(stage) + ": zero or non-finite pivot");
  if (h & 2) throw Error(ABDDC_EEIG, std::string(stage) + ": eigenproblem metric not positive definite");
}

void require_flag_clean(abddc_ctx* c, const char* stage) { throw_on_flag(check_flag(c), stage); }

// The n eigenvalues at d and the error flag, read back through pinned memory
// behind one wait; the flag is then checked as require_flag_clean does.
std::vector<double> eigenvalues_checked(abddc_ctx* c, const double* d, size_t n, const char* stage) {
  int32_t* buf = pinned_ints(2 * n + 2);   // n doubles, then the flag
  double* hv = reinterpret_cast<double*>(buf);
  int32_t* hf = buf + 2 * n;
  ABDDC_HIP(hipMemcpyAsync(hf, c->d_flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  if (n) ABDDC_HIP(hipMemcpyAsync(hv, d, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  ABDDC_HIP(hipStreamSynchronize(c->stream));
  throw_on_flag(*hf, stage);
  return std::vector<double>(hv, hv + n);
}

// Learned edge constraints: features -> network -> P-hat -> eigenpairs;
// the gate keeps an edge's prediction (basis = eigenvectors of P-hat with
// eigenvalue > 1/2, completed by QR into the edge basis) or appends the
// edge to `exact`.
void learned_edges(abddc_ctx* c, std::vector<int>& exact) {
  const Topology& T = c->topo;
  hipStream_t s = c->stream;
  const int ned = (int)T.edges.size();
  abddc_mlp* w = const_cast<abddc_mlp*>(c->opt.mlp);
  ABDDC_HIP(hipStreamSynchronize(w->stream));   // training launched on the network's stream has finished
  build_edge_geometry(c);
  DevBuf<float> X((size_t)ned * MLP_IN), Y((size_t)ned * MLP_OUT);
  launch_edge_features(c->d_egeom.p, ned, feature_params(c), c->d_nu.p, X.p, s);
  mlp_forward_dev(w, X.p, ned, Y.p, s);
  DevBuf<double> P((size_t)ned * 49), I((size_t)ned * 49), W((size_t)ned * 7), V((size_t)ned * 49);
  launch_phat(Y.p, ned, P.p, I.p, s);
  std::vector<SygvDesc> gv;
  for (int e = 0; e < ned; ++e)
    if (c->egeom[e].eligible) gv.push_back({P.p + 49 * e, I.p + 49 * e, W.p + 7 * e, V.p + 49 * e, MLP_NE});
  sygv_batched(gv, c->d_flag.p, s);
  DevBuf<int32_t> flag(std::max(ned, 1));
  flag.zero(s);
  if (w->have_ranges) launch_range_flags(X.p, ned, w->fmin.p, w->fmax.p, 0.1f, flag.p, s);
  std::vector<double> lam = to_host(W.p, (size_t)ned * 7, s);
  std::vector<int32_t> out = to_host(flag.p, ned, s);
  std::vector<QrDesc> qd;
  for (int e = 0; e < ned; ++e) {
    bool keep = c->egeom[e].eligible && !out[e];
    int r = 0;
    for (int q = 0; keep && q < MLP_NE; ++q) {
      const double l = lam[7 * e + q];
      if (l >= 0.3 && l <= 0.7) keep = false;
      if (l > 0.5) ++r;
    }
    if (!keep) {
      exact.push_back(e);
      continue;
    }
    c->rE[e] = r;
    c->nselE[e] = 0;
    qd.push_back({V.p + 49 * e + (MLP_NE - r), c->dTE.p + c->teoff[e], MLP_NE, r, MLP_NE});
  }
  qr_complete_batched(qd, s);
}

}  // namespace

// Index plan of the staged face eliminations: topology and interface sizes
// only, so assemble builds it while the device works.  The Schur complement
// of B^(nu) onto F, eliminating Gamma_nu minus F, is taken in three steps
// (Schur complements compose, so the work the faces of one subdomain share
// is done once):
//   (1) per subdomain: eliminate the edge and vertex dofs, leaving C on the
//       face dofs of Gamma_nu, ordered by normal axis;
//   (2) per (subdomain, axis): eliminate from C the faces normal to the
//       other axes, leaving the block of the one or two faces normal to this
//       axis;
//   (3) per face of a two-face block: eliminate the opposite face.
void plan_face_elimination(abddc_ctx* c, hipStream_t s) {
  const Topology& T = c->topo;
  const int nsub = T.n_sub, nf = (int)T.faces.size();
  FaceElimPlan& P = c->fplan;
  P = FaceElimPlan();
  auto face_axis = [&](int k) {
    // general partitions: every face is a group of its own, so step (3)
    // never runs and step (2) leaves exactly that face
    if (T.general) return 3 + T.kind_index[k];
    const int a = T.objects[k].subs[0], b = T.objects[k].subs[1];
    if (a % T.nsub[0] != b % T.nsub[0]) return 0;
    if ((a / T.nsub[0]) % T.nsub[1] != (b / T.nsub[0]) % T.nsub[1]) return 1;
    return 2;
  };
  struct FacePart { int f, side, off, n, axis; };
  std::vector<std::vector<FacePart>> sfaces(nsub);
  for (int f = 0; f < nf; ++f) {
    const int k = T.faces[f];
    for (int side = 0; side < 2; ++side) {
      const int sub = T.objects[k].subs[side];
      sfaces[sub].push_back({f, side, T.sub[sub].local_pos(k), T.objects[k].n, face_axis(k)});
    }
  }
  P.m1off.assign(nsub, 0);
  P.nR.assign(nsub, 0);
  P.nC.assign(nsub, 0);
  P.res3.assign(2 * nf, -1);
  P.k3of.assign(2 * nf, 0);
  P.ng3.assign(2 * nf, 0);
  P.grp_of.assign(2 * nf, -1);
  P.m3off.assign(2 * nf, 0);
  // (a) per subdomain, in parallel: its maps in pool order (step (1), then
  // per group the step (2) map and the step (3) maps of its faces) with
  // offsets relative to the subdomain's block; (b) serially, the blocks'
  // pool offsets, the group numbers and the work-array offsets in subdomain
  // order; (c) in parallel, every block into the pool
  struct FaceRec { int id, k3, ng3; int64_t m3; };   // m3: relative offset, -1 without step (3)
  struct GroupRec { FaceElimPlan::Group g; std::vector<FaceRec> faces; };
  struct SubPlan { std::vector<int32_t> ints; std::vector<GroupRec> groups; };
  std::vector<SubPlan> sp(nsub);
  host_parallel_for(nsub, 8, [&](int64_t sb, int64_t se) {
    for (int sub = (int)sb; sub < (int)se; ++sub) {
      std::vector<FacePart>& fp = sfaces[sub];
      if (fp.empty()) continue;
      std::stable_sort(fp.begin(), fp.end(), [](const FacePart& a, const FacePart& b) {
        return a.axis != b.axis ? a.axis < b.axis : a.off < b.off;
      });
      SubPlan& S = sp[sub];
      std::vector<int32_t>& v = S.ints;
      const int nB = c->nB[sub];
      std::vector<char> isface(nB, 0);
      for (const FacePart& q : fp)
        for (int t = 0; t < q.n; ++t) isface[q.off + t] = 1;
      for (int t = 0; t < nB; ++t)
        if (!isface[t]) v.push_back(t);
      const int nR = (int)v.size();
      std::vector<int> cpos(fp.size());
      for (size_t i = 0; i < fp.size(); ++i) {
        cpos[i] = (int)v.size() - nR;
        for (int t = 0; t < fp[i].n; ++t) v.push_back(fp[i].off + t);
      }
      P.nR[sub] = nR;
      const int nC = nB - nR;
      P.nC[sub] = nC;
      for (size_t i = 0; i < fp.size();) {
        size_t j = i + 1;
        while (j < fp.size() && fp[j].axis == fp[i].axis) ++j;
        GroupRec gr;
        FaceElimPlan::Group& g = gr.g;
        g.sub = sub;
        g.nfaces = (int)(j - i);
        g.cpos = cpos[i];
        g.ng = 0;
        for (size_t q = i; q < j; ++q) g.ng += fp[q].n;
        g.k2 = nC - g.ng;
        g.o2 = 0;
        g.m2 = v.size();
        for (int t = 0; t < nC; ++t)
          if (t < g.cpos || t >= g.cpos + g.ng) v.push_back(t);
        for (int t = 0; t < g.ng; ++t) v.push_back(g.cpos + t);
        int inner = 0;
        for (size_t q = i; q < j; ++q) {
          FaceRec fr{2 * fp[q].f + fp[q].side, g.ng - fp[q].n, g.ng, -1};
          if (g.nfaces > 1) {
            // [the other face of the pair; this face] inside the pair block
            fr.m3 = (int64_t)v.size();
            for (int t = 0; t < g.ng; ++t)
              if (t < inner || t >= inner + fp[q].n) v.push_back(t);
            for (int t = 0; t < fp[q].n; ++t) v.push_back(inner + t);
          }
          gr.faces.push_back(fr);
          inner += fp[q].n;
        }
        S.groups.push_back(std::move(gr));
        i = j;
      }
    }
  });
  std::vector<size_t> base(nsub + 1, 0);
  for (int sub = 0; sub < nsub; ++sub) {
    base[sub + 1] = base[sub] + sp[sub].ints.size();
    if (sp[sub].ints.empty()) continue;
    P.m1off[sub] = base[sub];
    const int nC = P.nC[sub];
    for (GroupRec& gr : sp[sub].groups) {
      FaceElimPlan::Group g = gr.g;
      g.o2 = P.w2tot;
      g.m2 += base[sub];
      P.w2tot += (int64_t)nC * nC;
      const int gi = (int)P.groups.size();
      P.groups.push_back(g);
      for (const FaceRec& fr : gr.faces) {
        P.grp_of[fr.id] = gi;
        if (fr.m3 < 0) continue;
        P.m3off[fr.id] = base[sub] + (size_t)fr.m3;
        P.res3[fr.id] = P.w3tot;
        P.k3of[fr.id] = fr.k3;
        P.ng3[fr.id] = fr.ng3;
        P.w3tot += (int64_t)fr.ng3 * fr.ng3;
      }
    }
  }
  const size_t total = base[nsub];
  std::unique_ptr<int32_t[]> pool(new int32_t[std::max<size_t>(total, 1)]);
  host_parallel_for(nsub, 16, [&](int64_t sb, int64_t se) {
    for (int64_t sub = sb; sub < se; ++sub)
      std::copy(sp[sub].ints.begin(), sp[sub].ints.end(), pool.get() + base[sub]);
  });
  P.d_pool.alloc(std::max<size_t>(total, 1));
  if (total) staged_upload(P.d_pool.p, pool.get(), total * sizeof(int32_t), s);
  P.ready = true;
}

void run_setup(abddc_ctx* c) {
  const Topology& T = c->topo;
  hipStream_t s = c->stream;
  const int nsub = T.n_sub;
  const int nf = (int)T.faces.size(), ned = (int)T.edges.size(), nvx = (int)T.vertices.size();
  const bool useS = c->opt.deluxe_source == ABDDC_DELUXE_S;
  const double* src_dx = useS ? c->dS.p : c->dB.p;
  auto Sblk = [&](const double* base, int sub, int obj) {
    const int off = T.sub[sub].local_pos(obj);
    return base + c->soff[sub] + (int64_t)off * c->nB[sub] + off;
  };
  HostTrace ht;
  c->d_flag.zero(s);

  ht.mark("deluxe");
  // ------------------------------------------------------------ deluxe
  record(c, 2);
  const int nobj = (int)T.objects.size();
  c->dxoff.assign((size_t)nobj * 8, -1);
  int64_t dxtot = 0;
  for (int k = 0; k < nobj; ++k) {
    const Object& o = T.objects[k];
    if (o.kind == KIND_VERTEX) continue;
    for (size_t q = 0; q < o.subs.size(); ++q) {
      c->dxoff[(size_t)k * 8 + q] = dxtot;
      dxtot += (int64_t)o.n * o.n;
    }
  }
  c->dD.alloc(std::max<int64_t>(dxtot, 1));
  {
    std::vector<int64_t> woff(nobj, -1);
    int64_t wtot = 0;
    for (int k = 0; k < nobj; ++k) {
      const Object& o = T.objects[k];
      if (o.kind == KIND_VERTEX) continue;
      woff[k] = wtot;
      wtot += (int64_t)2 * o.n * (o.subs.size() + 1) * o.n;
    }
    DevBuf<double> wk(std::max<int64_t>(wtot, 1));
    ht.mark("deluxe: offsets, buffers");
    // descriptors of the faces and edges (objects before the vertices), one
    // slot each, filled in parallel
    const int nfe = nf + ned;
    std::vector<int64_t> gstart(nfe + 1, 0);
    for (int k = 0; k < nfe; ++k) gstart[k + 1] = gstart[k] + (int64_t)T.objects[k].subs.size();
    std::vector<DeluxeDesc> dd(nfe);
    std::vector<PluDesc<double>> pd(nfe);
    std::vector<GatherDesc> gd(gstart[nfe]);
    host_parallel_for(nfe, 64, [&](int64_t kb, int64_t ke) {
      for (int k = (int)kb; k < (int)ke; ++k) {
        const Object& o = T.objects[k];
        DeluxeDesc d{};
        d.n = o.n;
        d.m = (int)o.subs.size();
        for (int q = 0; q < d.m; ++q) {
          d.src[q] = Sblk(src_dx, o.subs[q], k);
          d.lds[q] = c->nB[o.subs[q]];
        }
        d.dst = wk.p + woff[k];
        dd[k] = d;
        const int cols = (d.m + 1) * o.n;
        pd[k] = {wk.p + woff[k], 2 * o.n, cols, cols, o.n};
        for (int q = 0; q < d.m; ++q)
          gd[gstart[k] + q] = {wk.p + woff[k] + (int64_t)o.n * cols + o.n + (int64_t)q * o.n,
                               c->dD.p + c->dxoff[(size_t)k * 8 + q], nullptr, nullptr, o.n, o.n, cols, o.n, 1.0};
      }
    });
    ht.mark("deluxe: descriptors");
    deluxe_build_batched(dd, s);
    partial_lu<double>(pd, c->d_flag.p, s);
    gather_batched(gd, s);
  }

  ht.mark("faces");
  // ------------------------------------------------------------- faces
  record(c, 3);
  c->pF.assign(nf, 0);
  c->tfoff.assign(nf, 0);
  c->wfoff.assign(nf, 0);
  int64_t ftot = 0;
  for (int f = 0; f < nf; ++f) {
    c->tfoff[f] = ftot;
    c->wfoff[f] = 0;
    ftot += (int64_t)T.objects[T.faces[f]].n * T.objects[T.faces[f]].n;
  }
  {
    int64_t wsum = 0;
    for (int f = 0; f < nf; ++f) {
      c->wfoff[f] = wsum;
      wsum += T.objects[T.faces[f]].n;
    }
    c->dWF.alloc(std::max<int64_t>(wsum, 1));
  }
  c->dTF.alloc(std::max<int64_t>(ftot, 1));
  if (nf > 0) {
    DevBuf<double> W1(ftot), W2(ftot), BF(ftot), Sum(ftot), XF(ftot);
    ht.mark("B_F = D_j^T B_F^(i) D_j + D_i^T B_F^(j");
    // B_F = D_j^T B_F^(i) D_j + D_i^T B_F^(j) D_i
    std::vector<GemmDesc<double>> g1, g2, g3;
    for (int f = 0; f < nf; ++f) {
      const int k = T.faces[f];
      const Object& o = T.objects[k];
      const int i = o.subs[0], j = o.subs[1], n = o.n;
      const double* Di = c->dD.p + c->dxoff[(size_t)k * 8 + 0];
      const double* Dj = c->dD.p + c->dxoff[(size_t)k * 8 + 1];
      g1.push_back({Sblk(c->dB.p, i, k), Dj, W1.p + c->tfoff[f], n, n, n, c->nB[i], n, n});
      g1.push_back({Sblk(c->dB.p, j, k), Di, W2.p + c->tfoff[f], n, n, n, c->nB[j], n, n});
      g2.push_back({Dj, W1.p + c->tfoff[f], BF.p + c->tfoff[f], n, n, n, n, n, n});
      g3.push_back({Di, W2.p + c->tfoff[f], BF.p + c->tfoff[f], n, n, n, n, n, n});
    }
    gemm_batched<double>(g1, false, false, 1.0, 0.0, s);
    gemm_batched<double>(g2, true, false, 1.0, 0.0, s);
    gemm_batched<double>(g3, true, false, 1.0, 1.0, s);

    ht.mark("Btilde_F^(nu): Schur complement of B^(");
    // Btilde_F^(nu): Schur complement of B^(nu) onto F, eliminating
    // Gamma_nu minus F, in the three steps of plan_face_elimination.  Every
    // step is a symmetric gather and a partial LU.  Each pivot block is
    // a Schur complement of a principal submatrix of the one-step pivot block
    // B_{Gamma minus F}, so it is positive definite whenever that one is.
    if (!c->fplan.ready) plan_face_elimination(c, s);
    const FaceElimPlan& P = c->fplan;
    std::vector<const double*> res(2 * nf);
    std::vector<int> resld(2 * nf);
    auto pptr = [&](size_t off) { return P.d_pool.p + off; };
    DevBuf<double> Q1(c->dB.n), Q2(std::max<int64_t>(P.w2tot, 1)), Q3(std::max<int64_t>(P.w3tot, 1));
    {
      std::vector<GatherDesc> gd;
      std::vector<PluDesc<double>> pd;
      for (int sub = 0; sub < nsub; ++sub) {
        if (P.nC[sub] == 0) continue;   // no face dofs
        const int nB = c->nB[sub];
        gd.push_back({c->dB.p + c->soff[sub], Q1.p + c->soff[sub], pptr(P.m1off[sub]), pptr(P.m1off[sub]), nB, nB,
                      nB, nB, 1.0});
        pd.push_back({Q1.p + c->soff[sub], nB, nB, nB, P.nR[sub]});
      }
      gather_batched(gd, s);
      partial_lu<double>(pd, c->d_flag.p, s);
    }
    {
      std::vector<GatherDesc> gd;
      std::vector<PluDesc<double>> pd;
      for (const FaceElimPlan::Group& g : P.groups) {
        const int nB = c->nB[g.sub], n2 = P.nC[g.sub];
        const double* Cb = Q1.p + c->soff[g.sub] + (int64_t)P.nR[g.sub] * nB + P.nR[g.sub];
        gd.push_back({Cb, Q2.p + g.o2, pptr(g.m2), pptr(g.m2), n2, n2, nB, n2, 1.0});
        pd.push_back({Q2.p + g.o2, n2, n2, n2, g.k2});
      }
      gather_batched(gd, s);
      partial_lu<double>(pd, c->d_flag.p, s);
    }
    {
      std::vector<GatherDesc> gd;
      std::vector<PluDesc<double>> pd;
      for (int id = 0; id < 2 * nf; ++id) {
        const FaceElimPlan::Group& g = P.groups[P.grp_of[id]];
        const int n2 = P.nC[g.sub];
        const double* Pb = Q2.p + g.o2 + (int64_t)g.k2 * n2 + g.k2;   // block of the group's faces
        if (P.res3[id] < 0) {
          res[id] = Pb;
          resld[id] = n2;
          continue;
        }
        const int ng = P.ng3[id], k3 = P.k3of[id];
        gd.push_back({Pb, Q3.p + P.res3[id], pptr(P.m3off[id]), pptr(P.m3off[id]), ng, ng, n2, ng, 1.0});
        pd.push_back({Q3.p + P.res3[id], ng, ng, ng, k3});
        res[id] = Q3.p + P.res3[id] + (int64_t)k3 * ng + k3;
        resld[id] = ng;
      }
      gather_batched(gd, s);
      partial_lu<double>(pd, c->d_flag.p, s);
    }

    ht.mark("parallel sum Btilde_F = A (A + B)^+ B");
    // parallel sum Btilde_F = sym(A (A + B)^+ B) into Sum
    std::vector<PsumDesc> ps;
    for (int f = 0; f < nf; ++f)
      ps.push_back({res[2 * f], res[2 * f + 1], Sum.p + c->tfoff[f], T.objects[T.faces[f]].n, resld[2 * f],
                    resld[2 * f + 1]});
    parallel_sum_batched(ps, c->opt.pinv_rtol, s);

    ht.mark("Btilde_F y = mu B_F y");
    // Btilde_F y = mu B_F y
    std::vector<SygvDesc> gv;
    for (int f = 0; f < nf; ++f)
      gv.push_back({Sum.p + c->tfoff[f], BF.p + c->tfoff[f], c->dWF.p + c->wfoff[f], XF.p + c->tfoff[f],
                    T.objects[T.faces[f]].n});
    eig_selected(gv, 1.0 / c->opt.theta_face, c->d_flag.p, s);
    std::vector<double> mu =
        eigenvalues_checked(c, c->dWF.p, c->dWF.n, "deluxe / face elimination / face eigenproblem");
    std::vector<QrDesc> qd;
    for (int f = 0; f < nf; ++f) {
      const int n = T.objects[T.faces[f]].n;
      int p = 0;
      for (int q = 0; q < n; ++q) {
        const double m = mu[c->wfoff[f] + q];
        if (m <= 1.0 / c->opt.theta_face) ++p;
        const double lam = m > 0 ? 1.0 / m : INFINITY;
        if (std::fabs(lam - c->opt.theta_face) <= c->opt.tie_rtol * c->opt.theta_face) ++c->n_ties;
      }
      c->pF[f] = p;
      qd.push_back({XF.p + c->tfoff[f], c->dTF.p + c->tfoff[f], n, p, n});
    }
    qr_complete_batched(qd, s);
  }

  ht.mark("primal numbering: vertices, face prima");
  // primal numbering: vertices, face primals, edge primals
  c->n_vertex = nvx;
  std::vector<int> face_pbase(nf, 0);
  int nxt = nvx;
  for (int f = 0; f < nf; ++f) {
    face_pbase[f] = nxt;
    nxt += c->pF[f];
  }
  c->pnum_face = nxt - nvx;

  // Sbar = T^T S T and W_X = D_X T_X need the face and edge transforms and
  // the deluxe blocks, not the edge ranks: queued by the edge path that
  // builds the last transforms (before its rank readback, so the device
  // rotates while the host waits and then builds the local maps), or at the
  // change of basis
  DevBuf<double> Y(c->dS.n), Sb(c->dS.n);
  std::vector<std::vector<int64_t>> wpos(nsub);
  int64_t wt = 0;
  for (int sub = 0; sub < nsub; ++sub)
    for (int k : T.sub[sub].objs) {
      wpos[sub].push_back(wt);
      wt += (int64_t)T.objects[k].n * T.objects[k].n;
    }
  DevBuf<double> WX(std::max<int64_t>(wt, 1));
  // descriptors first (pointers and sizes only: built while the device runs
  // the edge stage), launches later
  std::vector<GemmDesc<double>> rot_gc, rot_gr, rot_wg;
  std::vector<SetDesc> rot_vset;
  std::vector<LinesDesc> rot_lcol, rot_lrow;
  IntPool rot_vp;
  bool rot_ready = false, rotated = false;
  auto prepare_rotation = [&]() {
    if (rot_ready) return;
    rot_ready = true;
    // Sbar = T^T S T: Y = S T, then Sbar = T^T Y on the face and edge
    // blocks; the vertex lines, which the rotation leaves alone, are copied
    std::vector<int32_t> zero1(1, 0);
    const size_t z_off = rot_vp.add(zero1);
    std::vector<size_t> voff(nsub);
    std::vector<int> vcnt(nsub);
    for (int sub = 0; sub < nsub; ++sub) {
      std::vector<int32_t> lines;
      const SubInfo& si = T.sub[sub];
      for (size_t q = 0; q < si.objs.size(); ++q)
        if (T.objects[si.objs[q]].kind == KIND_VERTEX) lines.push_back(si.obj_off[q]);
      vcnt[sub] = (int)lines.size();
      voff[sub] = rot_vp.add(lines);
    }
    rot_vp.upload(s);
    for (int sub = 0; sub < nsub; ++sub) {
      if (vcnt[sub] == 0) continue;
      rot_lcol.push_back({c->dS.p + c->soff[sub], Y.p + c->soff[sub], rot_vp.ptr(voff[sub]), vcnt[sub], c->nB[sub], 0});
      rot_lrow.push_back({Y.p + c->soff[sub], Sb.p + c->soff[sub], rot_vp.ptr(voff[sub]), vcnt[sub], c->nB[sub], 1});
    }
    for (int sub = 0; sub < nsub; ++sub) {
      const SubInfo& si = T.sub[sub];
      const int nB = c->nB[sub];
      for (size_t q = 0; q < si.objs.size(); ++q) {
        const int k = si.objs[q];
        const Object& o = T.objects[k];
        const int off = si.obj_off[q], n = o.n;
        double* wx = WX.p + wpos[sub][q];
        if (o.kind == KIND_VERTEX) {
          rot_vset.push_back({wx, rot_vp.ptr(z_off), rot_vp.ptr(z_off), 1, 1, 1.0 / (double)o.subs.size()});
          continue;
        }
        const double* TX = o.kind == KIND_FACE ? c->dTF.p + c->tfoff[T.kind_index[k]] : c->dTE.p + c->teoff[T.kind_index[k]];
        rot_gc.push_back({c->dS.p + c->soff[sub] + off, TX, Y.p + c->soff[sub] + off, nB, n, n, nB, n, nB});
        rot_gr.push_back({TX, Y.p + c->soff[sub] + (int64_t)off * nB, Sb.p + c->soff[sub] + (int64_t)off * nB, n, nB, n, n,
                          nB, nB});
        const int mem = (int)(std::lower_bound(o.subs.begin(), o.subs.end(), sub) - o.subs.begin());
        rot_wg.push_back({c->dD.p + c->dxoff[(size_t)k * 8 + mem], TX, wx, n, n, n, n, n, n});
      }
    }
    ht.mark("rotation descriptors");
  };
  auto queue_rotation = [&]() {
    if (rotated) return;
    rotated = true;
    prepare_rotation();
    gemm_batched<double>(rot_gc, false, false, 1.0, 0.0, s);
    copy_lines_batched(rot_lcol, s);
    copy_lines_batched(rot_lrow, s);
    gemm_batched<double>(rot_gr, true, false, 1.0, 0.0, s);
    gemm_batched<double>(rot_wg, false, false, 1.0, 0.0, s);   // W_X = D_X T_X
    set_batched(rot_vset, s);                                    // vertices: 1/|n(V)|
    ht.mark("Sbar = T^T S T, W_X = D_X T_X queued");
  };

  ht.mark("edges");
  // ------------------------------------------------------------- edges
  record(c, 4);
  c->rE.assign(ned, 0);
  c->nselE.assign(ned, 0);
  c->teoff.assign(ned, 0);
  c->weoff.assign(ned, 0);
  const bool old_edges = c->opt.edge_variant == ABDDC_EDGE_OLD;
  {
    int64_t tt = 0, wt = 0;
    for (int e = 0; e < ned; ++e) {
      const Object& o = T.objects[T.edges[e]];
      c->teoff[e] = tt;
      tt += (int64_t)o.n * o.n;
      c->weoff[e] = wt;
      wt += (int64_t)(old_edges ? 1 : o.subs.size() - 1) * o.n;   // eigenvalues per edge
    }
    c->dTE.alloc(std::max<int64_t>(tt, 1));
    c->dWE.alloc(std::max<int64_t>(wt, 1));
  }
  // edges whose constraints come from the exact eigenproblem: all of them,
  // or those the network's gate sends back
  std::vector<int> elist;
  if (ned > 0 && c->opt.constraint_source == ABDDC_CONSTRAINTS_MLP) {
    c->dWE.zero(s);
    learned_edges(c, elist);
  } else {
    for (int e = 0; e < ned; ++e) elist.push_back(e);
  }
  c->n_exact_edges = (int)elist.size();
  c->n_pred_edges = ned - c->n_exact_edges;
  if (old_edges && !elist.empty()) {
    ht.mark("earlier edge eigenproblem: member Schur");
    // The earlier edge eigenproblem (eq. equ-4-8-E): Btilde_E^(nu) = Schur
    // complement of B^(nu) onto E (C = Gamma_nu minus E) in two steps, per
    // subdomain all face dofs, then per (edge, member) the other edges' dofs
    // and the vertex dofs (each pivot block a Schur complement of a principal
    // submatrix of B^(nu)_CC, positive definite as that one is); Btilde_E =
    // their parallel sum; B_E from the deluxe weights; one constraint B_E v_l
    // per selected eigenvalue, completed to an orthonormal basis.
    IntPool pool;
    std::vector<size_t> m1off(nsub);
    std::vector<int> nfc(nsub), nW(nsub), nedof(nsub);
    std::vector<std::vector<int>> epos(nsub);   // per object of the subdomain: start among its edge dofs
    for (int sub = 0; sub < nsub; ++sub) {
      const SubInfo& si = T.sub[sub];
      std::vector<int32_t> fdofs, edofs, vdofs;
      epos[sub].assign(si.objs.size(), -1);
      for (size_t q = 0; q < si.objs.size(); ++q) {
        const Object& o = T.objects[si.objs[q]];
        const int off = si.obj_off[q];
        if (o.kind == KIND_FACE) {
          for (int l = 0; l < o.n; ++l) fdofs.push_back(off + l);
        } else if (o.kind == KIND_EDGE) {
          epos[sub][q] = (int)edofs.size();
          for (int l = 0; l < o.n; ++l) edofs.push_back(off + l);
        } else {
          vdofs.push_back(off);
        }
      }
      std::vector<int32_t> mp = fdofs;
      mp.insert(mp.end(), edofs.begin(), edofs.end());
      mp.insert(mp.end(), vdofs.begin(), vdofs.end());
      m1off[sub] = pool.add(mp);
      nfc[sub] = (int)fdofs.size();
      nedof[sub] = (int)edofs.size();
      nW[sub] = c->nB[sub] - nfc[sub];
    }
    std::vector<size_t> m2off((size_t)ned * MAX_EDGE_MEMBERS);
    std::vector<int64_t> e2off((size_t)ned * MAX_EDGE_MEMBERS);
    int64_t e2tot = 0;
    int maxm = 0;
    for (int e : elist) {
      const int k = T.edges[e];
      const Object& o = T.objects[k];
      ABDDC_REQUIRE(o.subs.size() >= 2 && (int)o.subs.size() <= MAX_EDGE_MEMBERS && o.n <= 32, ABDDC_EINVAL,
                    "earlier edge eigenproblem: edges need 2..8 members and at most 32 dofs");
      maxm = std::max(maxm, (int)o.subs.size());
      for (size_t q = 0; q < o.subs.size(); ++q) {
        const int sub = o.subs[q];
        const SubInfo& si = T.sub[sub];
        const int qi = (int)(std::lower_bound(si.objs.begin(), si.objs.end(), k) - si.objs.begin());
        const int ep = epos[sub][qi];
        std::vector<int32_t> mp;   // [other edge dofs; vertex dofs; E] inside W = [edge dofs; vertex dofs]
        for (int t = 0; t < nedof[sub]; ++t)
          if (t < ep || t >= ep + o.n) mp.push_back(t);
        for (int t = nedof[sub]; t < nW[sub]; ++t) mp.push_back(t);
        for (int t = 0; t < o.n; ++t) mp.push_back(ep + t);
        m2off[(size_t)e * MAX_EDGE_MEMBERS + q] = pool.add(mp);
        e2off[(size_t)e * MAX_EDGE_MEMBERS + q] = e2tot;
        e2tot += (int64_t)nW[sub] * nW[sub];
      }
    }
    pool.upload(s);
    DevBuf<double> E1(c->dB.n), E2(std::max<int64_t>(e2tot, 1));
    {
      std::vector<GatherDesc> gd;
      std::vector<PluDesc<double>> pd;
      for (int sub = 0; sub < nsub; ++sub) {
        const int nB = c->nB[sub];
        gd.push_back({c->dB.p + c->soff[sub], E1.p + c->soff[sub], pool.ptr(m1off[sub]), pool.ptr(m1off[sub]), nB, nB,
                      nB, nB, 1.0});
        pd.push_back({E1.p + c->soff[sub], nB, nB, nB, nfc[sub]});
      }
      gather_batched(gd, s);
      partial_lu<double>(pd, c->d_flag.p, s);
    }
    // per edge: the members' Schur complements symmetrised (slot q), two
    // slots for the parallel-sum fold, the metric and the eigenvectors
    std::vector<int64_t> eoff(ned);
    int64_t etot = 0;
    for (int e : elist) {
      const Object& o = T.objects[T.edges[e]];
      eoff[e] = etot;
      etot += (int64_t)(o.subs.size() + 4) * o.n * o.n;
    }
    DevBuf<double> EB(std::max<int64_t>(etot, 1));
    auto slot = [&](int e, int q) { return EB.p + eoff[e] + (int64_t)q * T.objects[T.edges[e]].n * T.objects[T.edges[e]].n; };
    {
      std::vector<GatherDesc> gd;
      std::vector<PluDesc<double>> pd;
      std::vector<SymDesc> sy;
      for (int e : elist) {
        const Object& o = T.objects[T.edges[e]];
        for (size_t q = 0; q < o.subs.size(); ++q) {
          const int sub = o.subs[q], nB = c->nB[sub], w = nW[sub], kk = w - o.n;
          const double* Wbase = E1.p + c->soff[sub] + (int64_t)nfc[sub] * nB + nfc[sub];
          double* dst = E2.p + e2off[(size_t)e * MAX_EDGE_MEMBERS + q];
          gd.push_back({Wbase, dst, pool.ptr(m2off[(size_t)e * MAX_EDGE_MEMBERS + q]), pool.ptr(m2off[(size_t)e * MAX_EDGE_MEMBERS + q]), w, w, nB,
                        w, 1.0});
          pd.push_back({dst, w, w, w, kk});
          sy.push_back({dst + (int64_t)kk * w + kk, slot(e, (int)q), o.n, w, o.n});
        }
      }
      gather_batched(gd, s);
      partial_lu<double>(pd, c->d_flag.p, s);
      sym_batched(sy, s);
    }
    ht.mark("parallel sums, metric, eigenproblems");
    // Btilde_E = ((Bt_1 : Bt_2) : Bt_3) : Bt_4, alternating between the two fold slots
    std::vector<const double*> cur(ned, nullptr);
    for (int e : elist) cur[e] = slot(e, 0);
    for (int q = 1; q < maxm; ++q) {
      std::vector<PsumDesc> ps;
      for (int e : elist) {
        const Object& o = T.objects[T.edges[e]];
        if ((int)o.subs.size() <= q) continue;
        double* out = slot(e, (int)o.subs.size() + (q & 1));
        ps.push_back({cur[e], slot(e, q), out, o.n, o.n, o.n});
        cur[e] = out;
      }
      parallel_sum_batched(ps, c->opt.pinv_rtol, s);
    }
    std::vector<EdgeOldDesc> md;
    std::vector<SygvDesc> gv;
    for (int e : elist) {
      const int k = T.edges[e];
      const Object& o = T.objects[k];
      const int m = (int)o.subs.size();
      EdgeOldDesc d{};
      d.nE = o.n;
      d.m = m;
      for (int q = 0; q < m; ++q) {
        d.D[q] = c->dD.p + c->dxoff[(size_t)k * 8 + q];
        d.BE[q] = Sblk(c->dB.p, o.subs[q], k);
        d.ldBE[q] = c->nB[o.subs[q]];
      }
      d.out = slot(e, m + 2);
      md.push_back(d);
      gv.push_back({cur[e], slot(e, m + 2), c->dWE.p + c->weoff[e], slot(e, m + 3), o.n});
    }
    edge_old_metric_batched(md, s);
    eig_selected(gv, 1.0 / c->opt.theta_edge, c->d_flag.p, s);
    prepare_rotation();   // while the device solves the edge eigenproblems
    std::vector<double> mu = eigenvalues_checked(c, c->dWE.p, c->dWE.n, "edge elimination / edge eigenproblem");
    std::vector<QrDesc> qd;
    for (int e : elist) {
      const Object& o = T.objects[T.edges[e]];
      int ns = 0;
      for (int q = 0; q < o.n; ++q) {
        const double m = mu[c->weoff[e] + q];
        if (m <= 1.0 / c->opt.theta_edge) ++ns;
        const double lam = m > 0 ? 1.0 / m : INFINITY;
        if (std::fabs(lam - c->opt.theta_edge) <= c->opt.tie_rtol * c->opt.theta_edge) ++c->n_ties;
      }
      c->nselE[e] = ns;
      c->rE[e] = ns;
      qd.push_back({slot(e, (int)o.subs.size() + 3), c->dTE.p + c->teoff[e], o.n, ns, o.n});
    }
    qr_complete_batched(qd, s);
    queue_rotation();
  } else if (!elist.empty()) {
    // only the subdomains of the edges solved here need the per-subdomain
    // steps (all of them for the exact method; those around the edges the
    // gate sent back for learned constraints)
    std::vector<char> need(nsub, 0);
    for (int e : elist)
      for (int sub : T.objects[T.edges[e]].subs) need[sub] = 1;
    ht.mark("face-rotated Bbar^(s) = T_F^T B^(s) T_");
    // face-rotated Bbar^(s) = T_F^T B^(s) T_F on every face block
    // (Y = B T_F, then Bbar = T_F^T Y; the edge and vertex lines, which the
    // rotation leaves alone, are copied instead)
    DevBuf<double> Y(c->dB.n), Bbar(c->dB.n);
    std::vector<GemmDesc<double>> gc, gr;
    IntPool lpool;
    std::vector<size_t> loff(nsub, 0);
    std::vector<int> lcnt(nsub, 0);
    for (int sub = 0; sub < nsub; ++sub) {
      if (!need[sub]) continue;
      const SubInfo& si = T.sub[sub];
      const int nB = c->nB[sub];
      std::vector<int32_t> lines;
      for (size_t q = 0; q < si.objs.size(); ++q) {
        const int k = si.objs[q];
        const int n = T.objects[k].n, off = si.obj_off[q];
        if (T.objects[k].kind != KIND_FACE) {
          for (int l = 0; l < n; ++l) lines.push_back(off + l);
          continue;
        }
        const int f = T.kind_index[k];
        gc.push_back({c->dB.p + c->soff[sub] + off, c->dTF.p + c->tfoff[f], Y.p + c->soff[sub] + off, nB, n, n, nB, n, nB});
        gr.push_back({c->dTF.p + c->tfoff[f], Y.p + c->soff[sub] + (int64_t)off * nB, Bbar.p + c->soff[sub] + (int64_t)off * nB,
                      n, nB, n, n, nB, nB});
      }
      lcnt[sub] = (int)lines.size();
      loff[sub] = lpool.add(lines);
    }
    lpool.upload(s);
    std::vector<LinesDesc> lcol, lrow;
    for (int sub = 0; sub < nsub; ++sub) {
      if (!need[sub] || lcnt[sub] == 0) continue;
      lcol.push_back({c->dB.p + c->soff[sub], Y.p + c->soff[sub], lpool.ptr(loff[sub]), lcnt[sub], c->nB[sub], 0});
      lrow.push_back({Y.p + c->soff[sub], Bbar.p + c->soff[sub], lpool.ptr(loff[sub]), lcnt[sub], c->nB[sub], 1});
    }
    gemm_batched<double>(gc, false, false, 1.0, 0.0, s);
    copy_lines_batched(lcol, s);
    copy_lines_batched(lrow, s);
    gemm_batched<double>(gr, true, false, 1.0, 0.0, s);

    ht.mark("stage 1: per subdomain eliminate all f");
    // stage 1: per subdomain eliminate all face dual coordinates; the Schur
    // complement W^(s) lives on [edge dofs, vertex dofs, face primals]
    IntPool pool;
    std::vector<size_t> m1off(nsub);
    std::vector<int> nfd(nsub), nW(nsub), nedof(nsub);
    std::vector<std::vector<int>> edge_pos_in_W(nsub);   // per object position list index
    std::vector<std::vector<int32_t>> Hpid(nsub);          // global primal ids of H_s (W order)
    std::vector<std::vector<int32_t>> m1(nsub);
    host_parallel_for(nsub, 8, [&](int64_t sb, int64_t se) {
      std::vector<int32_t> fdual, edofs, vdofs, fprim, pid_v, pid_f;
      for (int sub = (int)sb; sub < (int)se; ++sub) {
        if (!need[sub]) continue;
        const SubInfo& si = T.sub[sub];
        fdual.clear(), edofs.clear(), vdofs.clear(), fprim.clear(), pid_v.clear(), pid_f.clear();
        edge_pos_in_W[sub].assign(si.objs.size(), -1);
        for (size_t q = 0; q < si.objs.size(); ++q) {
          const int k = si.objs[q];
          const Object& o = T.objects[k];
          const int off = si.obj_off[q];
          if (o.kind == KIND_FACE) {
            const int f = T.kind_index[k], p = c->pF[f];
            for (int l = 0; l < p; ++l) {
              fprim.push_back(off + l);
              pid_f.push_back(face_pbase[f] + l);
            }
            for (int l = p; l < o.n; ++l) fdual.push_back(off + l);
          } else if (o.kind == KIND_EDGE) {
            edge_pos_in_W[sub][q] = (int)edofs.size();
            for (int l = 0; l < o.n; ++l) edofs.push_back(off + l);
          } else {
            vdofs.push_back(off);
            pid_v.push_back(T.kind_index[k]);
          }
        }
        std::vector<int32_t>& mp = m1[sub];
        mp = fdual;
        mp.insert(mp.end(), edofs.begin(), edofs.end());
        mp.insert(mp.end(), vdofs.begin(), vdofs.end());
        mp.insert(mp.end(), fprim.begin(), fprim.end());
        nfd[sub] = (int)fdual.size();
        nedof[sub] = (int)edofs.size();
        nW[sub] = c->nB[sub] - nfd[sub];
        Hpid[sub] = pid_v;
        Hpid[sub].insert(Hpid[sub].end(), pid_f.begin(), pid_f.end());
      }
    });
    for (int sub = 0; sub < nsub; ++sub)
      if (need[sub]) m1off[sub] = pool.add(m1[sub]);
    ht.mark("stage 2 maps per (edge, member): [othe");
    // stage 2 maps per (edge, member): [other edge dofs; E dofs; H] inside W
    std::vector<size_t> m2off((size_t)ned * MAX_EDGE_MEMBERS);
    std::vector<int64_t> e2off((size_t)ned * MAX_EDGE_MEMBERS);
    std::vector<size_t> roff((size_t)ned * MAX_EDGE_MEMBERS);
    std::vector<int> nHunion(ned);
    int64_t e2tot = 0;
    const bool separate = c->opt.edge_h_mode == ABDDC_H_SEPARATE;
    for (int e : elist) {
      const Object& o = T.objects[T.edges[e]];
      for (size_t q = 0; q < o.subs.size(); ++q) {
        const int sub = o.subs[q];
        m2off[(size_t)e * MAX_EDGE_MEMBERS + q] = pool.reserve(nW[sub]);
        e2off[(size_t)e * MAX_EDGE_MEMBERS + q] = e2tot;
        e2tot += (int64_t)nW[sub] * nW[sub];
        roff[(size_t)e * MAX_EDGE_MEMBERS + q] = pool.reserve(Hpid[sub].size());
      }
    }
    host_parallel_for((int64_t)elist.size(), 16, [&](int64_t eb, int64_t ee) {
      std::vector<int32_t> uni;
      for (int64_t ei = eb; ei < ee; ++ei) {
        const int e = elist[ei];
        const int k = T.edges[e];
        const Object& o = T.objects[k];
        uni.clear();
        for (int sub : o.subs) uni.insert(uni.end(), Hpid[sub].begin(), Hpid[sub].end());
        std::sort(uni.begin(), uni.end());
        uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
        int hbase = 0;
        for (size_t q = 0; q < o.subs.size(); ++q) {
          const int sub = o.subs[q];
          const SubInfo& si = T.sub[sub];
          const int qi = (int)(std::lower_bound(si.objs.begin(), si.objs.end(), k) - si.objs.begin());
          const int epos = edge_pos_in_W[sub][qi];
          int32_t* mp = pool.h.data() + m2off[(size_t)e * MAX_EDGE_MEMBERS + q];
          int t2 = 0;
          for (int t = 0; t < nedof[sub]; ++t)
            if (t < epos || t >= epos + o.n) mp[t2++] = t;
          for (int t = 0; t < o.n; ++t) mp[t2++] = epos + t;
          for (int t = nedof[sub]; t < nW[sub]; ++t) mp[t2++] = t;
          int32_t* R = pool.h.data() + roff[(size_t)e * MAX_EDGE_MEMBERS + q];
          for (size_t h = 0; h < Hpid[sub].size(); ++h)
            R[h] = separate ? hbase + (int)h
                            : (int)(std::lower_bound(uni.begin(), uni.end(), Hpid[sub][h]) - uni.begin());
          hbase += (int)Hpid[sub].size();
        }
        nHunion[e] = separate ? hbase : (int)uni.size();
      }
    });
    pool.upload(s);
    DevBuf<double> E1(c->dB.n);
    {
      std::vector<GatherDesc> gd;
      std::vector<PluDesc<double>> pd;
      for (int sub = 0; sub < nsub; ++sub) {
        if (!need[sub]) continue;
        const int nB = c->nB[sub];
        gd.push_back({Bbar.p + c->soff[sub], E1.p + c->soff[sub], pool.ptr(m1off[sub]), pool.ptr(m1off[sub]), nB, nB,
                      nB, nB, 1.0});
        pd.push_back({E1.p + c->soff[sub], nB, nB, nB, nfd[sub]});
      }
      gather_batched(gd, s);
      partial_lu<double>(pd, c->d_flag.p, s);
    }
    DevBuf<double> E2(std::max<int64_t>(e2tot, 1));
    {
      std::vector<GatherDesc> gd;
      std::vector<PluDesc<double>> pd;
      for (int e : elist) {
        const Object& o = T.objects[T.edges[e]];
        for (size_t q = 0; q < o.subs.size(); ++q) {
          const int sub = o.subs[q], nB = c->nB[sub], w = nW[sub];
          const double* Wbase = E1.p + c->soff[sub] + (int64_t)nfd[sub] * nB + nfd[sub];
          gd.push_back({Wbase, E2.p + e2off[(size_t)e * MAX_EDGE_MEMBERS + q], pool.ptr(m2off[(size_t)e * MAX_EDGE_MEMBERS + q]),
                        pool.ptr(m2off[(size_t)e * MAX_EDGE_MEMBERS + q]), w, w, nB, w, 1.0});
          pd.push_back({E2.p + e2off[(size_t)e * MAX_EDGE_MEMBERS + q], w, w, w, nedof[sub] - o.n});
        }
      }
      gather_batched(gd, s);
      partial_lu<double>(pd, c->d_flag.p, s);
    }
    ht.mark("M_E and the coupled matrix; Schur comp");
    // M_E and the coupled matrix; Schur complement onto the jumps
    std::vector<int64_t> meoff(ned), qoff(ned), btoff(ned);
    int64_t metot = 0, qtot = 0;
    for (int e : elist) {
      const Object& o = T.objects[T.edges[e]];
      const int nw = (int)(o.subs.size() - 1) * o.n;
      const int nv = (int)o.subs.size() * o.n + nHunion[e];
      meoff[e] = metot;
      metot += (int64_t)nw * nw;
      qoff[e] = qtot;
      qtot += (int64_t)nv * nv;
    }
    DevBuf<double> ME(std::max<int64_t>(metot, 1)), Qb(std::max<int64_t>(qtot, 1)), Btt(std::max<int64_t>(metot, 1)),
        XE(std::max<int64_t>(metot, 1));
    std::vector<EdgeAsmDesc> ea;
    std::vector<SchurPinvDesc> pd;
    std::vector<SymDesc> sy;
    for (int e : elist) {
      const int k = T.edges[e];
      const Object& o = T.objects[k];
      EdgeAsmDesc d{};
      d.nE = o.n;
      d.m = (int)o.subs.size();
      d.nH = nHunion[e];
      d.nv = d.m * d.nE + d.nH;
      for (int q = 0; q < d.m; ++q) {
        const int sub = o.subs[q], w = nW[sub];
        d.D[q] = c->dD.p + c->dxoff[(size_t)k * 8 + q];
        d.BE[q] = Sblk(c->dB.p, sub, k);
        d.ldBE[q] = c->nB[sub];
        const int kk = w - (nedof[sub] - o.n);  // trailing order n_E + n_H,s
        d.Bt[q] = E2.p + e2off[(size_t)e * MAX_EDGE_MEMBERS + q] + (int64_t)(w - kk) * w + (w - kk);
        d.ldBt[q] = w;
        d.nHk[q] = (int)Hpid[sub].size();
        d.R[q] = pool.ptr(roff[(size_t)e * MAX_EDGE_MEMBERS + q]);
      }
      d.ME = ME.p + meoff[e];
      d.Q = Qb.p + qoff[e];
      ea.push_back(d);
      const int nw = (d.m - 1) * d.nE;
      pd.push_back({Qb.p + qoff[e], d.nv, d.nv - nw, d.nv});
      sy.push_back({Qb.p + qoff[e] + (int64_t)(d.nv - nw) * d.nv + (d.nv - nw), Btt.p + meoff[e], nw, d.nv, nw});
    }
    edge_assemble_batched(ea, s);
    // the eliminated block [reference edge dofs; H] can be singular (a face
    // primal coordinate dependent on the others): pseudo-inverse, as in the
    // parallel sum
    schur_pinv_batched(pd, c->opt.pinv_rtol, c->d_flag.p, s);
    sym_batched(sy, s);
    std::vector<SygvDesc> gv;
    for (int e : elist) {
      const Object& o = T.objects[T.edges[e]];
      const int nw = (int)(o.subs.size() - 1) * o.n;
      gv.push_back({Btt.p + meoff[e], ME.p + meoff[e], c->dWE.p + c->weoff[e], XE.p + meoff[e], nw});
    }
    eig_selected(gv, 1.0 / c->opt.theta_edge, c->d_flag.p, s);
    prepare_rotation();   // while the device solves the edge eigenproblems
    std::vector<double> mu = eigenvalues_checked(c, c->dWE.p, c->dWE.n, "edge elimination / edge eigenproblem");
    ht.mark("G = [g_{l,k}] (n_E x (m-1) |N_E|) and ");
    // G = [g_{l,k}] (n_E x (m-1) |N_E|) and its left singular basis
    int64_t gtot = 0;
    std::vector<int64_t> goffE(ned);
    for (int e : elist) {
      const Object& o = T.objects[T.edges[e]];
      const int m1 = (int)o.subs.size() - 1, nw = m1 * o.n;
      int ns = 0;
      for (int q = 0; q < nw; ++q) {
        const double m = mu[c->weoff[e] + q];
        if (m <= 1.0 / c->opt.theta_edge) ++ns;
        const double lam = m > 0 ? 1.0 / m : INFINITY;
        if (std::fabs(lam - c->opt.theta_edge) <= c->opt.tie_rtol * c->opt.theta_edge) ++c->n_ties;
      }
      c->nselE[e] = ns;
      goffE[e] = gtot;
      gtot += (int64_t)o.n * m1 * ns;
    }
    DevBuf<double> G(std::max<int64_t>(gtot, 1));
    DevBuf<int32_t> ranks(std::max(ned, 1));
    IntPool gp;
    std::vector<int32_t> iota(64);
    for (int q = 0; q < 64; ++q) iota[q] = q;
    const size_t iota_off = gp.add(iota);
    std::vector<size_t> rowmap_off((size_t)ned * MAX_EDGE_MEMBERS);
    for (int e : elist) {
      const Object& o = T.objects[T.edges[e]];
      for (int b = 0; b < (int)o.subs.size() - 1; ++b) {
        std::vector<int32_t> rm(o.n);
        for (int i = 0; i < o.n; ++i) rm[i] = b * o.n + i;
        rowmap_off[(size_t)e * MAX_EDGE_MEMBERS + b] = gp.add(rm);
      }
    }
    gp.upload(s);
    std::vector<GatherDesc> gd;
    std::vector<SvdDesc> sv;
    for (int e : elist) {
      const Object& o = T.objects[T.edges[e]];
      const int m1 = (int)o.subs.size() - 1, nw = m1 * o.n, ns = c->nselE[e];
      for (int b = 0; b < m1 && ns > 0; ++b)
        gd.push_back({XE.p + meoff[e], G.p + goffE[e] + (int64_t)b * ns, gp.ptr(rowmap_off[(size_t)e * MAX_EDGE_MEMBERS + b]),
                      gp.ptr(iota_off), o.n, ns, nw, m1 * ns, 1.0});
      sv.push_back({G.p + goffE[e], c->dTE.p + c->teoff[e], ranks.p + e, o.n, m1 * ns, std::max(m1 * ns, 1)});
    }
    gather_batched(gd, s);
    svd_left_batched(sv, c->opt.svd_rtol, s);
    // the ranks into pinned memory behind an event, then the rotation, then
    // the wait (for the ranks only)
    int32_t* rk = pinned_ints((size_t)std::max(ned, 1));
    ABDDC_HIP(hipMemcpyAsync(rk, ranks.p, (size_t)ned * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    hipEvent_t rev = EventPool::take();
    ABDDC_HIP(hipEventRecord(rev, s));
    queue_rotation();
    const hipError_t werr = hipEventSynchronize(rev);
    EventPool::give(c->device, rev);
    ABDDC_HIP(werr);
    for (int e : elist) c->rE[e] = rk[e];
  }
  c->pnum_edge = 0;
  std::vector<int> edge_pbase(ned, 0);
  for (int e = 0; e < ned; ++e) {
    edge_pbase[e] = nxt;
    nxt += c->rE[e];
    c->pnum_edge += c->rE[e];
  }
  c->n_primal = nxt;

  ht.mark("change of basis + local");
  // -------------------------------------------- change of basis + local
  record(c, 5);
  queue_rotation();   // unless an edge path has queued it already
  // local coordinate order per object: [primal, dual]; Pi / Delta positions
  std::vector<std::vector<int32_t>> Pi(nsub), Dl(nsub), Pid(nsub);
  host_parallel_for(nsub, 8, [&](int64_t sb, int64_t se) {
    for (int sub = (int)sb; sub < (int)se; ++sub) {
      const SubInfo& si = T.sub[sub];
      Dl[sub].reserve(si.nB);
      for (size_t q = 0; q < si.objs.size(); ++q) {
        const int k = si.objs[q];
        const Object& o = T.objects[k];
        const int off = si.obj_off[q];
        int p = 0, base = 0;
        if (o.kind == KIND_VERTEX) {
          p = 1;
          base = T.kind_index[k];
        } else if (o.kind == KIND_FACE) {
          p = c->pF[T.kind_index[k]];
          base = face_pbase[T.kind_index[k]];
        } else {
          p = c->rE[T.kind_index[k]];
          base = edge_pbase[T.kind_index[k]];
        }
        for (int l = 0; l < p; ++l) {
          Pi[sub].push_back(off + l);
          Pid[sub].push_back(base + l);
        }
        for (int l = p; l < o.n; ++l) Dl[sub].push_back(off + l);
      }
    }
  });
  c->nPi.assign(nsub, 0);
  c->moff.assign(nsub, 0);
  c->uoff.assign(nsub, 0);
  c->ooff.assign(nsub, 0);
  c->poff.assign(nsub, 0);
  int64_t mt = 0, ut = 0, ot = 0, pt = 0, at = 0;
  std::vector<int64_t> aoff2(nsub);
  for (int sub = 0; sub < nsub; ++sub) {
    const int nB = c->nB[sub], nP = (int)Pi[sub].size(), nD = (int)Dl[sub].size();
    c->nPi[sub] = nP;
    c->moff[sub] = mt;
    mt += (int64_t)(nB + nP) * nB;
    c->uoff[sub] = ut;
    ut += (int64_t)nB * nP;
    c->ooff[sub] = ot;
    ot += nB + nP;
    c->poff[sub] = pt;
    pt += nP;
    aoff2[sub] = at;
    at += (int64_t)(2 * nB) * (2 * nB);
  }
  // the augmented systems and the apply operators in the factorisation's
  // precision: FP64, or FP32 throughout for the mixed form (no copies)
  const bool mixed = c->opt.precision == ABDDC_PREC_MIXED;
  DevBuf<double> Aug;
  DevBuf<float> Aug32;
  if (mixed) {
    Aug32.alloc(std::max<int64_t>(at, 1));
    c->dM32.alloc(std::max<int64_t>(mt, 1));
    c->dU32.alloc(std::max<int64_t>(ut, 1));
    c->dM.release();
    c->dU.release();
  } else {
    Aug.alloc(std::max<int64_t>(at, 1));
    c->dM.alloc(std::max<int64_t>(mt, 1));
    c->dU.alloc(std::max<int64_t>(ut, 1));
    c->dM32.release();
    c->dU32.release();
  }
  {
    ht.mark("augmented [[Sbar, W^T], [-W, 0]]");
    // Local constrained solve with the averaging folded in (the order of
    // rows and columns is [Delta; Pi] of rotated coordinates, then the nB
    // original coordinates):
    //   Aug = [[S_DD, S_DPi, W_D^T], [S_PiD, S_PiPi, W_Pi^T], [-W_D, -W_Pi, 0]].
    // Eliminating the Delta pivots leaves [[S_c, V], [-U, L]] with
    // X = S_DD^{-1}, S_c = S_PiPi - S_PiD X S_DPi (the local coarse matrix),
    // L = W_D X W_D^T, V = W_Pi^T - S_PiD X W_D^T, U = W_Pi - W_D X S_DPi:
    // M = [L; V] and U are read off the trailing block.
    IntPool pool;
    std::vector<size_t> am(nsub), sl(nsub), oo(nsub), on(nsub), ow(nsub), pidx(nsub);
    ABDDC_REQUIRE(wt < ((int64_t)1 << 31), ABDDC_EINVAL, "interface blocks too large");
    for (int sub = 0; sub < nsub; ++sub) {
      const size_t nB = c->nB[sub], no = T.sub[sub].objs.size();
      am[sub] = pool.reserve(nB);
      sl[sub] = pool.reserve(nB);
      oo[sub] = pool.reserve(no);
      on[sub] = pool.reserve(no);
      ow[sub] = pool.reserve(no);
      pidx[sub] = pool.reserve(Pid[sub].size());
    }
    host_parallel_for(nsub, 8, [&](int64_t sb, int64_t se) {
      for (int sub = (int)sb; sub < (int)se; ++sub) {
        const SubInfo& si = T.sub[sub];
        const int nD = (int)Dl[sub].size();
        int32_t* h = pool.h.data();
        int32_t* mp = h + am[sub];
        std::copy(Dl[sub].begin(), Dl[sub].end(), mp);
        std::copy(Pi[sub].begin(), Pi[sub].end(), mp + nD);
        for (size_t q = 0; q < si.objs.size(); ++q) {
          const int n = T.objects[si.objs[q]].n, off = si.obj_off[q];
          std::fill(h + sl[sub] + off, h + sl[sub] + off + n, (int32_t)q);
          h[oo[sub] + q] = off;
          h[on[sub] + q] = n;
          h[ow[sub] + q] = (int32_t)wpos[sub][q];
        }
        std::copy(Pid[sub].begin(), Pid[sub].end(), h + pidx[sub]);
      }
    });
    pool.upload(s);
    std::vector<AugDesc> ad;
    std::vector<PluDesc<double>> pd;
    std::vector<PluDesc<float>> pf;
    std::vector<AugOutDesc> od;
    for (int sub = 0; sub < nsub; ++sub) {
      const int nB = c->nB[sub], nD = (int)Dl[sub].size();
      void* a = mixed ? (void*)(Aug32.p + aoff2[sub]) : (void*)(Aug.p + aoff2[sub]);
      ad.push_back({Sb.p + c->soff[sub], a, pool.ptr(am[sub]), pool.ptr(sl[sub]), pool.ptr(oo[sub]),
                    pool.ptr(on[sub]), pool.ptr(ow[sub]), WX.p, nB});
      if (mixed) {
        pf.push_back({Aug32.p + aoff2[sub], 2 * nB, 2 * nB, 2 * nB, nD});
        od.push_back({a, c->dM32.p + c->moff[sub], c->dU32.p + c->uoff[sub], nB, nD});
      } else {
        pd.push_back({Aug.p + aoff2[sub], 2 * nB, 2 * nB, 2 * nB, nD});
        od.push_back({a, c->dM.p + c->moff[sub], c->dU.p + c->uoff[sub], nB, nD});
      }
    }
    aug_build_batched(ad, mixed, s);
    // the mixed form factors in FP32 on MFMA; the preconditioner it defines
    // is applied inside FP64 GMRES, which absorbs its rounding
    if (mixed) partial_lu<float>(pf, c->d_flag.p, s);
    else partial_lu<double>(pd, c->d_flag.p, s);

    ht.mark("M = [L; V], U from the trailing block");
    aug_extract_batched(od, mixed, s);

    ht.mark("apply metadata (device)");
    // ------------------------------------------- apply metadata (device)
    // (sizes and maps only: built while the device runs the local
    // factorisations, before the coarse factorisation is queued)
    record(c, 7);
    const int np = c->n_primal;
    std::vector<int32_t> pid_all, ptr_p, idx_p, kp, vp;
    for (int sub = 0; sub < nsub; ++sub) {
      const int nB = c->nB[sub];
      pid_all.insert(pid_all.end(), Pid[sub].begin(), Pid[sub].end());
      for (size_t l = 0; l < Pid[sub].size(); ++l) {
        kp.push_back(Pid[sub][l]);
        vp.push_back((int32_t)(c->ooff[sub] + nB + l));
      }
    }
    csr_group(np, kp, vp, ptr_p, idx_p);
    // interface dof -> its output rows, one per sharing subdomain in
    // subdomain order: dof gstart + q of object k sits at row
    // ooff[s] + (offset of k in Gamma_s) + q of every s in n(k); objects
    // are in interface order, so each object's entries form one range
    std::vector<int64_t> opos(T.objects.size() + 1, 0);
    for (size_t k = 0; k < T.objects.size(); ++k)
      opos[k + 1] = opos[k] + (int64_t)T.objects[k].n * (int64_t)T.objects[k].subs.size();
    std::vector<int32_t> ptr_a((size_t)T.n_gamma + 1), idx_a((size_t)opos.back());
    host_parallel_for((int64_t)T.objects.size(), 64, [&](int64_t kb, int64_t ke) {
      std::vector<int32_t> base;
      for (int64_t k = kb; k < ke; ++k) {
        const Object& o = T.objects[k];
        const int m = (int)o.subs.size();
        base.resize(m);
        for (int j = 0; j < m; ++j)
          base[j] = (int32_t)(c->ooff[o.subs[j]] + T.sub[o.subs[j]].local_pos((int)k));
        for (int q = 0; q < o.n; ++q) {
          const int64_t at = opos[k] + (int64_t)q * m;
          ptr_a[o.gstart + q] = (int32_t)at;
          for (int j = 0; j < m; ++j) idx_a[at + j] = base[j] + q;
        }
      }
    });
    ptr_a[T.n_gamma] = (int32_t)opos.back();
    ht.mark("metadata: owner lists");
    c->d_pid = to_device(pid_all, s);
    c->d_pown_ptr = to_device(ptr_p, s);
    c->d_pown_idx = to_device(idx_p, s);
    c->d_aown_ptr = to_device(ptr_a, s);
    c->d_aown_idx = to_device(idx_a, s);
    std::vector<GemvMat> mM, mU, mC;
    std::vector<char> activeU;
    for (int sub = 0; sub < nsub; ++sub) {
      const int nB = c->nB[sub], nP = c->nPi[sub];
      mM.push_back({c->moff[sub], c->goff[sub], c->ooff[sub], nB + nP, nB, nB, 0});
      mU.push_back({c->uoff[sub], c->poff[sub], c->ooff[sub], nB, nP, std::max(nP, 1), 0});
      activeU.push_back(nP > 0);
    }
    mC.push_back({0, 0, 0, np, np, std::max(np, 1), 0});
    auto gbytes = [](const std::vector<GemvMat>& v, bool gathered, double esize) {
      double b = 0.0;  // matrix + gathered input (value and index) + output
      for (const GemvMat& m : v) b += (double)m.nrows * m.ncols * esize + m.ncols * (gathered ? 12.0 : 8.0) + m.nrows * 8.0;
      return b;
    };
    ht.mark("metadata: uploads, fp32 copies");
    gemv_build(c->opM, mM, nullptr, gbytes(mM, true, mixed ? 4.0 : 8.0), s);
    gemv_build(c->opU, mU, &activeU, gbytes(mU, true, mixed ? 4.0 : 8.0), s);
    gemv_build(c->opC, mC, nullptr, gbytes(mC, false, 8.0), s);
    c->d_out.alloc(std::max<int64_t>(ot, 1));
    c->d_bpi.alloc(std::max(np, 1));
    c->d_xpi.alloc(std::max(np, 1));
    ht.mark("metadata: GEMV operators, buffers");
    ht.mark("coarse");
    // ----------------------------------------------------------- coarse
    record(c, 6);
    DevBuf<double> Aug2((size_t)std::max(1, 4 * np * np));
    DevBuf<double> SPi((size_t)std::max(1, np * np));
    SPi.zero(s);
    // colour the subdomains so that equal colours share no primal unknown:
    // by index parity on box partitions, greedily (first free colour in
    // subdomain order) on general ones
    std::vector<int> colour(nsub, 0);
    int ncolour = 8;
    if (T.general) {
      std::vector<std::vector<int>> owners(np);
      for (int sub = 0; sub < nsub; ++sub)
        for (int32_t q : Pid[sub]) owners[q].push_back(sub);
      ncolour = 0;
      std::vector<int> mark;
      for (int sub = 0; sub < nsub; ++sub) {
        mark.assign(ncolour + 1, 0);
        for (int32_t q : Pid[sub])
          for (int o : owners[q])
            if (o < sub) mark[colour[o]] = 1;
        int cl = 0;
        while (mark[cl]) ++cl;
        colour[sub] = cl;
        ncolour = std::max(ncolour, cl + 1);
      }
    } else {
      for (int sub = 0; sub < nsub; ++sub) {
        const int sx = sub % T.nsub[0], sy = (sub / T.nsub[0]) % T.nsub[1], sz = sub / (T.nsub[0] * T.nsub[1]);
        colour[sub] = (sx & 1) | ((sy & 1) << 1) | ((sz & 1) << 2);
      }
    }
    for (int color = 0; color < ncolour; ++color) {
      std::vector<CoarseAddDesc> cd;
      for (int sub = 0; sub < nsub; ++sub) {
        if (colour[sub] != color) continue;
        const int nP = (int)Pi[sub].size(), nD = (int)Dl[sub].size(), na = 2 * c->nB[sub];
        if (nP == 0) continue;
        const int64_t o = aoff2[sub] + (int64_t)nD * na + nD;   // the Pi x Pi block
        cd.push_back({mixed ? nullptr : Aug.p + o, pool.ptr(pidx[sub]), nP, na, mixed ? Aug32.p + o : nullptr});
      }
      coarse_add_batched(cd, SPi.p, np, s);
    }
    c->dSPinv.alloc((size_t)std::max(1, np * np));
    if (np > 0) {
      IntPool cp;
      std::vector<int32_t> mp(2 * np), r1(np), c1(np), r2(np), c2(np);
      for (int q = 0; q < 2 * np; ++q) mp[q] = q < np ? q : -1;
      for (int q = 0; q < np; ++q) {
        r1[q] = q;
        c1[q] = np + q;
        r2[q] = np + q;
        c2[q] = q;
      }
      const size_t o1 = cp.add(mp), o2 = cp.add(r1), o3 = cp.add(c1), o4 = cp.add(r2), o5 = cp.add(c2);
      cp.upload(s);
      gather_batched({{SPi.p, Aug2.p, cp.ptr(o1), cp.ptr(o1), 2 * np, 2 * np, np, 2 * np, 1.0}}, s);
      set_batched({{Aug2.p, cp.ptr(o2), cp.ptr(o3), np, 2 * np, 1.0}, {Aug2.p, cp.ptr(o4), cp.ptr(o5), np, 2 * np, -1.0}},
                  s);
      partial_lu<double>({{Aug2.p, 2 * np, 2 * np, 2 * np, np}}, c->d_flag.p, s);
      gather_batched({{Aug2.p + (int64_t)np * 2 * np + np, c->dSPinv.p, nullptr, nullptr, np, np, 2 * np, np, 1.0}}, s);
    }

    // variants of the three apply GEMVs (cached per architecture and size)
    ABDDC_HIP(hipMemsetAsync(c->d_bpi.p, 0, std::max(np, 1) * sizeof(double), s));
    ABDDC_HIP(hipMemsetAsync(c->d_xpi.p, 0, std::max(np, 1) * sizeof(double), s));
    if (mixed) {
      gemv_tune<float>(c->opM, "bddc_LV", c->device, c->dM32.p, c->d_ghat.p, c->d_gam.p, c->d_out.p, s);
      gemv_tune<float>(c->opU, "bddc_U", c->device, c->dU32.p, c->d_xpi.p, c->d_pid.p, c->d_out.p, s);
    } else {
      gemv_tune<double>(c->opM, "bddc_LV", c->device, c->dM.p, c->d_ghat.p, c->d_gam.p, c->d_out.p, s);
      gemv_tune<double>(c->opU, "bddc_U", c->device, c->dU.p, c->d_xpi.p, c->d_pid.p, c->d_out.p, s);
    }
    gemv_tune<double>(c->opC, "coarse", c->device, c->dSPinv.p, c->d_bpi.p, nullptr, c->d_xpi.p, s);
    ht.mark("metadata uploaded");
  }
  record(c, 8);
  // the stage buffers go back to the cache here, in stream order, before
  // the caller waits for the flag (setup_final_check)
}

void setup_final_check(abddc_ctx* c) {
  HostTrace ht;
  require_flag_clean(c, "local constrained / coarse factorisation");
  ht.mark("final flag check (sync)");
}

}  // namespace abddc
