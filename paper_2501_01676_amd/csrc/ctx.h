// The library context: problem, topology, device data of every stage.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <vector>

#include "apply.h"
#include "assemble.h"
#include "internal.h"
#include "kstats.h"
#include "mlp.h"
#include "topology.h"

namespace abddc {

// Index plan of the staged face eliminations (topology only): built by
// assemble while the device works, used by the coarse-space setup.
struct FaceElimPlan {
  struct Group {
    int sub, nfaces, cpos, ng;   // subdomain, faces of one normal axis, their position and size in C
    int64_t o2;                  // offset of the group's matrix
    int k2;                      // order eliminated in step (2)
    size_t m2;                   // pool offset of the step (2) map
  };
  bool ready = false;
  DevBuf<int32_t> d_pool;               // concatenated index maps
  std::vector<size_t> m1off;            // per subdomain: step (1) map
  std::vector<int> nR, nC;              // per subdomain: eliminated / kept in step (1)
  std::vector<Group> groups;
  std::vector<int64_t> res3;            // per (face, side): step (3) matrix offset, -1 when none
  std::vector<int> k3of, ng3, grp_of;   // per (face, side)
  std::vector<size_t> m3off;
  int64_t w2tot = 0, w3tot = 0;
};

}  // namespace abddc

struct abddc_ctx {
  // ---------------------------------------------------------- problem
  int device = 0;
  hipStream_t stream = nullptr;
  abddc::DevAlloc dalloc;   // caller's device allocation hooks (null: the library's cache)
  abddc::Topology topo;
  double length[3], beta0[3], beta1[9], c = 0, f_const = 0, tau = 0;
  bool have_fnodal = false;
  int element = 0;                  // ABDDC_ELEM_Q1 or ABDDC_ELEM_P1
  int state = 0;  // 1 assembled, 2 set up
  abddc_options opt{};

  // --------------------------------------------------- per-subdomain
  std::vector<int> nI, nB, nloc;           // interior, interface, total local dofs
  std::vector<int64_t> aoff;               // [A | f] matrices, ld = nloc + 1
  std::vector<int64_t> soff;               // S, B matrices (nB x nB)
  std::vector<int64_t> goff;               // vectors of length nB
  abddc::DevBuf<double> dA, dS, dB, dg;
  abddc::DevBuf<int32_t> d_gam;            // concatenated Gamma_i -> interface index
  abddc::DevBuf<int32_t> d_own_ptr, d_own_idx;   // interface dof -> positions in goff space
  abddc::DevBuf<double> d_ghat;
  abddc::DevBuf<double> d_nu, d_fnodal;
  abddc::DevBuf<int32_t> d_iface_dof, d_int_dof;  // recovery scatter maps (goff / interior space)
  std::vector<int64_t> ioff;               // interior offsets (concatenated interior dofs)

  // ---------------------------------------------------- coarse space
  std::vector<int> pF;                     // primal count per face (kind index)
  std::vector<int> rE;                     // primal count per edge (kind index)
  std::vector<int> nselE;                  // selected eigenvectors per edge
  std::vector<int64_t> dxoff;              // deluxe block of (object, member) [8 per object]
  abddc::DevBuf<double> dD;
  std::vector<int64_t> tfoff, teoff;       // face / edge bases
  abddc::DevBuf<double> dTF, dTE;
  std::vector<int64_t> wfoff, weoff;       // eigenvalues (mu) of face / edge GEPs
  abddc::DevBuf<double> dWF, dWE;
  abddc::FaceElimPlan fplan;
  int n_primal = 0, n_vertex = 0, pnum_face = 0, pnum_edge = 0, n_ties = 0;

  // ----------------------------------------------------- apply operators
  std::vector<int> nPi;                    // primal unknowns per subdomain
  std::vector<int64_t> moff;               // [L; V] (nB + nPi) x nB
  std::vector<int64_t> uoff;               // U  nB x nPi
  std::vector<int64_t> ooff;               // output vectors of length nB + nPi
  std::vector<int64_t> poff;               // concatenated primal ids per subdomain
  abddc::DevBuf<double> dM, dU, dSPinv;
  abddc::DevBuf<float> dM32, dU32;
  abddc::DevBuf<int32_t> d_pid;            // concatenated Pi_i -> global primal id
  abddc::DevBuf<int32_t> d_sown_ptr, d_sown_idx;   // interface dof -> positions in goff space
  abddc::DevBuf<int32_t> d_pown_ptr, d_pown_idx;   // primal id -> positions in ooff space
  abddc::DevBuf<int32_t> d_aown_ptr, d_aown_idx;   // interface dof -> positions in ooff space
  abddc::GemvOp opM, opU, opC, opS;                // [L; V], U, coarse inverse, Schur
  abddc::KStats kstats;
  abddc::DevBuf<double> d_out, d_wS, d_bpi, d_xpi;  // apply / Schur work vectors
  abddc::DevBuf<abddc::SubAsm> d_subs;

  // ------------------------------------------------------------- GMRES
  abddc::DevBuf<double> d_V, d_Z, d_w, d_r, d_x, d_h1, d_h2, d_nrm, d_partial;
  abddc::DevBuf<abddc::GmresState> d_gst;
  double* h_step = nullptr;    // pinned, device-coherent: scalars of two Arnoldi steps in flight and of the restart
  double* dh_step = nullptr;   // the same memory as the device sees it
  hipEvent_t ev_step[2] = {nullptr, nullptr};
  int gm_restart = 0;
  abddc::DevBuf<double> d_vcur, d_zcur;             // current Arnoldi vector and its preconditioned image
  hipStream_t cap_stream = nullptr;                 // private stream for graph capture
  hipGraph_t step_graph = nullptr;                  // one captured Arnoldi step
  hipGraphExec_t step_exec = nullptr;
  int step_restart = 0;
  bool graph_failed = false;

  // ------------------------------------------------- learned constraints
  std::vector<abddc::EdgeGeom> egeom;               // per edge (kind order)
  abddc::DevBuf<abddc::EdgeGeom> d_egeom;
  int n_pred_edges = 0, n_exact_edges = 0;

  // ------------------------------------------------------------- misc
  abddc::DevBuf<int> d_flag;
  std::array<double, 16> phase{};
  hipEvent_t ev[20] = {};
  bool events = false;
};
