// Assembly / recovery kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace abddc {

struct ElemParams {
  int64_t n_elem;
  int ne[3], nn[3];
  double h[3];
  double origin[3];
  double b0[3], b1[9];
  double c, tau, f_const;
  int element;                 // ABDDC_ELEM_Q1 / ABDDC_ELEM_P1
};

// Optional nodal fields of the element kernels (device pointers or null).
struct ElemFields {
  const double* f_nodal;       // source per grid node
  const double* a_nodal;       // velocity per grid node (3), P1 only
  const double* u_dirichlet;   // Dirichlet data per grid node (boundary read)
};

// Per-subdomain assembly metadata (device array, one entry per subdomain).
struct SubAsm {
  int64_t aoff;    // [A | f] matrix offset (doubles)
  int64_t soff;    // S / B offset
  int64_t goff;    // interface vector offset
  int64_t ioff;    // interior vector offset
  int64_t loff;    // first local row in the concatenated row list
  int32_t lmoff;   // box-local node map offset
  int32_t nloc, nI, ld;
  int32_t ebox[6]; // element ranges x0 x1 y0 y1 z0 z1 (node box is inclusive)
};

void launch_check_positive(const double* v, int64_t n, int* flag, hipStream_t s);
void launch_elem(const ElemParams& P, const double* nu, const ElemFields& F, double* Ae, double* Fe,
                 hipStream_t s);
void launch_scatter(const SubAsm* subs, const int32_t* rowsub, const int32_t* lnode, const int32_t* lmap,
                    int64_t nrows, const int nn[3], const int ne[3], const double* Ae, const double* Fe,
                    const int32_t* part, double* A, hipStream_t s);
void launch_extract(const SubAsm* subs, int nsub, int max_nB, const double* A, double* S, double* B, double* g,
                    hipStream_t s);
// interior recovery; max_nloc = max over subdomains of n_I + n_B (LDS size)
void launch_recover(const SubAsm* subs, int nsub, int max_nloc, const double* A, const int32_t* gam,
                    const double* uhat, const int32_t* int_dof, const int32_t* iface_dof, int64_t n_gamma, double* u,
                    hipStream_t s);

}  // namespace abddc
