// Per-iteration kernel launchers (GEMV, gather-sum, GMRES vector ops).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "internal.h"

namespace abddc {

// GEMV variants: rows per wave (a workgroup is 4 waves); the last one, for
// operators of at most 64 columns, gives every lane a row of its own
constexpr int GEMV_NVAR = 4;
constexpr int GEMV_ROWS[GEMV_NVAR] = {2, 4, 8, 64};
constexpr int GEMV_NARROW = 3;
constexpr int DOT_BLOCKS = 256;
constexpr int DOT_STRIDE = 64;   // partial-sum stride (>= restart + 1 vectors)
constexpr int GMRES_MAXR = 63;   // maximum restart length

struct GemvMat {
  int64_t moff;   // matrix offset (elements)
  int64_t xoff;   // input offset into x or into the gather index
  int64_t yoff;   // output offset
  int32_t nrows, ncols, ld, pad;
};

struct GemvBlock {
  int32_t mat;
  int32_t row0;
};

// Device-resident GMRES scalars (Hessenberg, rotations, rotated rhs).
struct GmresState {
  double H[(GMRES_MAXR + 1) * GMRES_MAXR];
  double cs[GMRES_MAXR], sn[GMRES_MAXR];
  double g[GMRES_MAXR + 1];
  double y[GMRES_MAXR];
  double beta, hn, inv_hn, res;
  int32_t j;   // Arnoldi step inside the cycle (kernels of one step read it)
  int32_t pad;
};

// A batched GEMV operator: its matrices, the workgroup lists of every
// variant, the variant in use and the algorithmic bytes of one launch.
struct GemvOp {
  DevBuf<GemvMat> mats;
  DevBuf<GemvBlock> blocks[GEMV_NVAR];
  int nblk[GEMV_NVAR] = {0, 0, 0, 0};
  int maxc = 1;
  int var = 1;
  double bytes = 0.0;
  int64_t rows = 0;
};

// Builds the operator; only matrices with active[i] != 0 get workgroups
// (all when active is null).
void gemv_build(GemvOp& op, const std::vector<GemvMat>& mats, const std::vector<char>* active, double bytes,
                hipStream_t s);
// y (+)= M x (x gathered through xidx when xidx is non-null)
template <class TM>
void gemv_run(const GemvOp& op, const TM* M, const double* x, const int32_t* xidx, double* y, bool accumulate,
              hipStream_t s);
// Picks the variant: ABDDC_GEMV_VARIANT (0..3) when set, else the cached
// choice for (architecture, operator name, element type, size buckets),
// else the fastest of timed launches on the operator's own data (x, y as in
// gemv_run; y is overwritten), recorded in the autotuner cache.
template <class TM>
void gemv_tune(GemvOp& op, const char* name, int device, const TM* M, const double* x, const int32_t* xidx,
               double* y, hipStream_t s);
void launch_gather_sum(const int32_t* ptr, const int32_t* idx, const double* src, double* dst, int64_t n,
                       hipStream_t s);
// the same, and a copy into column st->j of Z (leading dimension ldz)
void launch_gather_sum_col(const int32_t* ptr, const int32_t* idx, const double* src, double* dst, double* Z,
                           int64_t ldz, const GmresState* st, int64_t n, hipStream_t s);
void launch_dots(const double* V, int64_t ldv, int nv, const double* w, int64_t n, double* partial, double* out,
                 hipStream_t s);
void launch_axpy_multi(const double* V, int64_t ldv, int nv, const double* coef, double sign, double* w, int64_t n,
                       hipStream_t s);
// The same with the vector count j + 1 read from st->j on the device (the
// kernels of one Arnoldi step are then independent of j, so the step can be
// captured once in a HIP graph and replayed).  max_nv bounds j + 1.
void launch_dots_dev(const double* V, int64_t ldv, const GmresState* st, int max_nv, const double* w, int64_t n,
                     double* partial, double* out, hipStream_t s);
void launch_axpy_multi_dev(const double* V, int64_t ldv, const GmresState* st, const double* coef, double sign,
                           double* w, int64_t n, hipStream_t s);
// w -= V[:, 0..st->j] coef, then out = V[:, 0..st->j]^T w (norm: out[0] =
// w . w), the update fused into the partial products
void launch_axpy_dots_dev(const double* V, int64_t ldv, const GmresState* st, int max_nv, const double* coef,
                          double* w, int64_t n, bool norm, double* partial, double* out, hipStream_t s);
// V[:, st->j] = cur = src * st->inv_hn
void launch_scale_to_col(const double* src, const GmresState* st, double* V, int64_t ldv, double* cur, int64_t n,
                         hipStream_t s);
// Hessenberg column st->j (as launch_arnoldi_finish), then st->j += 1;
// with host_out (device view of pinned coherent host memory, 8 doubles),
// beta, hn, inv_hn, res of step j also go to host_out[4 (j % 2) ..]
void launch_arnoldi_finish_dev(GmresState* st, const double* h1, const double* h2, const double* nrm2,
                               double* host_out, hipStream_t s);
void launch_arnoldi_finish(GmresState* st, int j, const double* h1, const double* h2, const double* nrm2,
                           hipStream_t s);
void launch_gmres_trisolve(GmresState* st, int m, hipStream_t s);
// restart: g = (||r||, 0, ..), j = 0; beta, hn, inv_hn, res to host_out[0..4) when given
void launch_gmres_start(GmresState* st, const double* nrm2, double* host_out, hipStream_t s);
void launch_scale_copy(const double* src, const double* factor, double* dst, int64_t n, hipStream_t s);
void launch_sub(const double* a, const double* b, double* out, int64_t n, hipStream_t s);

}  // namespace abddc
