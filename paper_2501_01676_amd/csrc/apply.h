// Per-iteration kernel launchers (GEMV, gather-sum, GMRES vector ops).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace abddc {

constexpr int GEMV_ROWS_PER_WAVE = 4;
constexpr int GEMV_ROWS_PER_BLOCK = 4 * GEMV_ROWS_PER_WAVE;
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

template <class TM>
void launch_gemv(const GemvBlock* blocks, int nblk, const GemvMat* mats, int max_ncols, const TM* M,
                 const double* x, const int32_t* xidx, double* y, bool accumulate, hipStream_t s,
                 double bytes = 0.0);
void launch_gather_sum(const int32_t* ptr, const int32_t* idx, const double* src, double* dst, int64_t n,
                       hipStream_t s);
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
// Z[:, st->j] = src
void launch_store_col(const double* src, double* Z, int64_t ldz, const GmresState* st, int64_t n, hipStream_t s);
// V[:, st->j] = cur = src * st->inv_hn
void launch_scale_to_col(const double* src, const GmresState* st, double* V, int64_t ldv, double* cur, int64_t n,
                         hipStream_t s);
// Hessenberg column st->j (as launch_arnoldi_finish), then st->j += 1
void launch_arnoldi_finish_dev(GmresState* st, const double* h1, const double* h2, const double* nrm2,
                               hipStream_t s);
void launch_arnoldi_finish(GmresState* st, int j, const double* h1, const double* h2, const double* nrm2,
                           hipStream_t s);
void launch_gmres_trisolve(GmresState* st, int m, hipStream_t s);
void launch_gmres_start(GmresState* st, const double* nrm2, hipStream_t s);
void launch_scale_copy(const double* src, const double* factor, double* dst, int64_t n, hipStream_t s);
void launch_sub(const double* a, const double* b, double* out, int64_t n, hipStream_t s);

}  // namespace abddc
