// Batched dense kernels for gfx950: MFMA tile GEMM (FP64 16x16x4, FP32
// 16x16x4), blocked partial LU without pivoting that leaves the Schur
// complement in the trailing block, and matrix gathers.
//
// Every dense elimination of the method is a Schur complement of a row-
// major matrix onto its trailing rows/columns (local Schur complements and
// right-hand sides, Section 3; face and edge eliminations onto interface
// objects; deluxe solves and explicit inverses written as Schur complements
// of [[A, B], [-I, 0]]).  Pivots come from blocks whose symmetric part is
// positive definite (b(.,.) is SPD and z(.,.) skew, Section 2), so every
// leading principal minor is nonzero and no pivoting is needed.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "arena.h"
#include "buffer.h"
#include "htrace.h"
#include "internal.h"
#include "kstats.h"

namespace abddc {

namespace {

constexpr int TILE = 64;   // C tile is TILE x TILE, 4 waves of 32x32
constexpr int KC = 32;     // K chunk staged through LDS
constexpr int NB = 64;     // partial LU panel width
constexpr int LDS_PAD = TILE + 1;

// Tiled batched launches run on a 1-D grid renumbered for the 8 XCDs.  The
// hardware hands workgroup w to XCD w % 8, and each XCD has its own L2, so
// with the plain numbering neighbouring tiles of one matrix -- which read the
// same row strip of A and column strip of B -- land on different XCDs and
// every tile fetches its operands from HBM.  Matrix z instead goes to XCD
// z % 8 with its tiles in order (for batches of at least 8 matrices;
// otherwise each XCD takes a contiguous eighth of the (matrix, tile) range),
// so the operand strips are read from HBM about once per XCD.  The grid is
// ragged: every matrix gets exactly its own tiles (a host-built schedule of
// per-XCD prefix sums of the tile counts), so a batch of uneven problems
// launches no workgroup that only exits.
constexpr int N_XCD = 8;

// sched: for nb >= 8, N_XCD rows of J + 1 prefix sums (J = ceil(nb / 8)),
// row x over the matrices x, x + 8, ...; for nb < 8, nb + 1 prefix sums.
// Sets the matrix z and its tile u of this workgroup.
__device__ inline bool ragged_tile(const int32_t* __restrict__ sched, int nb, int& z, int& u) {
  const int w = blockIdx.x;
  if (nb >= N_XCD) {
    const int x = w % N_XCD, local = w / N_XCD, J = (nb + N_XCD - 1) / N_XCD;
    const int nj = (nb - x + N_XCD - 1) / N_XCD;   // matrices on this XCD
    const int32_t* P = sched + x * (J + 1);
    if (nj <= 0 || local >= P[nj]) return false;
    int lo = 0, hi = nj - 1;   // the last matrix that starts at or before local
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (P[mid] <= local) lo = mid;
      else hi = mid - 1;
    }
    z = x + N_XCD * lo;
    u = local - P[lo];
    return true;
  }
  const int t = (w % N_XCD) * (int)(gridDim.x / N_XCD) + w / N_XCD;
  if (t >= sched[nb]) return false;
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sched[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  z = lo;
  u = t - sched[lo];
  return true;
}

// The schedule and grid of a ragged launch with count[z] tiles of matrix z
// (grid 0: nothing to launch).
struct RaggedGrid {
  const int32_t* sched = nullptr;
  unsigned grid = 0;
};
inline RaggedGrid ragged_grid(const std::vector<int>& count, Arena& ar) {
  const int nb = (int)count.size();
  std::vector<int32_t> sched;
  int64_t g = 0;
  if (nb >= N_XCD) {
    const int J = (nb + N_XCD - 1) / N_XCD;
    sched.assign((size_t)N_XCD * (J + 1), 0);
    int64_t mx = 0;
    for (int x = 0; x < N_XCD; ++x) {
      int32_t* P = sched.data() + (size_t)x * (J + 1);
      int j = 0;
      for (int z = x; z < nb; z += N_XCD, ++j) P[j + 1] = P[j] + count[z];
      for (int q = j + 1; q <= J; ++q) P[q] = P[j];
      mx = std::max<int64_t>(mx, P[j]);
    }
    g = (int64_t)N_XCD * mx;
  } else {
    sched.assign(nb + 1, 0);
    for (int z = 0; z < nb; ++z) sched[z + 1] = sched[z] + count[z];
    g = ((int64_t)sched[nb] + N_XCD - 1) / N_XCD * N_XCD;
  }
  ABDDC_REQUIRE(g < (int64_t(1) << 24), ABDDC_EINVAL, "batched dense launch: too many tiles");
  RaggedGrid r;
  if (g == 0) return r;
  r.sched = ar.put(sched);
  r.grid = (unsigned)g;
  return r;
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  // output register q of lane l holds row (l/16) + 4q of the 16x16 block
  static __device__ inline int out_row(int kl, int q) { return kl + 4 * q; }
  static __device__ inline acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  typedef v4f acc_t;
  // output register q of lane l holds row 4(l/16) + q of the 16x16 block
  static __device__ inline int out_row(int kl, int q) { return 4 * kl + q; }
  static __device__ inline acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// 1 / x from the hardware reciprocal and Newton steps e = 1 - x r,
// r += r e (two for FP64, one for FP32): a few dependent operations instead
// of the IEEE division sequence, correct to about an ulp -- for the
// multipliers of the diagonal-block LU, where the pivot chain is the
// critical path.
template <class T>
__device__ inline T recip(T x);
template <>
__device__ inline double recip<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
template <>
__device__ inline float recip<float>(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// One 64x64 tile of C = alpha op(A) op(B) + beta C, op(A) m x k, op(B) k x n,
// tile origin (row0, col0); entries with row and column both >= kmask, or
// both < skip_lo, are left unwritten.  A wave owns a 32x32 quadrant made of 2x2 MFMA
// blocks of 16x16; lane l feeds A[l%16][k+l/16], B[k+l/16][l%16]; the
// output rows each lane holds depend on the instruction (Mfma::out_row).  Safe in place when C aliases op(A)'s
// rows (n <= TILE) or op(B)'s columns (m <= TILE): all reads of a tile
// precede its writes.
template <class T, bool TA, bool TB, bool C_LDS = false>
__device__ __forceinline__ void tile_gemm(const T* __restrict__ A, int lda, const T* __restrict__ B, int ldb, T* C,
                          int ldc, int m, int n, int k, T alpha, T beta, int row0, int col0,
                          T (*As)[LDS_PAD], T (*Bs)[LDS_PAD], int kmask = 0x7fffffff, int skip_lo = 0) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int PER = TILE * KC / 256;   // elements of each operand per thread and chunk (8)
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  // Load layouts (contiguous direction across lanes):
  //   A row-major (!TA): i = (tid >> 5) + 8q, kk = tid & 31
  //   A k-major  (TA):   kk = (tid >> 6) + 4q, i = tid & 63
  //   B k-major (!TB):   kk = (tid >> 6) + 4q, j = tid & 63
  //   B row-major (TB):  j = (tid >> 5) + 8q, kk = tid & 31
  const int a_i0 = TA ? (tid & 63) : (tid >> 5), a_k0 = TA ? (tid >> 6) : (tid & 31);
  const int b_j0 = TB ? (tid >> 5) : (tid & 63), b_k0 = TB ? (tid & 31) : (tid >> 6);
  const int a_di = TA ? 0 : 8, a_dk = TA ? 4 : 0;
  const int b_dj = TB ? 8 : 0, b_dk = TB ? 0 : 4;
  const int kl = lane >> 4, il = lane & 15;
  // C is read up front, straight into the accumulator layout, so its loads
  // overlap the first operand chunk instead of trailing the last MFMA; the
  // accumulators start at (beta / alpha) C and the result is alpha * acc
  // (alpha != 0).
  acc_t acc[2][2];
  const __amdgpu_buffer_rsrc_t rsa = buf_rsrc(A), rsb = buf_rsrc(B), rsc = buf_rsrc(C_LDS ? nullptr : C);
  if (beta != T(0)) {
    const T cs = beta / alpha;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = row0 + wr + 16 * bi + Mfma<T>::out_row(kl, q);
          const int c = col0 + wc + 16 * bj + il;
          if constexpr (C_LDS) {
            acc[bi][bj][q] = (r < m && c < n) ? cs * C[(size_t)r * ldc + c] : T(0);
          } else {
            const int oc = (r < m && c < n) ? (r * ldc + c) * (int)sizeof(T) : BUF_OUT;
            acc[bi][bj][q] = cs * buf_load<T>(rsc, oc, 0);
          }
        }
  } else {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
  }
  T ra[PER], rb[PER];
  // byte offsets of the thread's elements in chunk 0, BUF_OUT where the row
  // of op(A) or the column of op(B) lies outside; chunk k0 adds the
  // wave-uniform k0 * (bytes per unit of k) as the scalar offset
  const int ar = row0 + a_i0, bc = col0 + b_j0;
  int oa[PER], ob[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int ai = ar + q * a_di, ak = a_k0 + q * a_dk;
    oa[q] = ai < m ? (TA ? ak * lda + ai : ai * lda + ak) * (int)sizeof(T) : BUF_OUT;
    const int bj = bc + q * b_dj, bk = b_k0 + q * b_dk;
    ob[q] = bj < n ? (TB ? bj * ldb + bk : bk * ldb + bj) * (int)sizeof(T) : BUF_OUT;
  }
  const int ska = (TA ? lda : 1) * (int)sizeof(T), skb = (TB ? 1 : ldb) * (int)sizeof(T);
  auto fetch = [&](int k0) {
    const int sa = k0 * ska, sb = k0 * skb;
    if (k0 + KC <= k) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        ra[q] = buf_load<T>(rsa, oa[q], sa);
        rb[q] = buf_load<T>(rsb, ob[q], sb);
      }
    } else {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        ra[q] = buf_load<T>(rsa, k0 + a_k0 + q * a_dk < k ? oa[q] : BUF_OUT, sa);
        rb[q] = buf_load<T>(rsb, k0 + b_k0 + q * b_dk < k ? ob[q] : BUF_OUT, sb);
      }
    }
  };
  // which of the wave's 16 x 16 blocks have a row / column inside C (a full
  // 2 x 2 set on every interior tile)
  const bool rok0 = row0 + wr < m, rok1 = row0 + wr + 16 < m;
  const bool cok0 = col0 + wc < n, cok1 = col0 + wc + 16 < n;
  const bool full = rok1 && cok1;
  if (k > 0) fetch(0);
#pragma unroll 1
  for (int k0 = 0; k0 < k; k0 += KC) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      As[a_k0 + q * a_dk][a_i0 + q * a_di] = ra[q];
      Bs[b_k0 + q * b_dk][b_j0 + q * b_dj] = rb[q];
    }
    __syncthreads();
    if (k0 + KC < k) fetch(k0 + KC);   // next chunk in flight during the MFMAs
    if (full) {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        T a0 = As[kk + kl][wr + il];
        T a1 = As[kk + kl][wr + 16 + il];
        T b0 = Bs[kk + kl][wc + il];
        T b1 = Bs[kk + kl][wc + 16 + il];
        acc[0][0] = Mfma<T>::run(a0, b0, acc[0][0]);
        acc[0][1] = Mfma<T>::run(a0, b1, acc[0][1]);
        acc[1][0] = Mfma<T>::run(a1, b0, acc[1][0]);
        acc[1][1] = Mfma<T>::run(a1, b1, acc[1][1]);
      }
    } else if (rok0 && cok0) {
      // a tile at the edge of C: 16 x 16 blocks with no row or no column
      // inside C are skipped (wave-uniform tests)
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        T a0 = As[kk + kl][wr + il];
        T b0 = Bs[kk + kl][wc + il];
        acc[0][0] = Mfma<T>::run(a0, b0, acc[0][0]);
        if (cok1) acc[0][1] = Mfma<T>::run(a0, Bs[kk + kl][wc + 16 + il], acc[0][1]);
        if (rok1) acc[1][0] = Mfma<T>::run(As[kk + kl][wr + 16 + il], b0, acc[1][0]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int r = row0 + wr + 16 * bi + Mfma<T>::out_row(kl, q);
        int c = col0 + wc + 16 * bj + il;
        const bool st = r < m && c < n && (r < kmask || c < kmask) && !(r < skip_lo && c < skip_lo);
        if constexpr (C_LDS) {
          if (st) C[(size_t)r * ldc + c] = alpha * acc[bi][bj][q];
        } else {
          buf_store<T>(alpha * acc[bi][bj][q], rsc, st ? (r * ldc + c) * (int)sizeof(T) : BUF_OUT, 0);
        }
      }
}

template <class T, bool TA, bool TB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) gemm_batched_kernel(const GemmDesc<T>* __restrict__ descs,
                                                            const int32_t* __restrict__ sched, int nb, T alpha, T beta) {
  __shared__ T As[KC][LDS_PAD];
  __shared__ T Bs[KC][LDS_PAD];
  int z, t;
  if (!ragged_tile(sched, nb, z, t)) return;
  const GemmDesc<T> d = descs[z];
  const int tn = (d.n + TILE - 1) / TILE;
  const int tm = (d.m + TILE - 1) / TILE;
  if (t >= tm * tn) return;
  const int ti = t / tn, tj = t % tn;
  tile_gemm<T, TA, TB>(d.A, d.lda, d.B, d.ldb, d.C, d.ldc, d.m, d.n, d.k, alpha, beta, ti * TILE,
                       tj * TILE, As, Bs);
}

// C = alpha op(A) op(B) + beta C for thin products: k <= THIN and either
// n <= THIN ("tall") or m <= THIN ("wide"), where a 64 x 64 MFMA tile would
// leave most of its lanes idle (an interface edge of 7 dofs).
//   tall: a workgroup takes THIN_ROWS rows of C; op(A)'s rows (k entries
//         each) and op(B) (k x n) are staged in LDS, so a wave's loads cover
//         several rows of contiguous entries, and one thread per entry of C
//         writes the rows back;
//   wide: one thread per column of C, all its m rows, with op(A) (m x k)
//         staged in LDS and op(B)'s column read coalesced across threads.
// Safe in place when C aliases op(A)'s rows (tall) or op(B)'s columns
// (wide): a workgroup (thread) reads what it overwrites before it writes it.
constexpr int THIN = 32;
constexpr int THIN_ROWS = 64;

template <class T, bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_thin_kernel(const GemmDesc<T>* __restrict__ descs, int nd, T alpha,
                                                        T beta) {
  __shared__ T As[THIN_ROWS][THIN + 1];
  __shared__ T Bs[THIN][THIN + 1];
  for (int z = blockIdx.y; z < nd; z += gridDim.y) {
    const GemmDesc<T> d = descs[z];
    const bool tall = d.n <= THIN;
    const int span = tall ? THIN_ROWS : (int)blockDim.x;   // rows (tall) or columns (wide) per workgroup
    const int len = tall ? d.m : d.n, base = blockIdx.x * span;
    if (base >= len) continue;   // the same for the whole workgroup
    __syncthreads();             // the previous descriptor's tiles are no longer read
    if (tall) {
      const int rows = min(THIN_ROWS, d.m - base);
      for (int q = threadIdx.x; q < rows * d.k; q += blockDim.x) {
        const int r = q / d.k, kk = q % d.k;
        As[r][kk] = TA ? d.A[(size_t)kk * d.lda + base + r] : d.A[(size_t)(base + r) * d.lda + kk];
      }
      for (int q = threadIdx.x; q < d.k * d.n; q += blockDim.x) {
        const int kk = q / d.n, c = q % d.n;
        Bs[kk][c] = TB ? d.B[(size_t)c * d.ldb + kk] : d.B[(size_t)kk * d.ldb + c];
      }
      __syncthreads();
      for (int q = threadIdx.x; q < rows * d.n; q += blockDim.x) {
        const int r = q / d.n, c = q % d.n;
        T acc = T(0);
        for (int kk = 0; kk < d.k; ++kk) acc += As[r][kk] * Bs[kk][c];
        T* cp = d.C + (size_t)(base + r) * d.ldc + c;
        *cp = beta != T(0) ? alpha * acc + beta * *cp : alpha * acc;
      }
    } else {
      for (int q = threadIdx.x; q < d.m * d.k; q += blockDim.x) {
        const int r = q / d.k, kk = q % d.k;
        Bs[r][kk] = TA ? d.A[(size_t)kk * d.lda + r] : d.A[(size_t)r * d.lda + kk];
      }
      __syncthreads();
      const int i = base + threadIdx.x;
      if (i < len) {
        T v[THIN];
#pragma unroll
        for (int kk = 0; kk < THIN; ++kk)
          v[kk] = kk < d.k ? (TB ? d.B[(size_t)i * d.ldb + kk] : d.B[(size_t)kk * d.ldb + i]) : T(0);
        for (int r = 0; r < d.m; ++r) {
          T acc = T(0);
#pragma unroll
          for (int kk = 0; kk < THIN; ++kk)
            if (kk < d.k) acc += Bs[r][kk] * v[kk];
          T* cp = d.C + (size_t)r * d.ldc + i;
          *cp = beta != T(0) ? alpha * acc + beta * *cp : alpha * acc;
        }
      }
    }
  }
}

// --------------------------------------------------------------- partial LU
template <class T>
__device__ inline T read_lane(T v, int lane);
template <>
__device__ inline double read_lane<double>(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <>
__device__ inline float read_lane<float>(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Step 1 of panel t0: factor the diagonal block (b = min(NB, k - t0)) and
// write L\U back, L^{-1} (unit lower) and U^{-1} to scratch.  The block is
// padded in LDS to diag(D, I) of order 64, which factors and inverts to
// diag(L\U, I), diag(L^{-1}, I), diag(U^{-1}, I), so every loop below runs
// to 64 with no size tests.  The LU is blocked in 16-column sub-panels:
//   (a) wave 0 factors the 64 x 16 column panel in registers (lane = row;
//       pivot rows broadcast by readlane, no LDS traffic and no barriers),
//   (b) wave 0 solves the 16-row block row with the unit lower 16 x 16
//       factor (lane = column),
//   (c) all waves update the trailing block.
// The inverses are one column per lane: wave 0 forward-substitutes L,
// wave 1 back-substitutes U, each holding its column in registers.
template <class T>
__global__ void __launch_bounds__(256) plu_diag_kernel(const PluDesc<T>* __restrict__ descs, int t0,
                                                        T* __restrict__ scratch, int* dflag) {
  constexpr int H = NB / 2;
  __shared__ T D[NB][NB + 1];
  __shared__ T E[NB][NB + 1];
  __shared__ T dinv[NB];
  const PluDesc<T> d = descs[blockIdx.x];
  if (t0 >= d.k) return;
  const int b = min(NB, d.k - t0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  T* base = d.a + (size_t)t0 * d.ld + t0;
  {
    // all sixteen rows of the wave requested at once (buffer loads: entries
    // outside the b x b block read zero and become the identity padding)
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(base);
    T v[NB / 4];
#pragma unroll
    for (int i = 0; i < NB / 4; ++i) {
      const int r = wave + 4 * i;
      v[i] = buf_load<T>(rs, (r < b && lane < b) ? (r * d.ld + lane) * (int)sizeof(T) : BUF_OUT, 0);
    }
#pragma unroll
    for (int i = 0; i < NB / 4; ++i) {
      const int r = wave + 4 * i;
      D[r][lane] = (r < b && lane < b) ? v[i] : T(r == lane);
    }
  }
  __syncthreads();
  for (int kb = 0; kb < b; kb += 16) {
    if (wave == 0) {
      T P[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) P[j] = D[lane][kb + j];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int pr = kb + j;
        const T piv = read_lane(P[j], pr);
        const T inv = recip(piv);
        T u[16];
#pragma unroll
        for (int j2 = j + 1; j2 < 16; ++j2) u[j2] = read_lane(P[j2], pr);
        if (lane > pr) {
          const T l = P[j] * inv;
          P[j] = l;
#pragma unroll
          for (int j2 = j + 1; j2 < 16; ++j2) P[j2] -= l * u[j2];
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) D[lane][kb + j] = P[j];
    }
    __syncthreads();
    if (wave == 0 && lane >= kb + 16) {
      T X[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) X[t] = D[kb + t][lane];
#pragma unroll
      for (int t = 1; t < 16; ++t) {
        T a[2] = {T(0), T(0)};   // two independent chains
#pragma unroll
        for (int q = 0; q < t; ++q) a[q & 1] += D[kb + t][kb + q] * X[q];
        X[t] -= a[0] + a[1];
      }
#pragma unroll
      for (int t = 0; t < 16; ++t) D[kb + t][lane] = X[t];
    }
    __syncthreads();
    // trailing block [kb + 16, 64)^2 -= L(:, kb..kb+16) U(kb..kb+16, :) on
    // MFMA, one 16 x 16 output block per wave at a time (9, 4, 1 blocks)
    {
      const int nbk = (NB - kb - 16) / 16;
      const int kl = lane >> 4, il = lane & 15;
      for (int blk = wave; blk < nbk * nbk; blk += 4) {
        const int r0 = kb + 16 + 16 * (blk / nbk), c0 = kb + 16 + 16 * (blk % nbk);
        typename Mfma<T>::acc_t acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = D[r0 + Mfma<T>::out_row(kl, q)][c0 + il];
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) acc = Mfma<T>::run(-D[r0 + il][kb + kk + kl], D[kb + kk + kl][c0 + il], acc);
#pragma unroll
        for (int q = 0; q < 4; ++q) D[r0 + Mfma<T>::out_row(kl, q)][c0 + il] = acc[q];
      }
    }
    __syncthreads();
  }
  {
    // buffer stores (not counted with the LDS operations, so neither the
    // reads below nor the barrier wait for them)
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(base);
#pragma unroll
    for (int i = 0; i < NB / 4; ++i) {
      const int r = wave + 4 * i;
      buf_store<T>(D[r][lane], rs, (r < b && lane < b) ? (r * d.ld + lane) * (int)sizeof(T) : BUF_OUT, 0);
    }
  }
  if (wave == 1) {
    // the pivots are the diagonal of U: flag a zero or non-finite one
    const T dv = D[lane][lane];
    dinv[lane] = T(1) / dv;
    const bool bad = lane < b && (!(fabs((double)dv) > 0.0) || !isfinite((double)dv));
    if (__ballot(bad) && lane == 0) atomicOr(dflag, 1);
  }
  __syncthreads();
  T* gLi = scratch + (size_t)blockIdx.x * 2 * NB * NB;
  T* gUi = gLi + NB * NB;
  // Inverses by 32 x 32 blocks:
  //   L^{-1} = [[L11^{-1}, 0], [-L22^{-1} (L21 L11^{-1}), L22^{-1}]]
  //   U^{-1} = [[U11^{-1}, -U11^{-1} (U12 U22^{-1})], [0, U22^{-1}]]
  // with each 32 x 32 inverse built the same way from 16 x 16 blocks.  Layout
  // of the four 32 x 32 inverses in E: E11 = L11^{-1}, E22 = L22^{-1},
  // E21 = U11^{-1}, E12 = U22^{-1} (U block rows shifted by 32).
  // (1a) the eight 16 x 16 diagonal-block inverses, one column per lane
  //      (lane 16 j + c: column c of block j): wave 0 the unit lower L_jj,
  //      wave 1 the upper U_jj; waves 2 and 3 write the zero blocks
  {
    const int j = lane >> 4, c = lane & 15, o = 16 * j;
    if (wave == 0) {
      T X[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        T a[2] = {T(0), T(0)};   // two independent chains
#pragma unroll
        for (int q = 0; q < r; ++q) a[q & 1] += D[o + r][o + q] * X[q];
        X[r] = T(r == c) - (a[0] + a[1]);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) E[o + r][o + c] = X[r];
    } else if (wave == 1) {
      T X[16];
#pragma unroll
      for (int r = 15; r >= 0; --r) {
        T a[2] = {T(0), T(0)};
#pragma unroll
        for (int q = r + 1; q < 16; ++q) a[q & 1] += D[o + r][o + q] * X[q];
        X[r] = (T(r == c) - (a[0] + a[1])) * dinv[o + r];
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) E[((o + 32) & 63) + r][o + c] = X[r];
    } else {
      // zero blocks: upper right of each L 32-inverse (wave 2), lower left of
      // each U 32-inverse (wave 3); lane = block (j & 1) x column c, 16 rows
      const int p = j & 1, o32 = 32 * p;
      if (j < 2) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          if (wave == 2) E[o32 + r][o32 + 16 + c] = T(0);
          else E[((o32 + 32) & 63) + 16 + r][o32 + c] = T(0);
        }
      }
    }
  }
  __syncthreads();
  // (1b) the off-diagonal 16 x 16 block of each 32 x 32 inverse on MFMA:
  //      wave p (0, 1): L block p, T = L21 L11^{-1} over the L21 block of D,
  //      then -L22^{-1} T; wave 2 + p: U block p, T = U12 U22^{-1} over the U12
  //      block of D, then -U11^{-1} T (16 x 16 blocks inside the 32-block)
  {
    typedef typename Mfma<T>::acc_t acc_t;
    const int kl = lane >> 4, il = lane & 15;
    const bool isL = wave < 2;
    const int o = 32 * (wave & 1), eo = (o + 32) & 63;
    acc_t t1 = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      if (isL)
        t1 = Mfma<T>::run(D[o + 16 + il][o + kk + kl], E[o + kk + kl][o + il], t1);
      else
        t1 = Mfma<T>::run(D[o + il][o + 16 + kk + kl], E[eo + 16 + kk + kl][o + 16 + il], t1);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = Mfma<T>::out_row(kl, q);
      if (isL) D[o + 16 + r][o + il] = t1[q];
      else D[o + r][o + 16 + il] = t1[q];
    }
    __syncthreads();
    acc_t t2 = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      if (isL)
        t2 = Mfma<T>::run(E[o + 16 + il][o + 16 + kk + kl], D[o + 16 + kk + kl][o + il], t2);
      else
        t2 = Mfma<T>::run(E[eo + il][o + kk + kl], D[o + kk + kl][o + 16 + il], t2);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = Mfma<T>::out_row(kl, q);
      if (isL) E[o + 16 + r][o + il] = -t2[q];
      else E[eo + r][o + 16 + il] = -t2[q];
    }
  }
  __syncthreads();
  // (2), (3): the four 32 x 32 x 32 products on MFMA; wave w computes the
  // 16 x 16 block (w / 2, w % 2) of both products of a phase
  {
    typedef typename Mfma<T>::acc_t acc_t;
    const int kl = lane >> 4, il = lane & 15, bi = wave >> 1, bj = wave & 1;
    acc_t p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < H; kk += 4) {
      p1 = Mfma<T>::run(D[H + 16 * bi + il][kk + kl], E[kk + kl][16 * bj + il], p1);           // L21 L11^{-1}
      p2 = Mfma<T>::run(D[16 * bi + il][H + kk + kl], E[kk + kl][H + 16 * bj + il], p2);       // U12 U22^{-1}
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * bi + Mfma<T>::out_row(kl, q), cc = 16 * bj + il;
      D[H + r][cc] = p1[q];
      D[r][H + cc] = p2[q];
    }
    __syncthreads();
    acc_t p3 = {0, 0, 0, 0}, p4 = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < H; kk += 4) {
      p3 = Mfma<T>::run(E[H + 16 * bi + il][H + kk + kl], D[H + kk + kl][16 * bj + il], p3);   // L22^{-1} T1
      p4 = Mfma<T>::run(E[H + 16 * bi + il][kk + kl], D[kk + kl][H + 16 * bj + il], p4);       // U11^{-1} T2
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = 16 * bi + Mfma<T>::out_row(kl, q), cc = 16 * bj + il;
      gLi[(H + r) * NB + cc] = -p3[q];
      gUi[r * NB + H + cc] = -p4[q];
    }
  }
  // the block-diagonal parts and zeros
  const int pi = tid >> 3, pj = tid & 7;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = pj + 8 * q;
    gLi[pi * NB + j] = E[pi][j];
    gLi[(H + pi) * NB + H + j] = E[H + pi][H + j];
    gLi[pi * NB + H + j] = T(0);
    gUi[pi * NB + j] = E[H + pi][j];
    gUi[(H + pi) * NB + H + j] = E[pi][H + j];
    gUi[(H + pi) * NB + j] = T(0);
  }
}

// One 64-wide tile of a panel's triangular solves, by the explicit inverses
// of the diagonal block (K = b <= 64, two K chunks at most):
//   ROW:  C (m x b) <- C U^{-1}, U^{-1} upper triangular (the B operand)
//   !ROW: C (b x n) <- L^{-1} C, L^{-1} lower triangular (the A operand)
// Output block v (a 16-column block for ROW, a 16-row block otherwise)
// takes only k < 16 (v + 1): the zero 16 x 16 blocks of the triangular
// factor are skipped, 40 of the 64 MFMA steps of the dense product.  Wave w
// owns stripe w of the tile (16 rows for ROW, 16 columns otherwise) across
// all four blocks v, so every wave issues the same 40 steps (blocks beyond
// the edge of C multiply the zeros that the bounded loads read and are not
// stored; a per-block test here makes the compiler spill).  Loads follow
// tile_gemm<T, false, false>; in place (C aliasing A or B) is safe: every
// read of the tile has landed in LDS before the barrier that precedes the
// MFMAs of its last chunk, and the stores come after those.
template <class T, bool ROW>
__device__ __forceinline__ void tile_trsm(const T* __restrict__ A, int lda, const T* __restrict__ B, int ldb, T* C,
                                          int ldc, int m, int n, int k, T (*As)[LDS_PAD], T (*Bs)[LDS_PAD]) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int PER = TILE * KC / 256;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int kl = lane >> 4, il = lane & 15;
  // A row-major: i = (tid >> 5) + 8q, kk = tid & 31; B k-major: kk = (tid >> 6) + 4q, j = tid & 63
  const int a_i0 = tid >> 5, a_k0 = tid & 31, b_j0 = tid & 63, b_k0 = tid >> 6;
  const __amdgpu_buffer_rsrc_t rsa = buf_rsrc(A), rsb = buf_rsrc(B), rsc = buf_rsrc(C);
  int oa[PER], ob[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int ai = a_i0 + 8 * q;
    oa[q] = ai < m ? (ai * lda + a_k0) * (int)sizeof(T) : BUF_OUT;
    ob[q] = b_j0 < n ? ((b_k0 + 4 * q) * ldb + b_j0) * (int)sizeof(T) : BUF_OUT;
  }
  T ra[PER], rb[PER];
  auto fetch = [&](int k0) {
    const int sa = k0 * (int)sizeof(T), sb = k0 * ldb * (int)sizeof(T);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      ra[q] = buf_load<T>(rsa, k0 + a_k0 < k ? oa[q] : BUF_OUT, sa);
      rb[q] = buf_load<T>(rsb, k0 + b_k0 + 4 * q < k ? ob[q] : BUF_OUT, sb);
    }
  };
  acc_t acc[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = acc_t{0, 0, 0, 0};
  const bool wok = 16 * w < (ROW ? m : n);  // the wave's stripe holds part of C
  if (k > 0) fetch(0);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int k0 = c * KC;
    if (k0 >= k) break;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      As[a_k0][a_i0 + 8 * q] = ra[q];
      Bs[b_k0 + 4 * q][b_j0] = rb[q];
    }
    __syncthreads();
    if (c == 0 && KC < k) fetch(KC);   // the second chunk in flight during the first chunk's MFMAs
    if (wok) {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        const T sv = ROW ? As[kk + kl][16 * w + il] : Bs[kk + kl][16 * w + il];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (c * KC + kk >= 16 * (v + 1)) continue;   // zero block of the factor (compile time)
          if (ROW)
            acc[v] = Mfma<T>::run(sv, Bs[kk + kl][16 * v + il], acc[v]);
          else
            acc[v] = Mfma<T>::run(As[kk + kl][16 * v + il], sv, acc[v]);
        }
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = ROW ? 16 * w + Mfma<T>::out_row(kl, q) : 16 * v + Mfma<T>::out_row(kl, q);
      const int cc = ROW ? 16 * v + il : 16 * w + il;
      buf_store<T>(acc[v][q], rsc, (r < m && cc < n) ? (r * ldc + cc) * (int)sizeof(T) : BUF_OUT, 0);
    }
}

// Step 2: A21 <- A21 U11^{-1} (row tiles), A12 <- L11^{-1} A12 (column tiles).
template <class T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) plu_trsm_kernel(const PluDesc<T>* __restrict__ descs, int t0,
                                                        const T* __restrict__ scratch, const int32_t* __restrict__ sched, int nb) {
  __shared__ T As[KC][LDS_PAD];
  __shared__ T Bs[KC][LDS_PAD];
  int z, t;
  if (!ragged_tile(sched, nb, z, t)) return;
  const PluDesc<T> d = descs[z];
  if (t0 >= d.k) return;
  const int b = min(NB, d.k - t0);
  const int mr = d.nrow - t0 - b, nc = d.ncol - t0 - b;
  const int rt = (mr + TILE - 1) / TILE, ct = (nc + TILE - 1) / TILE;
  const T* Li = scratch + (size_t)z * 2 * NB * NB;
  const T* Ui = Li + NB * NB;
  if (t < rt) {
    T* C = d.a + (size_t)(t0 + b + t * TILE) * d.ld + t0;
    const int m = min(TILE, mr - t * TILE);
    tile_trsm<T, true>(C, d.ld, Ui, NB, C, d.ld, m, b, b, As, Bs);
  } else if (t < rt + ct) {
    const int c = t - rt;
    T* C = d.a + (size_t)t0 * d.ld + t0 + b + c * TILE;
    const int n = min(TILE, nc - c * TILE);
    tile_trsm<T, false>(Li, NB, C, d.ld, C, d.ld, b, n, b, As, Bs);
  }
}

// The leading k columns are factored in 64-column panels taken in groups of
// G (two; three when the batch's longest elimination has 257 to 512 pivots,
// four above 512).  After each panel but the last of a group, plu_band_kernel
// updates only what the next one needs (its column strip and its row strip)
// with every pivot of the group so far; after the last, plu_lead_kernel
// applies the whole group (depth 64 G) to the rest of the part still to be
// factored.  Every matrix entry of that part is thus read and written once
// per 64 G pivots rather than once per 64; the deeper groups move work into
// the narrower band updates, which pays only when there are many panels.

// Band update after panel [t0, s) of the group starting at g0, s = t0 + b,
// with the pivots [g0, s): rows [s, nrow) x cols [s, s + w) and rows
// [s, s + w) x cols [s + w, ncol), w = min(NB, k - s).
// Tile t < ceil((nrow - s) / TILE) is a tile of the column strip, the rest
// are tiles of the row strip.
template <class T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) plu_band_kernel(const PluDesc<T>* __restrict__ descs, int g0,
                                                                                                       int t0, const int32_t* __restrict__ sched, int nb) {
  __shared__ T As[KC][LDS_PAD];
  __shared__ T Bs[KC][LDS_PAD];
  int z, t;
  if (!ragged_tile(sched, nb, z, t)) return;
  const PluDesc<T> d = descs[z];
  if (t0 >= d.k) return;
  const int s0 = t0 + min(NB, d.k - t0), b = s0 - g0;   // pivots [g0, s0) of the group so far
  if (s0 >= d.k) return;
  const int w = min(NB, d.k - s0);
  const int mr = d.nrow - s0, nc = d.ncol - s0;
  const int rtl = (mr + TILE - 1) / TILE;
  const T* A21 = d.a + (size_t)s0 * d.ld + g0;
  const T* A12 = d.a + (size_t)g0 * d.ld + s0;
  T* A22 = d.a + (size_t)s0 * d.ld + s0;
  if (t < rtl) {
    tile_gemm<T, false, false>(A21, d.ld, A12, d.ld, A22, d.ld, mr, w, b, T(-1), T(1), t * TILE, 0, As, Bs);
  } else {
    const int col0 = w + (t - rtl) * TILE;
    if (col0 >= nc) return;
    tile_gemm<T, false, false>(A21, d.ld, A12, d.ld, A22, d.ld, w, nc, b, T(-1), T(1), 0, col0, As, Bs);
  }
}

// Update after the pivot columns [t0, s), s = t0 + b, b = min(kb, k - t0),
// restricted to what is still to be factored: rows [s, nrow) x cols [s, k)
// and rows [s, k) x cols [k, ncol).  The block beyond k in both directions
// is formed once at the end by plu_update_kernel.
template <class T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) plu_lead_kernel(const PluDesc<T>* __restrict__ descs, int t0,
                                                                                                      int kb, const int32_t* __restrict__ sched, int nb) {
  __shared__ T As[KC][LDS_PAD];
  __shared__ T Bs[KC][LDS_PAD];
  int z, t;
  if (!ragged_tile(sched, nb, z, t)) return;
  const PluDesc<T> d = descs[z];
  if (t0 >= d.k) return;
  const int b = min(kb, d.k - t0), s0 = t0 + b;
  if (s0 >= d.k) return;
  const int mr = d.nrow - s0, nc = d.ncol - s0, kr = d.k - s0;
  const int ct = (nc + TILE - 1) / TILE;
  const int row0 = (t / ct) * TILE, col0 = (t % ct) * TILE;  // relative to s0
  if (row0 >= mr || col0 >= nc) return;
  if (row0 >= kr && col0 >= kr) return;   // tile entirely in the trailing block
  const T* A21 = d.a + (size_t)s0 * d.ld + t0;
  const T* A12 = d.a + (size_t)t0 * d.ld + s0;
  T* A22 = d.a + (size_t)s0 * d.ld + s0;
  // only entries with row < kr or col < kr are written
  tile_gemm<T, false, false>(A21, d.ld, A12, d.ld, A22, d.ld, mr, nc, b, T(-1), T(1), row0, col0, As, Bs, kr);
}

// Trailing Schur complement A22 -= A21 A12 with K = k (one pass).
template <class T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) plu_update_kernel(const PluDesc<T>* __restrict__ descs, const int32_t* __restrict__ sched, int nb) {
  __shared__ T As[KC][LDS_PAD];
  __shared__ T Bs[KC][LDS_PAD];
  int z, t;
  if (!ragged_tile(sched, nb, z, t)) return;
  const PluDesc<T> d = descs[z];
  const int k = d.k;
  if (k == 0) return;
  const int mr = d.nrow - k, nc = d.ncol - k;
  const int ct = (nc + TILE - 1) / TILE;
  const int row0 = (t / ct) * TILE, col0 = (t % ct) * TILE;
  if (row0 >= mr || col0 >= nc) return;
  const T* A21 = d.a + (size_t)k * d.ld;
  const T* A12 = d.a + k;
  T* A22 = d.a + (size_t)k * d.ld + k;
  tile_gemm<T, false, false>(A21, d.ld, A12, d.ld, A22, d.ld, mr, nc, k, T(-1), T(1), row0, col0, As, Bs);
}

// One wave per destination row (rows strided over the grid's waves), lanes
// along the row: the row's source index is read once per wave, the column
// map and both rows are walked with unit stride across lanes.
__global__ void __launch_bounds__(256) gather_kernel(const GatherDesc* __restrict__ descs) {
  const GatherDesc d = descs[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int nwv = gridDim.x * (blockDim.x >> 6);
  for (int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < d.nr; r += nwv) {
    const int sr = d.rmap ? d.rmap[r] : r;
    double* drow = d.dst + (size_t)r * d.ldd;
    if (sr < 0) {
      for (int c = lane; c < d.nc; c += 64) drow[c] = 0.0;
      continue;
    }
    const double* srow = d.src + (size_t)sr * d.lds;
    // eight columns per lane at a time (a row of up to 512 in one round of
    // two load latencies: the column map, then the source), every load of a
    // group issued before its stores (the stores could alias the maps or the
    // source as far as the compiler knows, so a plain loop waits out both
    // load latencies per column)
    constexpr int U = 8;
    for (int c0 = lane; c0 < d.nc; c0 += 64 * U) {
      int sc[U];
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + 64 * u;
        sc[u] = c < d.nc ? (d.cmap ? d.cmap[c] : c) : -1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = sc[u] >= 0 ? srow[sc[u]] : 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + 64 * u;
        if (c < d.nc) drow[c] = d.scale * v[u];
      }
    }
  }
}

__global__ void set_kernel(const SetDesc* __restrict__ descs) {
  const SetDesc d = descs[blockIdx.y];
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < d.n; q += gridDim.x * blockDim.x)
    d.dst[(size_t)d.rows[q] * d.ld + d.cols[q]] = d.val;
}

__global__ void sym_kernel(const SymDesc* __restrict__ descs) {
  const SymDesc d = descs[blockIdx.y];
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < d.n * d.n; idx += gridDim.x * blockDim.x) {
    const int r = idx / d.n, c = idx % d.n;
    d.dst[(size_t)r * d.ldd + c] = 0.5 * (d.src[(size_t)r * d.lds + c] + d.src[(size_t)c * d.lds + r]);
  }
}

}  // namespace


template <class T>
void partial_lu(const std::vector<PluDesc<T>>& descs_in, int* dflag, hipStream_t s) {
  if (descs_in.empty()) return;
  // largest eliminations first: on ragged batches their workgroups are
  // dispatched first and the small ones fill in behind them
  std::vector<PluDesc<T>> descs(descs_in);
  std::stable_sort(descs.begin(), descs.end(), [](const PluDesc<T>& a, const PluDesc<T>& b) {
    return (double)a.k * a.nrow * a.ncol > (double)b.k * b.nrow * b.ncol;
  });
  int maxk = 0;
  for (auto& d : descs) {
    ABDDC_REQUIRE(d.k >= 0 && d.k <= d.nrow && d.k <= d.ncol && d.ld >= d.ncol, ABDDC_EINVAL,
                  "partial_lu: bad matrix shape");
    ABDDC_REQUIRE((int64_t)d.nrow * d.ld * (int64_t)sizeof(T) < BUF_LIMIT, ABDDC_EINVAL,
                  "partial_lu: matrix spans 2 GiB or more");
    maxk = std::max(maxk, d.k);
  }
  if (maxk == 0) return;
  HostTrace ht;
  Arena& ar = Arena::for_stream(s);
  const PluDesc<T>* dd = ar.put(descs);
  static thread_local DevBuf<char> scratch;
  size_t need = descs.size() * 2 * NB * NB * sizeof(T);
  if (scratch.n < need) {
    ABDDC_HIP(hipStreamSynchronize(s));
    AllocScope own(nullptr);   // outlives every context: the library's cache
    scratch.alloc(need);
  }
  T* scr = reinterpret_cast<T*>(scratch.p);
  const int nb = (int)descs.size();
  // The band / lead launch of panel t0 also updates the next diagonal block
  // (one more tile at the same depth), so the diag kernel of panel t0 + NB
  // follows it and factors the block as it finds it.
  const int grp = maxk > 512 ? 4 : (maxk > 256 ? 3 : 2);   // panels per group
  // Algorithmic flops of each launch for the live kernel statistics (only
  // counted when a statistics sink is set):
  //   diag  LU of the b x b diagonal block, 2/3 b^3
  //   trsm  bytes, not flops (b^2 flops per 16 b bytes of strip is below
  //         the FP64 ridge): each strip entry of L21 and U12 read and written
  //         once, the two b x b inverses read once
  //   band  the strips of the next panel at the group's depth
  auto diag_launch = [&](int t0) {
    double f = 0.0;
    if (kstats_on(KC_PLU_DIAG))
      for (auto& d : descs)
        if (t0 < d.k) {
          const double b = std::min(NB, d.k - t0);
          f += 2.0 / 3.0 * b * b * b;
        }
    hipEvent_t ea = nullptr, eb = nullptr;
    tracked_events(KC_PLU_DIAG, f, &ea, &eb);
    hipExtLaunchKernelGGL(plu_diag_kernel<T>, dim3(nb), dim3(256), 0, s, ea, eb, 0, dd, t0, scr, dflag);
  };
  diag_launch(0);
  auto tiles_of = [](int n) { return n > 0 ? (n + TILE - 1) / TILE : 0; };
  std::vector<int> cnt(nb);
  for (int t0 = 0; t0 < maxk; t0 += NB) {
    // triangular solves: the row strip and the column strip of every matrix
    // with pivots left
    for (int z = 0; z < nb; ++z) {
      const PluDesc<T>& d = descs[z];
      const int b = std::min(NB, d.k - t0);
      cnt[z] = t0 < d.k ? tiles_of(d.nrow - t0 - b) + tiles_of(d.ncol - t0 - b) : 0;
    }
    const RaggedGrid gt = ragged_grid(cnt, ar);
    if (gt.grid) {
      double f = 0.0;
      if (kstats_on(KC_PLU_TRSM))
        for (auto& d : descs)
          if (t0 < d.k) {
            const double b = std::min(NB, d.k - t0);
            f += 16.0 * b * ((double)(d.nrow - t0 - b) + (double)(d.ncol - t0 - b)) + 16.0 * b * b;
          }
      hipEvent_t ea = nullptr, eb = nullptr;
      tracked_events(KC_PLU_TRSM, f, &ea, &eb);
      hipExtLaunchKernelGGL(plu_trsm_kernel<T>, dim3(gt.grid), dim3(256), 0, s, ea, eb, 0, dd, t0, (const T*)scr,
                            gt.sched, nb);
    }
    const int g0 = t0 - ((t0 / NB) % grp) * NB;
    if ((t0 / NB) % grp != grp - 1) {
      // not the last panel of its group: the band the next panel needs
      if (t0 + NB < maxk) {
        // column strip tiles + row strip tiles (the row strip starts at
        // column w of the trailing part)
        for (int z = 0; z < nb; ++z) {
          const PluDesc<T>& d = descs[z];
          cnt[z] = 0;
          if (t0 >= d.k) continue;
          const int s0 = t0 + std::min(NB, d.k - t0);
          if (s0 >= d.k) continue;
          const int w = std::min(NB, d.k - s0);
          cnt[z] = tiles_of(d.nrow - s0) + tiles_of(d.ncol - s0 - w);
        }
        const RaggedGrid gb = ragged_grid(cnt, ar);
        if (gb.grid) {
          double f = 0.0;
          if (kstats_on(KC_PLU_BAND))
            for (auto& d : descs)
              if (t0 < d.k) {
                const int s0 = t0 + std::min(NB, d.k - t0);
                if (s0 >= d.k) continue;
                const double w = std::min(NB, d.k - s0), mr = d.nrow - s0, nc = d.ncol - s0;
                f += 2.0 * (s0 - g0) * (mr * w + w * (nc - w));
              }
          hipEvent_t ea = nullptr, eb = nullptr;
          tracked_events(KC_PLU_BAND, f, &ea, &eb);
          hipExtLaunchKernelGGL(plu_band_kernel<T>, dim3(gb.grid), dim3(256), 0, s, ea, eb, 0, dd, g0, t0, gb.sched,
                                nb);
        }
        diag_launch(t0 + NB);
      }
      continue;
    }
    // last panel of a group: all its panels, depth grp NB
    const int p0 = g0, sp = p0 + grp * NB;
    for (int z = 0; z < nb; ++z) {
      const PluDesc<T>& d = descs[z];
      const int s0 = p0 + std::min(grp * NB, d.k - p0);
      cnt[z] = (p0 < d.k && s0 < d.k) ? tiles_of(d.nrow - s0) * tiles_of(d.ncol - s0) : 0;
    }
    const RaggedGrid gl = ragged_grid(cnt, ar);
    if (sp < maxk && gl.grid) {
      hipEvent_t ea = nullptr, eb = nullptr;
      if (kstats_on(KC_PLU_LEAD)) {
        // rows [s, nrow) x cols [s, k) and rows [s, k) x cols [k, ncol) at
        // depth b
        double flops = 0.0;
        for (auto& d : descs)
          if (sp < d.k) {
            flops += 2.0 * (grp * NB) * ((double)(d.nrow - sp) * (d.k - sp) + (double)(d.k - sp) * (d.ncol - d.k));
          }
        tracked_events(KC_PLU_LEAD, flops, &ea, &eb);
      }
      hipExtLaunchKernelGGL(plu_lead_kernel<T>, dim3(gl.grid), dim3(256), 0, s, ea, eb, 0, dd, p0, grp * NB,
                            gl.sched, nb);
    }
    if (t0 + NB < maxk) diag_launch(t0 + NB);
  }
  // trailing Schur complement with K = k
  double flops = 0.0;
  for (int z = 0; z < nb; ++z) {
    const PluDesc<T>& d = descs[z];
    cnt[z] = d.k > 0 ? tiles_of(d.nrow - d.k) * tiles_of(d.ncol - d.k) : 0;
    flops += 2.0 * (double)(d.nrow - d.k) * (double)(d.ncol - d.k) * d.k;
  }
  const RaggedGrid gu = ragged_grid(cnt, ar);
  if (gu.grid) {
    hipEvent_t ea, eb;
    tracked_events(KC_PLU_UPDATE, flops, &ea, &eb);
    hipExtLaunchKernelGGL(plu_update_kernel<T>, dim3(gu.grid), dim3(256), 0, s, ea, eb, 0, dd, gu.sched, nb);
  }
  ABDDC_HIP(hipGetLastError());
  ht.mark("partial LU queued");
}

template <class T>
void gemm_batched(const std::vector<GemmDesc<T>>& descs_in, bool transA, bool transB, T alpha, T beta,
                  hipStream_t s) {
  if (descs_in.empty()) return;
  ABDDC_REQUIRE(alpha != T(0) || beta == T(0), ABDDC_EINVAL, "gemm: alpha = 0 with beta != 0");
  // thin products (k and one side of C at most THIN) to the streaming kernel
  std::vector<GemmDesc<T>> descs, thin;
  int thin_len = 0;
  for (const auto& d : descs_in) {
    ABDDC_REQUIRE(d.m >= 0 && d.n >= 0 && d.k >= 0, ABDDC_EINVAL, "gemm: negative size");
    const int64_t ea = (int64_t)(transA ? d.k : d.m) * d.lda, eb = (int64_t)(transB ? d.n : d.k) * d.ldb;
    ABDDC_REQUIRE(std::max({ea, eb, (int64_t)d.m * d.ldc}) * (int64_t)sizeof(T) < BUF_LIMIT, ABDDC_EINVAL,
                  "gemm: operand spans 2 GiB or more");
    if (d.m == 0 || d.n == 0) continue;
    if (d.k <= THIN && (d.n <= THIN || d.m <= THIN)) {
      thin.push_back(d);
      // workgroups along the long side: THIN_ROWS rows (tall) or 256 columns (wide)
      thin_len = std::max(thin_len, d.n <= THIN ? (d.m + THIN_ROWS - 1) / THIN_ROWS : (d.n + 255) / 256);
    } else {
      descs.push_back(d);
    }
  }
  Arena& ar = Arena::for_stream(s);
  if (!thin.empty()) {
    const GemmDesc<T>* dt = ar.put(thin);
    const int nd = (int)thin.size();
    const dim3 grid(thin_len, std::min(nd, 65535));
    if (!transA && !transB) gemm_thin_kernel<T, false, false><<<grid, 256, 0, s>>>(dt, nd, alpha, beta);
    else if (transA && !transB) gemm_thin_kernel<T, true, false><<<grid, 256, 0, s>>>(dt, nd, alpha, beta);
    else if (!transA && transB) gemm_thin_kernel<T, false, true><<<grid, 256, 0, s>>>(dt, nd, alpha, beta);
    else gemm_thin_kernel<T, true, true><<<grid, 256, 0, s>>>(dt, nd, alpha, beta);
    ABDDC_HIP(hipGetLastError());
  }
  if (descs.empty()) return;
  std::vector<int> cnt(descs.size());
  for (size_t z = 0; z < descs.size(); ++z) {
    const auto& d = descs[z];
    cnt[z] = ((d.m + TILE - 1) / TILE) * ((d.n + TILE - 1) / TILE);
  }
  const RaggedGrid rg = ragged_grid(cnt, ar);
  if (rg.grid == 0) return;
  const GemmDesc<T>* dd = ar.put(descs);
  const int nb = (int)descs.size();
  const dim3 grid(rg.grid);
  if (!transA && !transB) gemm_batched_kernel<T, false, false><<<grid, 256, 0, s>>>(dd, rg.sched, nb, alpha, beta);
  else if (transA && !transB) gemm_batched_kernel<T, true, false><<<grid, 256, 0, s>>>(dd, rg.sched, nb, alpha, beta);
  else if (!transA && transB) gemm_batched_kernel<T, false, true><<<grid, 256, 0, s>>>(dd, rg.sched, nb, alpha, beta);
  else gemm_batched_kernel<T, true, true><<<grid, 256, 0, s>>>(dd, rg.sched, nb, alpha, beta);
  ABDDC_HIP(hipGetLastError());
}

void gather_batched(const std::vector<GatherDesc>& descs, hipStream_t s) {
  if (descs.empty()) return;
  int maxe = 0, maxr = 0;
  for (auto& d : descs) {
    maxe = std::max(maxe, d.nr * d.nc);
    maxr = std::max(maxr, d.nr);
  }
  if (maxe == 0) return;
  Arena& ar = Arena::for_stream(s);
  const GatherDesc* dd = ar.put(descs);
  const int gx = std::min((maxr + 3) / 4, 1024);   // four rows (waves) per workgroup
  gather_kernel<<<dim3(gx, descs.size()), 256, 0, s>>>(dd);
  ABDDC_HIP(hipGetLastError());
}

void set_batched(const std::vector<SetDesc>& descs, hipStream_t s) {
  int maxe = 0;
  for (auto& d : descs) maxe = std::max(maxe, d.n);
  if (descs.empty() || maxe == 0) return;
  const SetDesc* dd = Arena::for_stream(s).put(descs);
  set_kernel<<<dim3(std::min((maxe + 255) / 256, 256), descs.size()), 256, 0, s>>>(dd);
  ABDDC_HIP(hipGetLastError());
}

void sym_batched(const std::vector<SymDesc>& descs, hipStream_t s) {
  int maxe = 0;
  for (auto& d : descs) maxe = std::max(maxe, d.n * d.n);
  if (descs.empty() || maxe == 0) return;
  const SymDesc* dd = Arena::for_stream(s).put(descs);
  sym_kernel<<<dim3(std::min((maxe + 255) / 256, 256), descs.size()), 256, 0, s>>>(dd);
  ABDDC_HIP(hipGetLastError());
}

template void partial_lu<double>(const std::vector<PluDesc<double>>&, int*, hipStream_t);
template void partial_lu<float>(const std::vector<PluDesc<float>>&, int*, hipStream_t);
template void gemm_batched<double>(const std::vector<GemmDesc<double>>&, bool, bool, double, double,
                                   hipStream_t);
template void gemm_batched<float>(const std::vector<GemmDesc<float>>&, bool, bool, float, float,
                                  hipStream_t);

}  // namespace abddc
