// Assembly of the GLS-stabilised system (Section 2) on trilinear boxes or on
// six linear tetrahedra per box into dense per-subdomain matrices
// [A^(i) | f^(i)] in local order [interior; Gamma_i] (Section 3), extraction
// of S^(i), g^(i), B^(i) after the interior elimination, and interior
// recovery u_I = A_II^{-1}(f_I - A_IB u_B).
//
// a(u, v) = int nu grad u . grad v + C_K Lu Lv + ctilde u v
//           + 1/2 (a . grad u v - a . grad v u),
// g(v)    = int f v + C_K f Lv,   L u = a . grad u + c u inside an element,
// C_K from the Peclet switch with tau; entry (i, j) = a(phi_j, phi_i).
// Nonzero Dirichlet data u_0 are lifted: the load of row i loses
// sum_j A_K[i][j] u_0[j] over the box's boundary corners j.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "assemble.h"
#include "internal.h"

namespace abddc {

namespace {

// Trilinear basis function i at reference point (s, t, u) of a box with
// reciprocal edge lengths (ihx, ihy, ihz): value and physical gradient.
// (+-1) / h equals +-(1 / h) exactly, so passing reciprocals changes no bit
// against dividing here.
__device__ inline void shape(double s, double t, double u, int i, double ihx, double ihy, double ihz,
                             double& phi, double& gx, double& gy, double& gz) {
  const int a = i & 1, b = (i >> 1) & 1, c = (i >> 2) & 1;
  const double fs = a ? s : 1.0 - s, ft = b ? t : 1.0 - t, fu = c ? u : 1.0 - u;
  phi = fs * ft * fu;
  gx = (a ? ihx : -ihx) * ft * fu;
  gy = fs * (b ? ihy : -ihy) * fu;
  gz = fs * ft * (c ? ihz : -ihz);
}

// Lifting of Dirichlet data into the load of row i of a box: F_K[i] -=
// A_K[i][j] u_0[j] for every corner j on the grid boundary.
__device__ inline double lift_row(const ElemParams& P, const double* __restrict__ u0, const double (&row)[8],
                                  int ex, int ey, int ez, double fi) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int ix = ex + (j & 1), iy = ey + ((j >> 1) & 1), iz = ez + ((j >> 2) & 1);
    const bool bnd = ix == 0 || iy == 0 || iz == 0 || ix == P.nn[0] - 1 || iy == P.nn[1] - 1 || iz == P.nn[2] - 1;
    if (bnd) fi -= row[j] * u0[ix + (int64_t)P.nn[0] * (iy + (int64_t)P.nn[1] * iz)];
  }
  return fi;
}

// One thread per (element, test function i): row i of A_K and F_K[i].
// NODAL: the load is interpolated from nodal values (a separate instance, so
// the constant-load one keeps its state in registers).
template <bool NODAL>
__global__ void elem_kernel(ElemParams P, const double* __restrict__ nu, ElemFields Fd, double* __restrict__ Ae,
                            double* __restrict__ Fe) {
  const double* __restrict__ fnodal = Fd.f_nodal;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= P.n_elem * 8) return;
  const int64_t e = tid >> 3;
  const int i = (int)(tid & 7);
  const int ex = (int)(e % P.ne[0]);
  const int ey = (int)((e / P.ne[0]) % P.ne[1]);
  const int ez = (int)(e / ((int64_t)P.ne[0] * P.ne[1]));
  const double hx = P.h[0], hy = P.h[1], hz = P.h[2];
  const double ihx = 1.0 / hx, ihy = 1.0 / hy, ihz = 1.0 / hz;
  const double x0 = P.origin[0] + ex * hx, y0 = P.origin[1] + ey * hy, z0 = P.origin[2] + ez * hz;
  const double nue = nu[e];
  // |a|_K: maximum over the corners (|a| is convex for affine a)
  double amax = 0.0;
  for (int k = 0; k < 8; ++k) {
    const double xc = x0 + (k & 1) * hx, yc = y0 + ((k >> 1) & 1) * hy, zc = z0 + ((k >> 2) & 1) * hz;
    const double ax = P.b0[0] + P.b1[0] * xc + P.b1[1] * yc + P.b1[2] * zc;
    const double ay = P.b0[1] + P.b1[3] * xc + P.b1[4] * yc + P.b1[5] * zc;
    const double az = P.b0[2] + P.b1[6] * xc + P.b1[7] * yc + P.b1[8] * zc;
    amax = fmax(amax, sqrt(ax * ax + ay * ay + az * az));
  }
  const double hK = sqrt(hx * hx + hy * hy + hz * hz);
  const double peclet = hK * amax / (2.0 * nue);
  const double CK = (peclet >= 1.0) ? P.tau * hK / (2.0 * amax) : P.tau * hK * hK / (4.0 * nue);
  const double ctil = P.c - 0.5 * (P.b1[0] + P.b1[4] + P.b1[8]);
  // 3-point Gauss rule per axis; the 27 points in one loop (s slowest, u
  // fastest), not unrolled, and no indexed local arrays, so the thread's
  // state stays in registers
  const double q0 = 0.5 - 0.5 * sqrt(0.6), q2 = 0.5 + 0.5 * sqrt(0.6);
  const double w0 = 5.0 / 18.0, w1 = 8.0 / 18.0;
  const double vol = hx * hy * hz;
  double row[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double fi = 0.0;
#pragma unroll 1
  for (int qi = 0; qi < 27; ++qi) {
    const int a = qi / 9, b = (qi / 3) % 3, cq = qi % 3;
    const double s = a == 0 ? q0 : (a == 1 ? 0.5 : q2);
    const double t = b == 0 ? q0 : (b == 1 ? 0.5 : q2);
    const double u = cq == 0 ? q0 : (cq == 1 ? 0.5 : q2);
    const double w = (a == 1 ? w1 : w0) * (b == 1 ? w1 : w0) * (cq == 1 ? w1 : w0) * vol;
    const double xq = x0 + s * hx, yq = y0 + t * hy, zq = z0 + u * hz;
    const double ax = P.b0[0] + P.b1[0] * xq + P.b1[1] * yq + P.b1[2] * zq;
    const double ay = P.b0[1] + P.b1[3] * xq + P.b1[4] * yq + P.b1[5] * zq;
    const double az = P.b0[2] + P.b1[6] * xq + P.b1[7] * yq + P.b1[8] * zq;
    double phii, gix, giy, giz;
    shape(s, t, u, i, ihx, ihy, ihz, phii, gix, giy, giz);
    const double agi = ax * gix + ay * giy + az * giz;
    const double Li = agi + P.c * phii;
    double fq = P.f_const;
    if constexpr (NODAL) {
      fq = 0.0;
      for (int k = 0; k < 8; ++k) {
        double pk, g1, g2, g3;
        shape(s, t, u, k, ihx, ihy, ihz, pk, g1, g2, g3);
        const int64_t node =
            (ex + (k & 1)) + (int64_t)P.nn[0] * ((ey + ((k >> 1) & 1)) + (int64_t)P.nn[1] * (ez + ((k >> 2) & 1)));
        fq += fnodal[node] * pk;
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      double phij, gjx, gjy, gjz;
      shape(s, t, u, j, ihx, ihy, ihz, phij, gjx, gjy, gjz);
      const double agj = ax * gjx + ay * gjy + az * gjz;
      const double Lj = agj + P.c * phij;
      row[j] += w * (nue * (gix * gjx + giy * gjy + giz * gjz) + CK * Li * Lj + ctil * phii * phij +
                     0.5 * (agj * phii - agi * phij));
    }
    fi += w * (fq * phii + CK * fq * Li);
  }
  if (Fd.u_dirichlet) fi = lift_row(P, Fd.u_dirichlet, row, ex, ey, ez, fi);
  for (int j = 0; j < 8; ++j) Ae[e * 64 + i * 8 + j] = row[j];
  Fe[e * 8 + i] = fi;
}

// The six tetrahedra of a box: tetrahedron t is the corner path
// 0 -> e_p0 -> e_p0 + e_p1 -> 7 for the t-th ordering (p0, p1, p2) of the
// axes in lexicographic order.  With xi_a the box-local coordinates in
// [0, 1], its barycentric coordinates are 1 - xi_p0, xi_p0 - xi_p1,
// xi_p1 - xi_p2, xi_p2, whose gradients are read off directly.
__device__ constexpr int KUHN_PERM[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// One thread per (box, test function i): row i of the box matrix and load as
// the sum over the box's tetrahedra that contain corner i.  Velocity and
// source are interpolated linearly on each tetrahedron from the corner
// values; the symmetric 4-point rule (barycentric alpha, beta, beta, beta,
// alpha = (5 + 3 sqrt 5) / 20, beta = (5 - sqrt 5) / 20) is exact for every
// product of two linear factors.  ctilde = c - div(a_h) / 2 per tetrahedron,
// |a|_K = the largest vertex speed, h_K = the box diagonal (the longest
// tetrahedron edge).
template <bool NODAL_F, bool NODAL_A>
__global__ void elem_p1_kernel(ElemParams P, const double* __restrict__ nu, ElemFields Fd,
                               double* __restrict__ Ae, double* __restrict__ Fe) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= P.n_elem * 8) return;
  const int64_t e = tid >> 3;
  const int i = (int)(tid & 7);
  const int ex = (int)(e % P.ne[0]);
  const int ey = (int)((e / P.ne[0]) % P.ne[1]);
  const int ez = (int)(e / ((int64_t)P.ne[0] * P.ne[1]));
  const double h[3] = {P.h[0], P.h[1], P.h[2]};
  const double ih[3] = {1.0 / h[0], 1.0 / h[1], 1.0 / h[2]};
  double av[8][3], fc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ix = ex + (k & 1), iy = ey + ((k >> 1) & 1), iz = ez + ((k >> 2) & 1);
    const int64_t node = ix + (int64_t)P.nn[0] * (iy + (int64_t)P.nn[1] * iz);
    if constexpr (NODAL_A) {
      av[k][0] = Fd.a_nodal[3 * node];
      av[k][1] = Fd.a_nodal[3 * node + 1];
      av[k][2] = Fd.a_nodal[3 * node + 2];
    } else {
      const double xc = P.origin[0] + ix * h[0], yc = P.origin[1] + iy * h[1], zc = P.origin[2] + iz * h[2];
#pragma unroll
      for (int d = 0; d < 3; ++d) av[k][d] = P.b0[d] + P.b1[3 * d] * xc + P.b1[3 * d + 1] * yc + P.b1[3 * d + 2] * zc;
    }
    if constexpr (NODAL_F) fc[k] = Fd.f_nodal[node];
    else fc[k] = P.f_const;
  }
  const double hK = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
  const double w = h[0] * h[1] * h[2] / 6.0 * 0.25;
  const double qa = (5.0 + 3.0 * sqrt(5.0)) / 20.0, qb = (5.0 - sqrt(5.0)) / 20.0;
  double row[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double fi = 0.0;
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    const int p0 = KUHN_PERM[t][0], p1 = KUHN_PERM[t][1], p2 = KUHN_PERM[t][2];
    const int v[4] = {0, 1 << p0, (1 << p0) + (1 << p1), 7};
    const int li = i == v[0] ? 0 : (i == v[1] ? 1 : (i == v[2] ? 2 : (i == v[3] ? 3 : -1)));
    if (li < 0) continue;
    double G[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    G[0][p0] = -ih[p0];
    G[1][p0] = ih[p0];
    G[1][p1] = -ih[p1];
    G[2][p1] = ih[p1];
    G[2][p2] = -ih[p2];
    G[3][p2] = ih[p2];
    const double nut = nu[e * 6 + t];
    double diva = 0.0, amax = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double* a = av[v[k]];
      diva += a[0] * G[k][0] + a[1] * G[k][1] + a[2] * G[k][2];
      amax = fmax(amax, sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]));
    }
    const double peclet = hK * amax / (2.0 * nut);
    const double CK = (peclet >= 1.0) ? P.tau * hK / (2.0 * amax) : P.tau * hK * hK / (4.0 * nut);
    const double ctil = P.c - 0.5 * diva;
    const double gi0 = li == 0 ? G[0][0] : (li == 1 ? G[1][0] : (li == 2 ? G[2][0] : G[3][0]));
    const double gi1 = li == 0 ? G[0][1] : (li == 1 ? G[1][1] : (li == 2 ? G[2][1] : G[3][1]));
    const double gi2 = li == 0 ? G[0][2] : (li == 1 ? G[1][2] : (li == 2 ? G[2][2] : G[3][2]));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double aq[3] = {0, 0, 0}, fq = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double lk = k == q ? qa : qb;
#pragma unroll
        for (int d = 0; d < 3; ++d) aq[d] += lk * av[v[k]][d];
        fq += lk * fc[v[k]];
      }
      const double lami = li == q ? qa : qb;
      const double agi = aq[0] * gi0 + aq[1] * gi1 + aq[2] * gi2;
      const double Li = agi + P.c * lami;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double lk = k == q ? qa : qb;
        const double agk = aq[0] * G[k][0] + aq[1] * G[k][1] + aq[2] * G[k][2];
        const double Lk = agk + P.c * lk;
        row[v[k]] += w * (nut * (gi0 * G[k][0] + gi1 * G[k][1] + gi2 * G[k][2]) + CK * Li * Lk +
                          ctil * lami * lk + 0.5 * (agk * lami - agi * lk));
      }
      fi += w * (fq * lami + CK * fq * Li);
    }
  }
  if (Fd.u_dirichlet) fi = lift_row(P, Fd.u_dirichlet, row, ex, ey, ez, fi);
  for (int j = 0; j < 8; ++j) Ae[e * 64 + i * 8 + j] = row[j];
  Fe[e * 8 + i] = fi;
}

// One thread per local row (subdomain s, local node p): the 27 possible
// couplings and the load, summed over the elements of s in a fixed order.
__global__ void scatter_kernel(const SubAsm* __restrict__ subs, const int32_t* __restrict__ rowsub,
                               const int32_t* __restrict__ lnode, const int32_t* __restrict__ lmap,
                               int64_t nrows, int nn0, int nn1, int ne0, int ne1, const double* __restrict__ Ae,
                               const double* __restrict__ Fe, const int32_t* __restrict__ part,
                               double* __restrict__ A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrows) return;
  const int s = rowsub[t];
  const SubAsm S = subs[s];
  const int p = (int)(t - S.loff);
  const int node = lnode[t];
  const int ix = node % nn0, iy = (node / nn0) % nn1, iz = node / (nn0 * nn1);
  const int bx = S.ebox[1] - S.ebox[0] + 1, by = S.ebox[3] - S.ebox[2] + 1;
  double* arow = A + S.aoff + (int64_t)p * S.ld;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int qx = ix + dx, qy = iy + dy, qz = iz + dz;
        if (qx < S.ebox[0] || qx > S.ebox[1] || qy < S.ebox[2] || qy > S.ebox[3] || qz < S.ebox[4] ||
            qz > S.ebox[5])
          continue;
        const int lq = lmap[S.lmoff + (qx - S.ebox[0]) + bx * ((qy - S.ebox[2]) + by * (qz - S.ebox[4]))];
        if (lq < 0) continue;
        double sum = 0.0;
        for (int ez = max(max(iz, qz) - 1, S.ebox[4]); ez <= min(min(iz, qz), S.ebox[5] - 1); ++ez)
          for (int ey = max(max(iy, qy) - 1, S.ebox[2]); ey <= min(min(iy, qy), S.ebox[3] - 1); ++ey)
            for (int ex = max(max(ix, qx) - 1, S.ebox[0]); ex <= min(min(ix, qx), S.ebox[1] - 1); ++ex) {
              const int64_t e = ex + (int64_t)ne0 * (ey + (int64_t)ne1 * ez);
              if (part && part[e] != s) continue;
              const int il = (ix - ex) + 2 * (iy - ey) + 4 * (iz - ez);
              const int jl = (qx - ex) + 2 * (qy - ey) + 4 * (qz - ez);
              sum += Ae[e * 64 + il * 8 + jl];
            }
        arow[lq] = sum;
      }
  double f = 0.0;
  for (int ez = max(iz - 1, S.ebox[4]); ez <= min(iz, S.ebox[5] - 1); ++ez)
    for (int ey = max(iy - 1, S.ebox[2]); ey <= min(iy, S.ebox[3] - 1); ++ey)
      for (int ex = max(ix - 1, S.ebox[0]); ex <= min(ix, S.ebox[1] - 1); ++ex) {
        const int64_t e = ex + (int64_t)ne0 * (ey + (int64_t)ne1 * ez);
        if (part && part[e] != s) continue;
        f += Fe[e * 8 + (ix - ex) + 2 * (iy - ey) + 4 * (iz - ez)];
      }
  arow[S.nloc] = f;
}

// S^(i) = trailing block after eliminating the interior, g^(i) = trailing
// rhs column, B^(i) = (S + S^T) / 2.
__global__ void __launch_bounds__(256) extract_kernel(const SubAsm* __restrict__ subs, const double* __restrict__ A,
                                                      double* __restrict__ S, double* __restrict__ B,
                                                      double* __restrict__ g) {
  // one pair of 32 x 32 tiles (I, J) and (J, I), I <= J, of the trailing
  // block per workgroup: both are read once with unit-stride rows into LDS,
  // and S and B = (S + S^T) / 2 are written for both, so the transposed
  // operand costs neither strided global reads nor a second read
  __shared__ double Ta[32][33], Tb[32][33];
  const SubAsm d = subs[blockIdx.y];
  const int nB = d.nloc - d.nI, nt = (nB + 31) / 32;
  if ((int)blockIdx.x >= nt * nt) return;
  const int I = blockIdx.x / nt, J = blockIdx.x % nt;
  if (I > J) return;   // its pair is handled by workgroup (J, I)
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double* T = A + d.aoff + (int64_t)d.nI * d.ld + d.nI;
  for (int r = ty; r < 32; r += 8) {
    const int i = I * 32 + r, j = J * 32 + tx, i2 = J * 32 + r, j2 = I * 32 + tx;
    Ta[r][tx] = (i < nB && j < nB) ? T[(int64_t)i * d.ld + j] : 0.0;
    if (I != J) Tb[r][tx] = (i2 < nB && j2 < nB) ? T[(int64_t)i2 * d.ld + j2] : 0.0;
  }
  __syncthreads();
  const double (*Tm)[33] = I != J ? Tb : Ta;   // the mirror tile (J, I)
  for (int r = ty; r < 32; r += 8) {
    const int i = I * 32 + r, j = J * 32 + tx;
    if (i < nB && j < nB) {
      const double sij = Ta[r][tx];
      S[d.soff + (int64_t)i * nB + j] = sij;
      B[d.soff + (int64_t)i * nB + j] = 0.5 * (sij + Tm[tx][r]);
    }
    if (I != J) {
      const int i2 = J * 32 + r, j2 = I * 32 + tx;
      if (i2 < nB && j2 < nB) {
        const double sji = Tb[r][tx];
        S[d.soff + (int64_t)i2 * nB + j2] = sji;
        B[d.soff + (int64_t)i2 * nB + j2] = 0.5 * (sji + Ta[tx][r]);
      }
    }
  }
  if (I == J && ty == 0 && I * 32 + tx < nB) {
    const int i = I * 32 + tx;
    g[d.goff + i] = T[(int64_t)i * d.ld + nB];
  }
}

__device__ inline double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ inline double read_lane_d(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// u_I = U11^{-1} (c - U12 u_B) with A_II = L11 U11, c = L11^{-1} f_I and
// U12 = L11^{-1} A_IB left in place by the interior elimination.  One
// workgroup per subdomain: t = c - U12 u_B one row per wave (lanes stride
// the row, coalesced); then back substitution in 64-row panels from the
// bottom: the panel's right-hand side b = t_p - U_{p,below} x_below (one
// row per wave), and its 64 x 64 triangular solve in one wave with the
// panel's diagonal block staged in LDS (lane l holds b_l; step r takes x_r
// from lane r by readlane and updates the lanes above it).
__global__ void __launch_bounds__(1024) recover_kernel(const SubAsm* __restrict__ subs, const double* __restrict__ A,
                                                      const int32_t* __restrict__ gam, const double* __restrict__ uhat,
                                                      const int32_t* __restrict__ int_dof, double* __restrict__ u) {
  extern __shared__ double sm[];
  __shared__ double Ud[64][65];
  __shared__ double bv[64];
  const SubAsm d = subs[blockIdx.x];
  const int nI = d.nI, nB = d.nloc - d.nI;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  double* xs = sm;        // t, then x (nI)
  double* ub = sm + nI;   // u_B gathered (nB)
  const double* M = A + d.aoff;
  for (int c = tid; c < nB; c += blockDim.x) ub[c] = uhat[gam[d.goff + c]];
  __syncthreads();
  // two rows per wave at a time, so their load chains overlap
  for (int r = 2 * wave; r < nI; r += 2 * nw) {
    const bool two = r + 1 < nI;
    const double* row = M + (int64_t)r * d.ld + nI;
    double v0 = 0.0, v1 = 0.0;
    for (int c = lane; c < nB; c += 64) {
      const double x = ub[c];
      v0 += row[c] * x;
      if (two) v1 += row[d.ld + c] * x;
    }
    v0 = wave_sum_d(v0);
    v1 = wave_sum_d(v1);
    if (lane == 0) {
      xs[r] = M[(int64_t)r * d.ld + d.nloc] - v0;
      if (two) xs[r + 1] = M[(int64_t)(r + 1) * d.ld + d.nloc] - v1;
    }
  }
  __syncthreads();
  for (int p1 = nI; p1 > 0;) {
    const int p0 = ((p1 - 1) / 64) * 64, len = p1 - p0;
    for (int i = wave; i < 64; i += nw)
      Ud[i][lane] = (i < len && lane < len) ? M[(int64_t)(p0 + i) * d.ld + p0 + lane] : (i == lane ? 1.0 : 0.0);
    for (int r = p0 + wave; r < p1; r += nw) {
      const double* row = M + (int64_t)r * d.ld;
      double v = 0.0;
      for (int q = p1 + lane; q < nI; q += 64) v += row[q] * xs[q];
      v = wave_sum_d(v);
      if (lane == 0) bv[r - p0] = xs[r] - v;
    }
    __syncthreads();
    if (wave == 0) {
      // reciprocal pivots, one per lane, off the substitution chain
      const double rp = 1.0 / Ud[lane][lane];
      double b = lane < len ? bv[lane] : 0.0, x = 0.0;
      for (int r = len - 1; r >= 0; --r) {
        const double xr = read_lane_d(b, r) * read_lane_d(rp, r);
        if (lane == r) x = xr;
        if (lane < r) b -= Ud[lane][r] * xr;
      }
      if (lane < len) xs[p0 + lane] = x;
    }
    __syncthreads();
    p1 = p0;
  }
  for (int r = tid; r < nI; r += blockDim.x) u[int_dof[d.ioff + r]] = xs[r];
}

__global__ void check_positive_kernel(const double* __restrict__ v, int64_t n, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(v[i] > 0.0 && isfinite(v[i]))) atomicOr(flag, 4);
}

__global__ void iface_scatter_kernel(const double* __restrict__ uhat, const int32_t* __restrict__ iface_dof,
                                     int64_t n, double* __restrict__ u) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) u[iface_dof[g]] = uhat[g];
}

}  // namespace

void launch_check_positive(const double* v, int64_t n, int* flag, hipStream_t s) {
  if (n == 0) return;
  check_positive_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(v, n, flag);
  ABDDC_HIP(hipGetLastError());
}

void launch_elem(const ElemParams& P, const double* nu, const ElemFields& F, double* Ae, double* Fe,
                 hipStream_t s) {
  const int64_t n = P.n_elem * 8;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (P.element == ABDDC_ELEM_P1) {
    if (F.f_nodal && F.a_nodal) elem_p1_kernel<true, true><<<grid, 256, 0, s>>>(P, nu, F, Ae, Fe);
    else if (F.f_nodal) elem_p1_kernel<true, false><<<grid, 256, 0, s>>>(P, nu, F, Ae, Fe);
    else if (F.a_nodal) elem_p1_kernel<false, true><<<grid, 256, 0, s>>>(P, nu, F, Ae, Fe);
    else elem_p1_kernel<false, false><<<grid, 256, 0, s>>>(P, nu, F, Ae, Fe);
  } else if (F.f_nodal) {
    elem_kernel<true><<<grid, 256, 0, s>>>(P, nu, F, Ae, Fe);
  } else {
    elem_kernel<false><<<grid, 256, 0, s>>>(P, nu, F, Ae, Fe);
  }
  ABDDC_HIP(hipGetLastError());
}

void launch_scatter(const SubAsm* subs, const int32_t* rowsub, const int32_t* lnode, const int32_t* lmap,
                    int64_t nrows, const int nn[3], const int ne[3], const double* Ae, const double* Fe,
                    const int32_t* part, double* A, hipStream_t s) {
  scatter_kernel<<<(unsigned)((nrows + 255) / 256), 256, 0, s>>>(subs, rowsub, lnode, lmap, nrows, nn[0], nn[1],
                                                                  ne[0], ne[1], Ae, Fe, part, A);
  ABDDC_HIP(hipGetLastError());
}

void launch_extract(const SubAsm* subs, int nsub, int max_nB, const double* A, double* S, double* B, double* g,
                    hipStream_t s) {
  const int nt = (max_nB + 31) / 32;
  if (nt == 0 || nsub == 0) return;
  extract_kernel<<<dim3(nt * nt, nsub), 256, 0, s>>>(subs, A, S, B, g);
  ABDDC_HIP(hipGetLastError());
}

void launch_recover(const SubAsm* subs, int nsub, int max_nloc, const double* A, const int32_t* gam,
                    const double* uhat, const int32_t* int_dof, const int32_t* iface_dof, int64_t n_gamma, double* u,
                    hipStream_t s) {
  ABDDC_REQUIRE((size_t)max_nloc * sizeof(double) <= 64 * 1024, ABDDC_EINVAL, "subdomain too large for recovery");
  // 16 waves per subdomain: the row sweeps are latency-bound chains of loads
  recover_kernel<<<nsub, 1024, (size_t)std::max(max_nloc, 1) * sizeof(double), s>>>(subs, A, gam, uhat, int_dof, u);
  if (n_gamma > 0) iface_scatter_kernel<<<(unsigned)((n_gamma + 255) / 256), 256, 0, s>>>(uhat, iface_dof, n_gamma, u);
  ABDDC_HIP(hipGetLastError());
}

}  // namespace abddc
