// 2D extension of the EV-FDLB step for MI355X (gfx950): a fluid homogeneous
// in z, F(x, y, p_x, p_y) = int f dp_z and G = int p_z^2/2 f dp_z on the
// tensor-product Gauss-Hermite set (p_k, p_l), k, l < 16.  The paper solves
// the 1D model and names more dimensions as the next goal (conclusions); the
// same ingredients reduced over p_z give the right-hand side
//   L = -p . grad f - F . grad_p f - nu (f - f^S) + J1
// with the Shakhov f^S (Sec. II B) and J1 (eq:J1) reduced over p_z, the
// mean-field force of eq:force integrated along z, and the averaged density
// of Sec. II A integrated along z.
//
// State d_f[2][16][16][ny][nx] (plane d*256 + k*16 + l, node fastest).  One
// TVD-RK3 stage is three kernels:
//   fields_kernel  32 x 8 nodes per workgroup, density tile with the force
//                  radius as halo in LDS: disc-averaged density, contact value
//                  (eq:carnstar), force (antisymmetric cell pairs), transport
//                  (eq:viscosity, eq:tau, eq:prandtl), 4th-order central
//                  gradients of X = n^2 chi T, T and u along x and y.
//   adv_kernel     one wavefront per strip of 58 columns x 128 rows of one
//                  velocity plane, marching down the rows with register
//                  rings; every WENO-5 face computed once from per-node
//                  stencil terms that three faces share,
//                  W = a f^n + b f^(s-1) + c Adv(f^(s-1)).
//   vel_kernel     16 nodes per wavefront, lanes = (node, group g of four p_x
//                  rows): d/dp_x as (Dp x I) on the f64 MFMA (the node's 16 x 16
//                  velocity matrix is the B operand), d/dp_y as (I x Dp) on the
//                  VALU, Hermite equilibrium, Shakhov and J1 terms,
//                  f^(s) = W + c R, and the velocity moments of f^(s).
#include "evlb2d.h"

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "tables.h"

namespace evlb2d {
namespace {

// Workgroups go to the eight XCDs in turn (workgroup b to XCD b mod 8), and
// each XCD has its own L2.  xcd_block gives XCD x the contiguous blocks
// x q + min(x, r) + i (nb = 8 q + r), so that neighbouring tiles, which share
// halo lines, run on one XCD.  A bijection of 0 .. nb - 1.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned q = nb >> 3, r = nb & 7u;
  const unsigned x = b & 7u, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

constexpr int Q = 16;
constexpr int V = Q * Q;
constexpr int HMAX = 24;  // max halo of the fields tile (force radius / averaging disc + 2)

enum {
  F_N, F_UX, F_UY, F_T, F_SQX, F_SQY, F_NU, F_PRE, F_FX, F_FY,
  F_AX, F_AY, F_BX, F_BY, F_UXX, F_UXY, F_UYX, F_UYY, NF
};

struct Dev {
  int nx, ny;
  long long ntot;
  double inv_dx;
  double b;      // 2 pi sigma^3 / 3
  double eta_c;  // pi sigma^3 / 6
  double mu0c;   // 5 / (16 sigma^2 sqrt(pi))
  double weno_eps, g_ext;
  double T_iso;  // > 0: isothermal, the temperature the next stage sees
  int force_model, term_mask;
  int navg, npair, halo;
  int* status;
};

__device__ __forceinline__ int wrap(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// Raw velocity sums of one node -> n, u, T, q (Sec. II B moments with the
// reduced G carrying the p_z energy):
//   3/2 n T = sum (|xi|^2/2 F + G),  q = sum xi (|xi|^2/2 F + G).
struct Raw {
  double n, jx, jy, pxx, pxy, pyy, rx, ry, g0, hx, hy;
};

__device__ __forceinline__ void finish_moments(const Raw& m, double* out6, long long N, long long node,
                                               int* status, double T_iso) {
  const double n = m.n;
  const double ux = m.jx / n, uy = m.jy / n;
  const double u2 = ux * ux + uy * uy;
  const double tr = m.pxx + m.pyy;
  const double T = (2.0 / 3.0) * (0.5 * tr + m.g0 - 0.5 * n * u2) / n;
  const double qx = 0.5 * (m.rx - 2.0 * (ux * m.pxx + uy * m.pxy) - ux * tr + 2.0 * n * ux * u2) + (m.hx - ux * m.g0);
  const double qy = 0.5 * (m.ry - 2.0 * (ux * m.pxy + uy * m.pyy) - uy * tr + 2.0 * n * uy * u2) + (m.hy - uy * m.g0);
  out6[node] = n;
  out6[N + node] = ux;
  out6[2 * N + node] = uy;
  out6[3 * N + node] = T_iso > 0.0 ? T_iso : T;
  out6[4 * N + node] = qx;
  out6[5 * N + node] = qy;
  if (!(n > 0.0) || !(T > 0.0) || !isfinite(n) || !isfinite(T) || !isfinite(ux) || !isfinite(uy) ||
      !isfinite(qx) || !isfinite(qy))
    status[0] = 1;
}

// ---------------------------------------------------------------------------
// moments of a state (first stage of a step, evlb_moments)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void moments_kernel(Dev D, const double* __restrict__ f, double* __restrict__ out6,
                                                      const double* __restrict__ vel, int stage_input) {
  const long long node = (long long)blockIdx.x * 256 + threadIdx.x;
  if (node >= D.ntot) return;
  const long long N = D.ntot;
  Raw m{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
  for (int k = 0; k < Q; ++k) {
    const double pk = vel[k];
#pragma unroll 4
    for (int l = 0; l < Q; ++l) {
      const double pl = vel[l];
      const double F = f[(long long)(k * Q + l) * N + node];
      const double G = f[(long long)(V + k * Q + l) * N + node];
      const double p2 = pk * pk + pl * pl;
      m.n += F;
      m.jx += pk * F;
      m.jy += pl * F;
      m.pxx += pk * pk * F;
      m.pxy += pk * pl * F;
      m.pyy += pl * pl * F;
      m.rx += pk * p2 * F;
      m.ry += pl * p2 * F;
      m.g0 += G;
      m.hx += pk * G;
      m.hy += pl * G;
    }
  }
  // as the input of a stage, an isothermal run sees its fixed temperature
  finish_moments(m, out6, N, node, D.status, stage_input ? D.T_iso : 0.0);
}

// Hermite equilibrium of one velocity component at unit density:
// a_0 = 1, a_1 = u, a_{m+1} = u a_m + m (T - 1) a_{m-1};  e_k = sum_m meq[k][m] a_m.
__device__ __forceinline__ void hermite_coeffs(double u, double T, double* a) {
  a[0] = 1.0;
  a[1] = u;
#pragma unroll
  for (int m = 1; m < Q - 1; ++m) a[m + 1] = u * a[m] + (double)m * (T - 1.0) * a[m - 1];
}

__global__ __launch_bounds__(256) void equilibrium_kernel(Dev D, const double* __restrict__ n_in,
                                                          const double* __restrict__ u_in,
                                                          const double* __restrict__ T_in, double* __restrict__ f,
                                                          const double* __restrict__ meq) {
  const long long node = (long long)blockIdx.x * 256 + threadIdx.x;
  if (node >= D.ntot) return;
  const long long N = D.ntot;
  const double n = n_in[node], ux = u_in[node], uy = u_in[N + node], T = T_in[node];
  double ax[Q], ay[Q], ey[Q];
  hermite_coeffs(ux, T, ax);
  hermite_coeffs(uy, T, ay);
#pragma unroll
  for (int l = 0; l < Q; ++l) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < Q; ++m) s += meq[l * Q + m] * ay[m];
    ey[l] = s;
  }
#pragma unroll 1
  for (int k = 0; k < Q; ++k) {
    double ex = 0.0;
#pragma unroll
    for (int m = 0; m < Q; ++m) ex += meq[k * Q + m] * ax[m];
    const double nex = n * ex;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      const double E = nex * ey[l];
      f[(long long)(k * Q + l) * N + node] = E;
      f[(long long)(V + k * Q + l) * N + node] = 0.5 * T * E;
    }
  }
}

// ---------------------------------------------------------------------------
// node fields
// ---------------------------------------------------------------------------
constexpr int FTX = 32, FTY = 8, FNT = FTX * FTY;
constexpr int GX = FTX + 4, GY = FTY + 4;  // tile +-2 (gradient stencil)

__global__ __launch_bounds__(FNT) void fields_kernel(Dev D, const double* __restrict__ mom, double* __restrict__ fld,
                                                     const int* __restrict__ avg_ofs,
                                                     const double* __restrict__ avg_w,
                                                     const int* __restrict__ pair_ofs,
                                                     const double* __restrict__ pair_cx,
                                                     const double* __restrict__ pair_cy) {
  extern __shared__ double sm[];
  const int H = D.halo, PX = FTX + 2 * H, PY = FTY + 2 * H;
  double* sn = sm;             // [PY][PX] density, node (x0 - H + c, y0 - H + r)
  double* sX = sn + PX * PY;   // [GY][GX] node (x0 - 2 + c, y0 - 2 + r)
  double* sT = sX + GX * GY;
  double* sux = sT + GX * GY;
  double* suy = sux + GX * GY;
  double* sC = suy + GX * GY;
  const int tid = threadIdx.x;
  // contiguous ranges of tiles per XCD (row-major over the tile grid): the
  // density halos of neighbouring tiles meet in one L2
  const unsigned tb = xcd_block(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int x0 = (int)(tb % gridDim.x) * FTX, y0 = (int)(tb / gridDim.x) * FTY;
  const long long N = D.ntot;
  for (int i = tid; i < PX * PY; i += FNT) {
    const int r = i / PX, c = i - r * PX;
    sn[i] = mom[(long long)wrap(y0 - H + r, D.ny) * D.nx + wrap(x0 - H + c, D.nx)];
  }
  for (int i = tid; i < GX * GY; i += FNT) {
    const int r = i / GX, c = i - r * GX;
    const long long node = (long long)wrap(y0 - 2 + r, D.ny) * D.nx + wrap(x0 - 2 + c, D.nx);
    sux[i] = mom[N + node];
    suy[i] = mom[2 * N + node];
    sT[i] = mom[3 * N + node];
  }
  __syncthreads();
  // averaged density over the disc, contact value, X on the tile +-2
  for (int i = tid; i < GX * GY; i += FNT) {
    const int r = i / GX, c = i - r * GX;
    const int ctr = (r - 2 + H) * PX + (c - 2 + H);
    double s0 = 0.0, s1 = 0.0;
    int t = 0;
    for (; t + 1 < D.navg; t += 2) {
      s0 += avg_w[t] * sn[ctr + avg_ofs[t]];
      s1 += avg_w[t + 1] * sn[ctr + avg_ofs[t + 1]];
    }
    if (t < D.navg) s0 += avg_w[t] * sn[ctr + avg_ofs[t]];
    const double eta = D.eta_c * (s0 + s1);
    const double om = 1.0 - eta;
    const double chi = (2.0 - eta) / (2.0 * om * om * om);
    const double n = sn[ctr];
    sC[i] = chi;
    sX[i] = n * n * chi * sT[i];
  }
  __syncthreads();

  const int tx = tid % FTX, ty = tid / FTX;
  const int x = x0 + tx, y = y0 + ty;
  if (x >= D.nx || y >= D.ny) return;
  const long long node = (long long)y * D.nx + x;
  const int g = (ty + 2) * GX + (tx + 2);
  const int ctr = (ty + H) * PX + (tx + H);
  const double n = sn[ctr], T = sT[g], ux = sux[g], uy = suy[g], chi = sC[g];
  double Fx = D.g_ext, Fy = 0.0;
  if (D.force_model == EVLB_FORCE_EV1) {
    double ax0 = 0.0, ax1 = 0.0, ay0 = 0.0, ay1 = 0.0;
    int t = 0;
    for (; t + 1 < D.npair; t += 2) {
      const double d0 = sn[ctr + pair_ofs[t]] - sn[ctr - pair_ofs[t]];
      const double d1 = sn[ctr + pair_ofs[t + 1]] - sn[ctr - pair_ofs[t + 1]];
      ax0 += pair_cx[t] * d0;
      ay0 += pair_cy[t] * d0;
      ax1 += pair_cx[t + 1] * d1;
      ay1 += pair_cy[t + 1] * d1;
    }
    if (t < D.npair) {
      const double d0 = sn[ctr + pair_ofs[t]] - sn[ctr - pair_ofs[t]];
      ax0 += pair_cx[t] * d0;
      ay0 += pair_cy[t] * d0;
    }
    Fx += ax0 + ax1;
    Fy = ay0 + ay1;
  }
  const double c12 = D.inv_dx * (1.0 / 12.0);
  const double X = sX[g];
  const double Ax = (sX[g - 2] - 8.0 * sX[g - 1] + 8.0 * sX[g + 1] - sX[g + 2]) * c12 / X;
  const double Ay = (sX[g - 2 * GX] - 8.0 * sX[g - GX] + 8.0 * sX[g + GX] - sX[g + 2 * GX]) * c12 / X;
  const double Bx = (sT[g - 2] - 8.0 * sT[g - 1] + 8.0 * sT[g + 1] - sT[g + 2]) * c12 / T;
  const double By = (sT[g - 2 * GX] - 8.0 * sT[g - GX] + 8.0 * sT[g + GX] - sT[g + 2 * GX]) * c12 / T;
  const double Uxx = (sux[g - 2] - 8.0 * sux[g - 1] + 8.0 * sux[g + 1] - sux[g + 2]) * c12;
  const double Uxy = (suy[g - 2] - 8.0 * suy[g - 1] + 8.0 * suy[g + 1] - suy[g + 2]) * c12;
  const double Uyx = (sux[g - 2 * GX] - 8.0 * sux[g - GX] + 8.0 * sux[g + GX] - sux[g + 2 * GX]) * c12;
  const double Uyy = (suy[g - 2 * GX] - 8.0 * suy[g - GX] + 8.0 * suy[g + GX] - suy[g + 2 * GX]) * c12;
  const double bn = D.b * n;
  const double yv = bn * chi;
  const double k12 = 0.16 * (1.0 + 12.0 / M_PI);
  const double k32 = 0.36 * (1.0 + 32.0 / (9.0 * M_PI));
  const double mu = D.mu0c * sqrt(T) * (1.0 / chi + 0.8 * bn + k12 * bn * bn * chi);
  const double nu = chi * n * T * (1.0 + 0.4 * yv) / mu;
  const double Pr = (2.0 / 3.0) * (1.0 + 0.6 * yv) * (1.0 + 0.8 * yv + k12 * yv * yv) /
                    ((1.0 + 0.4 * yv) * (1.0 + 1.2 * yv + k32 * yv * yv));
  const double s = (1.0 - Pr) / (5.0 * n * T * T);
  const double vals[NF] = {n, ux, uy, T, s * mom[4 * N + node], s * mom[5 * N + node], nu, -bn * chi, Fx, Fy,
                           Ax, Ay, Bx, By, Uxx, Uxy, Uyx, Uyy};
#pragma unroll
  for (int i = 0; i < NF; ++i) fld[i * N + node] = vals[i];
}

// ---------------------------------------------------------------------------
// advection: one wavefront per strip of 58 columns x AR rows of one plane
// ---------------------------------------------------------------------------
// WENO-5 (Jiang & Shu) rewritten around stencil centres.  A face between
// v2 and v3 (v0 .. v4 ordered from the upwind side) combines three
// candidate parabolas on the triples (v0 v1 v2), (v1 v2 v3), (v2 v3 v4).  In
// terms of one triple (a, m, b), a on the upwind side, with c = a - 2m + b and
// g = b - a, the candidate value and four times the smoothness indicator in
// each of the three roles are
//   role p (far upwind):  m + 13c/12 + 3g/4,  13c^2/3 + (2c + g)^2
//   role 0 (centred):     m +   c/12 +  g/4,  13c^2/3 + g^2
//   role m (downwind):    m +   c/12 -  g/4,  13c^2/3 + (2c - g)^2
// so every node computes its triple once and three faces share it.  The
// nonlinear weights 0.1, 0.6, 0.3 over (eps + beta_k)^2 are taken over the
// common denominator; scaling every beta by 4 and eps with it multiplies all
// three weights by the same 256, which cancels.  The division is a hardware
// reciprocal refined by two Newton steps r <- r (2 - d r).
//
// Lane t holds column x0 - 3 + t and marches down 128 rows.  Along y the
// triples of rows y - 1 .. y + 2 and the raw rows y .. y + 3 sit in rings of
// four registers indexed by row mod 4; the loop is unrolled by four so that
// every ring index is a constant.  Along x each lane builds the triple of its
// own column from its neighbours' row values and fetches the two triples it
// lacks from the lanes that own them; the face on its right comes from lane
// t + 1.  Lanes 3 .. 60 produce the 58 outputs.  No LDS, no barrier.
constexpr int AW = 58;   // output columns per wavefront
constexpr int AR = 128;  // output rows per wavefront (a multiple of 4)
constexpr int ANT = 256; // four strips per workgroup

struct AdvArgs {
  const double* fs;  // f^(s-1)
  const double* f0;  // f^n
  double* W;         // a f^n + b f^(s-1) + c Adv(f^(s-1)); may alias f0
  double a, b, c;
  int first;         // f0 == fs
};

struct Tri {
  double bp, b0, bm;  // 4 beta in the roles p, 0, m
  double qp, q0, qm;  // candidate values in the roles p, 0, m
};

__device__ __forceinline__ Tri tri(double a, double m, double b) {
  const double c = fma(-2.0, m, a + b);
  const double g = b - a;
  const double a4 = (13.0 / 3.0) * c * c;
  const double u = fma(2.0, c, g), w = fma(2.0, c, -g);
  const double h = fma(1.0 / 12.0, c, m);
  Tri t;
  t.bp = fma(u, u, a4);
  t.b0 = fma(g, g, a4);
  t.bm = fma(w, w, a4);
  t.qp = fma(0.75, g, fma(13.0 / 12.0, c, m));
  t.q0 = fma(0.25, g, h);
  t.qm = fma(-0.25, g, h);
  return t;
}

// Face value from the triple in role p (bp, qp), role 0 and role m; eps4 = 4 eps.
__device__ __forceinline__ double face3(double bp, double qp, double b0, double q0, double bm, double qm,
                                        double eps4) {
  double t0 = eps4 + bp; t0 *= t0;
  double t1 = eps4 + b0; t1 *= t1;
  double t2 = eps4 + bm; t2 *= t2;
  const double w0 = 0.1 * (t1 * t2), w1 = 0.6 * (t0 * t2), w2 = 0.3 * (t0 * t1);
  const double num = fma(w2, qm, fma(w1, q0, w0 * qp));
  const double den = w0 + w1 + w2;
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  r = fma(r, fma(-den, r, 1.0), r);
  return num * r;
}

// Oriented triple centred on m with its neighbours lo (lower index) and hi.
template <bool POS>
__device__ __forceinline__ Tri tri_dir(double lo, double m, double hi) {
  return POS ? tri(lo, m, hi) : tri(hi, m, lo);
}

struct AdvStrip {
  const double* fs;   // this plane of f^(s-1)
  const double* f0;   // this plane of f^n
  double* W;          // this plane of W
  int nx, ny, xc, yr, y0;
  bool outcol;
  double pxi, pyi, eps4;  // p_x / dx, p_y / dx
  double rw[4];       // raw rows, slot = (row - y0) mod 4
  Tri ct[4];          // triples of rows, slot = (row - y0) mod 4
  double fyl;         // face between rows y - 1 and y
  double nxr;         // row y + 3, loaded one row ahead
  double f0n;         // f^n of row y, loaded one row ahead
};

// Row y = y0 + r with r = PH (mod 4): take row y + 3 (loaded one row ahead)
// and load row y + 4, build the triple of row y + 2, the face between rows y
// and y + 1, the two x faces of row y, update.
template <bool PX, bool PY, int PH>
__device__ __forceinline__ void adv_row(AdvStrip& S, const AdvArgs& A, int r) {
  constexpr int s0 = PH & 3, s1 = (PH + 1) & 3, s2 = (PH + 2) & 3, s3 = (PH + 3) & 3;
  S.rw[s3] = S.nxr;
  S.nxr = S.fs[(long long)S.yr * S.nx + S.xc];
  if (++S.yr == S.ny) S.yr = 0;
  S.ct[s2] = tri_dir<PY>(S.rw[s1], S.rw[s2], S.rw[s3]);
  // upwind below: triples of rows y - 1, y, y + 1; above: y + 2, y + 1, y
  const double fyr = PY ? face3(S.ct[s3].bp, S.ct[s3].qp, S.ct[s0].b0, S.ct[s0].q0, S.ct[s1].bm, S.ct[s1].qm, S.eps4)
                        : face3(S.ct[s2].bp, S.ct[s2].qp, S.ct[s1].b0, S.ct[s1].q0, S.ct[s0].bm, S.ct[s0].qm, S.eps4);
  const double c0 = S.rw[s0];
  const double m1 = __shfl_up(c0, 1), p1 = __shfl_down(c0, 1);
  const Tri tx = tri_dir<PX>(m1, c0, p1);
  double fxl;  // face between columns x - 1 and x
  if (PX) {    // upwind left: triples of columns x - 2, x - 1, x
    fxl = face3(__shfl_up(tx.bp, 2), __shfl_up(tx.qp, 2), __shfl_up(tx.b0, 1), __shfl_up(tx.q0, 1), tx.bm, tx.qm,
                S.eps4);
  } else {     // upwind right: triples of columns x + 1, x, x - 1
    fxl = face3(__shfl_down(tx.bp, 1), __shfl_down(tx.qp, 1), tx.b0, tx.q0, __shfl_up(tx.bm, 1), __shfl_up(tx.qm, 1),
                S.eps4);
  }
  const double fxr = __shfl_down(fxl, 1);
  const int y = S.y0 + r;
  const double f0v = A.first ? c0 : S.f0n;
  // f^n of the next row of this strip (W may alias f^n: only rows this
  // wavefront owns are read ahead)
  if (!A.first && S.outcol && r + 1 < AR && y + 1 < S.ny) S.f0n = S.f0[(long long)(y + 1) * S.nx + S.xc];
  if (S.outcol && y < S.ny) {
    const long long node = (long long)y * S.nx + S.xc;
    const double adv = fma(S.pxi, fxl - fxr, S.pyi * (S.fyl - fyr));
    S.W[node] = fma(A.c, adv, fma(A.b, c0, A.a * f0v));
  }
  S.fyl = fyr;
}

template <bool PX, bool PY>
__device__ __forceinline__ void adv_strip(AdvStrip& S, const AdvArgs& A) {
  // rows y0 - 3 .. y0 + 2: triples of rows y0 - 2 .. y0 + 1, raw rows y0 .. y0 + 2
  double p[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    p[i] = S.fs[(long long)S.yr * S.nx + S.xc];
    if (++S.yr == S.ny) S.yr = 0;
  }
  S.ct[2] = tri_dir<PY>(p[0], p[1], p[2]);  // row y0 - 2
  S.ct[3] = tri_dir<PY>(p[1], p[2], p[3]);  // row y0 - 1
  S.ct[0] = tri_dir<PY>(p[2], p[3], p[4]);  // row y0
  S.ct[1] = tri_dir<PY>(p[3], p[4], p[5]);  // row y0 + 1
  S.rw[0] = p[3];
  S.rw[1] = p[4];
  S.rw[2] = p[5];
  S.nxr = S.fs[(long long)S.yr * S.nx + S.xc];  // row y0 + 3
  if (++S.yr == S.ny) S.yr = 0;
  S.f0n = 0.0;
  if (!A.first && S.outcol && S.y0 < S.ny) S.f0n = S.f0[(long long)S.y0 * S.nx + S.xc];
  // face between rows y0 - 1 and y0
  S.fyl = PY ? face3(S.ct[2].bp, S.ct[2].qp, S.ct[3].b0, S.ct[3].q0, S.ct[0].bm, S.ct[0].qm, S.eps4)
             : face3(S.ct[1].bp, S.ct[1].qp, S.ct[0].b0, S.ct[0].q0, S.ct[3].bm, S.ct[3].qm, S.eps4);
  for (int r = 0; r < AR; r += 4) {
    adv_row<PX, PY, 0>(S, A, r);
    adv_row<PX, PY, 1>(S, A, r + 1);
    adv_row<PX, PY, 2>(S, A, r + 2);
    adv_row<PX, PY, 3>(S, A, r + 3);
  }
}

__global__ __launch_bounds__(ANT) void adv_kernel(Dev D, AdvArgs A, const double* __restrict__ vel) {
  const int nsx = (D.nx + AW - 1) / AW, nsy = (D.ny + AR - 1) / AR;
  // contiguous ranges of strips per XCD: neighbouring strips share its L2
  const unsigned b = xcd_block(blockIdx.x, gridDim.x);
  const unsigned wave = (unsigned)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const unsigned strip = b * 4u + wave;
  const unsigned per_plane = (unsigned)nsx * (unsigned)nsy;
  const int plane = (int)(strip / per_plane);
  if (plane >= 2 * V) return;  // whole wavefront past the last strip
  const unsigned sp = strip - (unsigned)plane * per_plane;
  const int sy = (int)(sp / (unsigned)nsx), sx = (int)(sp - (unsigned)sy * (unsigned)nsx);
  const int v = plane % V, k = v / Q, l = v - k * Q;
  const double px = vel[k], py = vel[l];
  const long long base = (long long)plane * D.ntot;
  const int t = threadIdx.x & 63;
  AdvStrip S;
  S.fs = A.fs + base;
  S.f0 = A.f0 + base;
  S.W = A.W + base;
  S.nx = D.nx;
  S.ny = D.ny;
  S.y0 = sy * AR;
  const int x0 = sx * AW;
  S.xc = wrap(x0 - 3 + t, D.nx);
  S.yr = wrap(S.y0 - 3, D.ny);
  S.outcol = t >= 3 && t < 3 + AW && x0 + t - 3 < D.nx;
  S.pxi = px * D.inv_dx;
  S.pyi = py * D.inv_dx;
  S.eps4 = 4.0 * D.weno_eps;
  if (px > 0.0) {
    if (py > 0.0) adv_strip<true, true>(S, A);
    else adv_strip<true, false>(S, A);
  } else {
    if (py > 0.0) adv_strip<false, true>(S, A);
    else adv_strip<false, false>(S, A);
  }
}

// W = a f^n + b f^(s-1) without advection (term tests)
__global__ __launch_bounds__(256) void combine_kernel(Dev D, AdvArgs A) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= 2 * V * D.ntot) return;
  const double fv = A.fs[i];
  const double f0v = A.first ? fv : A.f0[i];
  A.W[i] = A.a * f0v + A.b * fv;
}

// ---------------------------------------------------------------------------
// velocity space: 16 nodes per wavefront
// ---------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned))));

// Raw buffer access: a uniform base (SGPRs) plus a 32-bit per-lane byte
// offset; an offset at or above num_records is out of range, so the store is
// dropped (lanes past the row end) without a branch.
constexpr int BUF_DWORD3 = 0x00020000;
constexpr unsigned BUF_RANGE = 0x7fffffffu;
constexpr unsigned BUF_OFF = 0xfffffff0u;  // out of range

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const double* base) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)BUF_RANGE, BUF_DWORD3);
}
__device__ __forceinline__ double bload(const double* base, unsigned vo) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(buf(base), vo, 0, 0));
}
__device__ __forceinline__ void bstore(double v, double* base, unsigned vo) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), buf(base), vo, 0, 0);
}

struct VelArgs {
  const double* fs;   // f^(s-1)
  double* W;          // in: advection part; out: f^(s) = W + c R(f^(s-1))
  const double* fld;  // [NF][ntot]
  double* mom;        // [6][ntot] moments of f^(s) (want_mom)
  double c;
  int want_mom;
};

// Lane (nd, g) = (lane & 15, lane >> 4) owns node x = x_w + nd and the velocity
// rows k = g + 4 j, j < 4, for every l: M[j][l] = f[k][l] (64 values).
// (Dp x I) M on the MFMA (v_mfma_f64_16x16x4: A operand element [i][c] from
// lane i + 16 c, B operand element [c][col] from lane col + 16 c, result
// element [4 j + c][col] in register j of lane col + 16 c): D = sum_b A_b B_b
// over b < 4 with A_b[i][c] = Dp[i][c + 4b] (lane holds Dp[nd][g + 4b]) and
// B_b[c][node] = M_node[c + 4b][l] (lane holds M[b][l]); D[k][node] comes back
// as D[g + 4j][nd] in register j, the rows the lane owns.  (I x Dp) M
// contracts over l, which the lane holds whole: VALU.
//
// Collision terms.  With xi = (xx, xy), th = |xi|^2 / T and the reduced
// forms of the Shakhov and J1 terms (F: factor 1, th - 4; G: factor T/2,
// th - 2), nu f^S + J1 = tf E P(xx, xy) with
//   P = nu + pre (xx A_x + xy A_y) + (th - th0)(xx S_x + xy S_y + C)
//       + 0.4 pre / T (xx^2 U_xx + xx xy (U_xy + U_yx) + xy^2 U_yy),
//   S_x = nu s q_x + 0.3 pre B_x,  S_y = nu s q_y + 0.3 pre B_y,
//   C = 0.2 pre div u,  pre = -b n chi.
// For a fixed row (xx) P is a cubic in xy: alpha + xy (beta + xy (gamma +
// delta xy)), set up once per row and pass.
//
// Occupancy: the unconstrained allocation takes about 300 registers (one
// wavefront per SIMD); capped at 256 a few values spill to scratch, and the
// second wavefront per SIMD hides more memory latency than the spills cost.
template <bool FRC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void vel_kernel(Dev D, VelArgs A, const double* __restrict__ vel,
                                                  const double* __restrict__ meq,
                                                  const double* __restrict__ dpm) {
  __shared__ double s_ey[4][Q][16];  // per wave: e_l(u_y) of its 16 nodes (node fastest: no bank conflicts)
  __shared__ double s_pc[4][4][4][64];  // per wave: row polynomial coefficients [al be ga ne][j][lane]
  __shared__ double s_aop[4][64];       // MFMA A operands Dp[nd][g + 4 b] (the same for every wave)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nd = lane & 15, g = lane >> 4;
  const int nseg = (D.nx + 63) >> 6;
  const int y = blockIdx.x / nseg, seg = blockIdx.x - y * nseg;
  const int x = seg * 64 + wave * 16 + nd;
  const bool valid = x < D.nx;
  const long long N = D.ntot;
  // lanes past the row end work on the last node and store nothing
  const long long node = (long long)y * D.nx + (valid ? x : D.nx - 1);
  const bool j0 = (D.term_mask & EVLB_TERM_J0) != 0;
  const bool j1 = (D.term_mask & EVLB_TERM_J1) != 0;

  // unit-density Hermite equilibria: e_k(u_x) of the own rows in registers,
  // e_l(u_y) shared by the four lanes of a node through LDS
  double ex[4] = {0.0, 0.0, 0.0, 0.0};
  {
    const double ux = A.fld[F_UX * N + node], uy = A.fld[F_UY * N + node], T = A.fld[F_T * N + node];
    double a[Q];
    hermite_coeffs(uy, T, a);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < Q; ++m) s += meq[(g + 4 * i) * Q + m] * a[m];
      s_ey[wave][g + 4 * i][nd] = s;
    }
    hermite_coeffs(ux, T, a);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < Q; ++m) s += meq[k * Q + m] * a[m];
      if ((k & 3) == g) ex[k >> 2] = s;
    }
  }
  double pkv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    pkv[j] = vel[g + 4 * j];
    if (wave == 0) s_aop[j][lane] = dpm[nd * Q + g + 4 * j];
  }
  __syncthreads();
  const double* eyv = &s_ey[wave][0][nd];  // e_l at eyv[16 l]

  // per-lane byte offset of (row g, node) from a plane base; < 2^31 by the
  // node-count limit of the 2D path
  const unsigned vo = (unsigned)(((long long)g * Q * N + node) * 8);
  const unsigned vs = valid ? vo : BUF_OFF;
  Raw m{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
  for (int d = 0; d < 2; ++d) {
    // Opaque copies: what the F and G passes share (Dp rows, plane bases,
    // node fields) is recomputed in each pass instead of being hoisted out of
    // the loop and held live across both.
    long long Nd = N;
    int z = 0;  // an opaque zero keeps the pointers' address space and uniformity
    asm volatile("" : "+s"(Nd), "+s"(z));
    const double* dp = dpm + z;
    const double* vl = vel + z;
    const double* fd = A.fld + z;
    const double* fsd = A.fs + (long long)d * V * Nd;
    double* wd = A.W + (long long)d * V * Nd;
    // plane of own row j (k = g + 4 j) and column l, relative to row g
#define PLANE(base, j, l) ((base) + (long long)(4 * (j) * Q + (l)) * Nd)
    double M[4][Q];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int l = 0; l < Q; ++l) M[j][l] = bload(PLANE(fsd, j, l), vo);
    // W of column l is loaded PF columns ahead of its use
    constexpr int PF = 1;
    double wb[PF][4];
#pragma unroll
    for (int p = 0; p < PF; ++p)
#pragma unroll
      for (int j = 0; j < 4; ++j) wb[p][j] = bload(PLANE(wd, j, p), vo);

    // row polynomials of the collision terms
    // the row polynomials live in LDS (registers are the occupancy limit)
    double(*pc)[4][64] = s_pc[wave];
    double de, nu, Fx, Fy, uy;
    {
      const double n = fd[F_N * Nd + node], ux = fd[F_UX * Nd + node], T = fd[F_T * Nd + node];
      uy = fd[F_UY * Nd + node];
      const double nu0 = fd[F_NU * Nd + node];
      nu = j0 ? nu0 : 0.0;
      const double pre = j1 ? fd[F_PRE * Nd + node] : 0.0;
      Fx = fd[F_FX * Nd + node];
      Fy = fd[F_FY * Nd + node];
      const double invT = 1.0 / T;
      const double tf = d == 0 ? 1.0 : 0.5 * T;
      const double th0 = d == 0 ? 4.0 : 2.0;
      const double uxx = fd[F_UXX * Nd + node], uyy = fd[F_UYY * Nd + node];
      const double Sx = nu * fd[F_SQX * Nd + node] + 0.3 * pre * fd[F_BX * Nd + node];
      const double Sy = nu * fd[F_SQY * Nd + node] + 0.3 * pre * fd[F_BY * Nd + node];
      const double C = 0.2 * pre * (uxx + uyy);
      const double W4 = 0.4 * pre * invT;
      const double pAx = pre * fd[F_AX * Nd + node], pAy = pre * fd[F_AY * Nd + node];
      const double Uc = W4 * (fd[F_UXY * Nd + node] + fd[F_UYX * Nd + node]);
      de = invT * Sy;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double xx = pkv[j] - ux;
        const double t0 = xx * xx * invT - th0;
        const double r = xx * Sx + C;
        pc[0][j][lane] = nu + pAx * xx + t0 * r + W4 * uxx * xx * xx;
        pc[1][j][lane] = pAy + t0 * Sy + Uc * xx;
        pc[2][j][lane] = invT * r + W4 * uyy;
        pc[3][j][lane] = (j0 || j1) ? tf * n * ex[j] : 0.0;
      }
    }
    // velocity sums of the new state: 1, p_x, p_y (both passes), p_x^2,
    // p_x p_y, p_y^2, p_x |p|^2, p_y |p|^2 (used for F only)
    double S[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // fully unrolled: every M[j][l] index is static, M stays in registers
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      double wcur[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) wcur[j] = wb[l % PF][j];
      if (l + PF < Q) {
#pragma unroll
        for (int j = 0; j < 4; ++j) wb[l % PF][j] = bload(PLANE(wd, j, l + PF), vo);
      }
      // an opaque copy of the lane index per column keeps the MFMA operands
      // and polynomial coefficients in LDS instead of being hoisted back into
      // registers
      int pli = lane;
      asm volatile("" : "+v"(pli));
      dbl4 acc = {0.0, 0.0, 0.0, 0.0};
      if (FRC) {
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(s_aop[0][pli], M[0][l], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(s_aop[1][pli], M[1][l], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(s_aop[2][pli], M[2][l], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(s_aop[3][pli], M[3][l], acc, 0, 0, 0);
      }
      const double pl = vl[l];
      const double xy = pl - uy;
      const double eyl = eyv[16 * l];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double R = pc[3][j][pli] * eyl * (pc[0][j][pli] + xy * (pc[1][j][pli] + xy * (pc[2][j][pli] + de * xy))) -
                   nu * M[j][l];
        if (FRC) {
          double d0 = 0.0, d1 = 0.0;
#pragma unroll
          for (int l2 = 0; l2 < Q; l2 += 2) {
            d0 += dp[l * Q + l2] * M[j][l2];
            d1 += dp[l * Q + l2 + 1] * M[j][l2 + 1];
          }
          R -= Fx * acc[j] + Fy * (d0 + d1);
        }
        const double out = wcur[j] + A.c * R;
        bstore(out, PLANE(wd, j, l), vs);
        const double pk = pkv[j];
        const double a1 = pk * out, a2 = pl * out;
        const double p2 = pk * pk + pl * pl;
        S[0] += out;
        S[1] += a1;
        S[2] += a2;
        S[3] += pk * a1;
        S[4] += pl * a1;
        S[5] += pl * a2;
        S[6] += p2 * a1;
        S[7] += p2 * a2;
      }
      // one column at a time: keeps later columns' work from being hoisted
      __builtin_amdgcn_sched_barrier(0);
    }
#undef PLANE
    if (d == 0) {
      m.n = S[0]; m.jx = S[1]; m.jy = S[2]; m.pxx = S[3]; m.pxy = S[4]; m.pyy = S[5]; m.rx = S[6]; m.ry = S[7];
    } else {
      m.g0 = S[0]; m.hx = S[1]; m.hy = S[2];
    }
  }
  if (!A.want_mom) return;
  // the four lanes of a node (g = 0..3) hold partial sums over their rows
#define EVLB2D_REDUCE(v) v += __shfl_xor(v, 16); v += __shfl_xor(v, 32)
  EVLB2D_REDUCE(m.n); EVLB2D_REDUCE(m.jx); EVLB2D_REDUCE(m.jy); EVLB2D_REDUCE(m.pxx);
  EVLB2D_REDUCE(m.pxy); EVLB2D_REDUCE(m.pyy); EVLB2D_REDUCE(m.rx); EVLB2D_REDUCE(m.ry);
  EVLB2D_REDUCE(m.g0); EVLB2D_REDUCE(m.hx); EVLB2D_REDUCE(m.hy);
#undef EVLB2D_REDUCE
  if (valid && g == 0) finish_moments(m, A.mom, N, node, D.status, D.T_iso);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t tab_d, tab_i, f1, f2, mom, fld, status, total;
  int navg, npair, halo;
};

bool is_integer_multiple(double a, double dx, int* m) {
  const double r = a / dx;
  const long long k = llround(r);
  if (k <= 0 || std::fabs(r - (double)k) > 1e-9 * r) return false;
  *m = (int)k;
  return true;
}

Layout make_layout(const evlb_params* p, const evlb::DiscTables& t) {
  Layout L{};
  const long long N = (long long)p->nx[0] * p->ny;
  L.navg = (int)t.avg_w.size();
  L.npair = (int)t.pair_cx.size();
  L.halo = t.pair_reach > t.avg_reach + 2 ? t.pair_reach : t.avg_reach + 2;
  size_t off = 0;
  L.tab_d = off;
  off += align256(sizeof(double) * (size_t)(Q + 2 * Q * Q + L.navg + 2 * (L.npair > 0 ? L.npair : 1)));
  L.tab_i = off;
  off += align256(sizeof(int) * (size_t)(L.navg + (L.npair > 0 ? L.npair : 1)));
  const size_t fbytes = align256(sizeof(double) * 2 * (size_t)V * (size_t)N);
  L.f1 = off; off += fbytes;
  L.f2 = off; off += fbytes;
  L.mom = off; off += align256(sizeof(double) * 6 * (size_t)N);
  L.fld = off; off += align256(sizeof(double) * NF * (size_t)N);
  L.status = off; off += 256;
  L.total = off;
  return L;
}

void disc_tables(const evlb_params* p, evlb::DiscTables& t) {
  evlb::build_disc_tables(p->dx, p->sigma, p->phi_sigma, p->r_cut, p->force_model == EVLB_FORCE_EV1, t);
}

size_t fields_lds_bytes(int halo) {
  return sizeof(double) * ((size_t)(FTX + 2 * halo) * (FTY + 2 * halo) + 5 * (size_t)GX * GY);
}

}  // namespace

struct Ctx {
  evlb_params p;
  int nx, ny;
  long long N;
  Layout L;
  Dev dev;
  char* ws;
  const double *vel, *meq, *dpm, *avg_w, *pair_cx, *pair_cy;
  const int *avg_ofs, *pair_ofs;
  std::vector<double> hvel;
};

int validate(const evlb_params* p) {
  if (!p || p->dim != 2) return EVLB_EINVAL;
  if (p->n_sys != 1 || !p->nx) return EVLB_EINVAL;
  if (p->nx[0] < 8 || p->ny < 8) return EVLB_EINVAL;
  const long long N = (long long)p->nx[0] * p->ny;
  if (N > (1ll << 22)) return EVLB_EINVAL;  // 32-bit buffer offsets of the velocity kernel
  if (p->q != Q) return EVLB_EUNSUPPORTED;
  if (!(p->dx > 0) || !(p->dt > 0) || !std::isfinite(p->dx) || !std::isfinite(p->dt)) return EVLB_EINVAL;
  if (!(p->sigma > 0) || !std::isfinite(p->sigma) || !(p->phi_sigma >= 0) || !std::isfinite(p->phi_sigma))
    return EVLB_EINVAL;
  if (p->force_model < 0 || p->force_model > 2) return EVLB_EINVAL;
  if (p->force_model == EVLB_FORCE_EV2) return EVLB_EUNSUPPORTED;
  if (p->gamma != 6.0) return EVLB_EUNSUPPORTED;  // the z-integrated kernel is tabulated for gamma = 6
  if (p->term_mask & ~EVLB_TERM_ALL) return EVLB_EINVAL;
  if (!(p->weno_eps > 0) || !std::isfinite(p->g_ext)) return EVLB_EINVAL;
  if (p->exec_mode < 0 || p->exec_mode > 2) return EVLB_EINVAL;
  if (p->exec_mode == EVLB_EXEC_PERSISTENT) return EVLB_EUNSUPPORTED;
  if (p->tile_nodes != 0) return EVLB_EINVAL;
  if (p->adjoint != 0 && p->adjoint != 1) return EVLB_EINVAL;
  if (p->adjoint) return EVLB_EUNSUPPORTED;
  if (!(p->T_iso >= 0.0) || !std::isfinite(p->T_iso)) return EVLB_EINVAL;
  if ((int)std::ceil(p->sigma / p->dx) + 2 > HMAX) return EVLB_EINVAL;
  if (p->force_model == EVLB_FORCE_EV1) {
    int mf;
    if (!is_integer_multiple(p->r_cut, p->dx, &mf) || mf > HMAX) return EVLB_EINVAL;
  }
  // WENO-5 + TVD-RK3 along two axes: dt (|p_x| + |p_y|)_max / dx <= 1
  std::vector<double> v, w;
  evlb::gauss_hermite_nodes(Q, v, w);
  if (p->dt * 2.0 * v.back() / p->dx > 1.0) return EVLB_ECFL;
  return EVLB_OK;
}

size_t workspace_bytes(const evlb_params* p) {
  if (validate(p) != EVLB_OK) return 0;
  evlb::DiscTables t;
  disc_tables(p, t);
  return make_layout(p, t).total;
}

int init(const evlb_params* p, char* ws, size_t bytes, hipStream_t st, Ctx** out) {
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  evlb::DiscTables t;
  disc_tables(p, t);
  const Layout L = make_layout(p, t);
  if (!ws || bytes < L.total || ((uintptr_t)ws & 255)) return EVLB_EWORKSPACE;
  Ctx* c = new (std::nothrow) Ctx();
  if (!c) return EVLB_EINVAL;
  c->p = *p;
  c->nx = p->nx[0];
  c->ny = p->ny;
  c->N = (long long)c->nx * c->ny;
  c->L = L;
  c->ws = ws;
  evlb::TableParams tp{Q, p->dx, p->sigma, p->phi_sigma, p->gamma, p->r_cut};
  evlb::HostTables ht;
  evlb::build_tables(tp, ht);
  c->hvel = ht.vel;
  const int PX = FTX + 2 * L.halo;
  std::vector<double> hd;
  hd.insert(hd.end(), ht.vel.begin(), ht.vel.end());
  hd.insert(hd.end(), ht.meq.begin(), ht.meq.end());
  hd.insert(hd.end(), ht.dpm.begin(), ht.dpm.end());
  hd.insert(hd.end(), t.avg_w.begin(), t.avg_w.end());
  const size_t o_cx = hd.size();
  hd.insert(hd.end(), t.pair_cx.begin(), t.pair_cx.end());
  if (t.pair_cx.empty()) hd.push_back(0.0);
  const size_t o_cy = hd.size();
  hd.insert(hd.end(), t.pair_cy.begin(), t.pair_cy.end());
  if (t.pair_cy.empty()) hd.push_back(0.0);
  std::vector<int> hi;
  for (size_t i = 0; i < t.avg_w.size(); ++i) hi.push_back(t.avg_dj[i] * PX + t.avg_di[i]);
  const size_t o_po = hi.size();
  for (size_t i = 0; i < t.pair_cx.size(); ++i) hi.push_back(t.pair_dj[i] * PX + t.pair_di[i]);
  if (t.pair_cx.empty()) hi.push_back(0);
  double* tabd = (double*)(ws + L.tab_d);
  int* tabi = (int*)(ws + L.tab_i);
  // ordered on the caller's stream, which is synchronised before the host
  // vectors go out of scope
  if (hipMemcpyAsync(tabd, hd.data(), hd.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(tabi, hi.data(), hi.size() * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemsetAsync(ws + L.status, 0, 256, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    delete c;
    return EVLB_EHIP;
  }
  c->vel = tabd;
  c->meq = tabd + Q;
  c->dpm = tabd + Q + Q * Q;
  c->avg_w = tabd + Q + 2 * Q * Q;
  c->pair_cx = tabd + o_cx;
  c->pair_cy = tabd + o_cy;
  c->avg_ofs = tabi;
  c->pair_ofs = tabi + o_po;
  Dev& d = c->dev;
  d.nx = c->nx;
  d.ny = c->ny;
  d.ntot = c->N;
  d.inv_dx = 1.0 / p->dx;
  const double sg = p->sigma;
  d.b = 2.0 * M_PI * sg * sg * sg / 3.0;
  d.eta_c = M_PI * sg * sg * sg / 6.0;
  d.mu0c = 5.0 / (16.0 * sg * sg * std::sqrt(M_PI));
  d.weno_eps = p->weno_eps;
  d.g_ext = p->g_ext;
  d.force_model = p->force_model;
  d.term_mask = p->term_mask;
  d.T_iso = p->T_iso;
  d.navg = L.navg;
  d.npair = p->force_model == EVLB_FORCE_EV1 ? L.npair : 0;
  d.halo = L.halo;
  d.status = (int*)(ws + L.status);
  *out = c;
  return EVLB_OK;
}

void destroy(Ctx* c) { delete c; }
long long node_count(const Ctx* c) { return c->N; }
const std::vector<double>& velocities(const Ctx* c) { return c->hvel; }
int* status_word(const Ctx* c) { return c->dev.status; }

namespace {

int launched() { return hipGetLastError() == hipSuccess ? EVLB_OK : EVLB_EHIP; }

int launch_moments(Ctx* c, const double* f, double* out6, hipStream_t st, int stage_input = 1) {
  const unsigned nb = (unsigned)((c->N + 255) / 256);
  hipLaunchKernelGGL(moments_kernel, dim3(nb), dim3(256), 0, st, c->dev, f, out6, c->vel, stage_input);
  return launched();
}

int launch_fields(Ctx* c, hipStream_t st) {
  const dim3 grid((c->nx + FTX - 1) / FTX, (c->ny + FTY - 1) / FTY);
  hipLaunchKernelGGL(fields_kernel, grid, dim3(FNT), fields_lds_bytes(c->L.halo), st, c->dev,
                     (const double*)(c->ws + c->L.mom), (double*)(c->ws + c->L.fld), c->avg_ofs, c->avg_w,
                     c->pair_ofs, c->pair_cx, c->pair_cy);
  return launched();
}

int launch_adv(Ctx* c, const AdvArgs& A, hipStream_t st) {
  if (!(c->dev.term_mask & EVLB_TERM_ADV)) {
    const long long nb = (2 * V * c->N + 255) / 256;
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)nb), dim3(256), 0, st, c->dev, A);
    return launched();
  }
  const long long strips = (long long)((c->nx + AW - 1) / AW) * ((c->ny + AR - 1) / AR) * 2 * V;
  const long long nb = (strips + 3) / 4;
  hipLaunchKernelGGL(adv_kernel, dim3((unsigned)nb), dim3(ANT), 0, st, c->dev, A, c->vel);
  return launched();
}

int launch_vel(Ctx* c, const VelArgs& A, hipStream_t st) {
  const unsigned nb = (unsigned)(((c->nx + 63) / 64) * c->ny);
  if (c->dev.term_mask & EVLB_TERM_FORCE)
    hipLaunchKernelGGL(vel_kernel<true>, dim3(nb), dim3(256), 0, st, c->dev, A, c->vel, c->meq, c->dpm);
  else
    hipLaunchKernelGGL(vel_kernel<false>, dim3(nb), dim3(256), 0, st, c->dev, A, c->vel, c->meq, c->dpm);
  return launched();
}

// one evaluation: fields of the moments in the workspace, then
// W = a f0 + b fs + c Adv(fs) and out = W + c R(fs)
int stage(Ctx* c, const double* fs, const double* f0, double* W, double a, double b, double cc, int first,
          int want_mom, hipStream_t st) {
  int rc = launch_fields(c, st);
  if (rc) return rc;
  AdvArgs A{fs, f0, W, a, b, cc, first};
  rc = launch_adv(c, A, st);
  if (rc) return rc;
  VelArgs B{fs, W, (const double*)(c->ws + c->L.fld), (double*)(c->ws + c->L.mom), cc, want_mom};
  return launch_vel(c, B, st);
}

}  // namespace

int set_equilibrium(Ctx* c, const double* n, const double* u, const double* T, double* f, hipStream_t st) {
  const unsigned nb = (unsigned)((c->N + 255) / 256);
  hipLaunchKernelGGL(equilibrium_kernel, dim3(nb), dim3(256), 0, st, c->dev, n, u, T, f, c->meq);
  return launched();
}

int step(Ctx* c, double* f, int nsteps, hipStream_t st) {
  static const double RKA[3] = {0.0, 0.75, 1.0 / 3.0};
  static const double RKB[3] = {1.0, 0.25, 2.0 / 3.0};
  double* f1 = (double*)(c->ws + c->L.f1);
  double* f2 = (double*)(c->ws + c->L.f2);
  int rc = launch_moments(c, f, (double*)(c->ws + c->L.mom), st);
  if (rc) return rc;
  const double dt = c->p.dt;
  for (int n = 0; n < nsteps; ++n) {
    for (int s = 0; s < 3; ++s) {
      const double* fs = s == 0 ? f : (s == 1 ? f1 : f2);
      double* W = s == 0 ? f1 : (s == 1 ? f2 : f);  // stage 3 overwrites f^n in place, element by element
      rc = stage(c, fs, f, W, RKA[s], RKB[s], RKB[s] * dt, s == 0, 1, st);
      if (rc) return rc;
    }
  }
  return EVLB_OK;
}

int rhs(Ctx* c, const double* f, double* L, hipStream_t st) {
  int rc = launch_moments(c, f, (double*)(c->ws + c->L.mom), st);
  if (rc) return rc;
  return stage(c, f, f, L, 0.0, 0.0, 1.0, 1, 0, st);
}

int moments(Ctx* c, const double* f, double* n, double* u, double* T, double* q, hipStream_t st) {
  double* m = (double*)(c->ws + c->L.mom);
  int rc = launch_moments(c, f, m, st, 0);
  if (rc) return rc;
  const size_t nb = sizeof(double) * (size_t)c->N;
  if (hipMemcpyAsync(n, m, nb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(u, m + c->N, 2 * nb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(T, m + 3 * c->N, nb, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return EVLB_EHIP;
  if (q && hipMemcpyAsync(q, m + 4 * c->N, 2 * nb, hipMemcpyDeviceToDevice, st) != hipSuccess) return EVLB_EHIP;
  return EVLB_OK;
}

}  // namespace evlb2d
