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
// TVD-RK3 stage is two kernels:
//   fields_kernel  32 x 8 nodes per workgroup, density tile with the force
//                  radius as halo in LDS: n, u, T, q from the raw velocity
//                  sums, disc-averaged density, contact value (eq:carnstar),
//                  force (antisymmetric cell pairs), transport
//                  (eq:viscosity, eq:tau, eq:prandtl), 4th-order central
//                  gradients of X = n^2 chi T, T and u along x and y.
//   fused_kernel   one workgroup per strip of 8 columns, distribution and
//                  segment of rows, all 256 velocities: WENO-5 faces along y
//                  from a ring of rows in registers and along x from the row
//                  in LDS, (Dp x I) and (I x Dp) on the f64 MFMA, Hermite
//                  equilibrium, Shakhov and J1 terms, f^(s) = a f^n +
//                  b f^(s-1) + c L(f^(s-1)), and the raw velocity sums of
//                  f^(s) for the next stage's fields.
#include "evlb2d.h"

#include <cmath>
#include <cstddef>
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
// moments of a state (first stage of a step, evlb_moments).  State layout:
// distribution d, node i, velocity (k, l) at ((d ntot + i) V + Q k + l): the
// 2 KiB of a node's distribution are contiguous, so one wavefront reads a
// node with lane L taking the velocities L + 64 m.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ Raw velocity_sums(const Dev& D, const double* __restrict__ f,
                                             const double* __restrict__ vel, long long node, int lane) {
  const double* F = f + node * V;
  const double* G = f + (D.ntot + node) * V;
  double a[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const double pl = vel[lane & 15];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int v = lane + 64 * m;
    const double pk = vel[v >> 4];
    const double Fv = F[v], Gv = G[v];
    const double p2 = pk * pk + pl * pl;
    a[0] += Fv;
    a[1] += pk * Fv;
    a[2] += pl * Fv;
    a[3] += pk * pk * Fv;
    a[4] += pk * pl * Fv;
    a[5] += pl * pl * Fv;
    a[6] += pk * p2 * Fv;
    a[7] += pl * p2 * Fv;
    a[8] += Gv;
    a[9] += pk * Gv;
    a[10] += pl * Gv;
  }
#pragma unroll
  for (int i = 0; i < 11; ++i) a[i] = wave_sum(a[i]);
  return Raw{a[0], a[1], a[2], a[3], a[4], a[5], a[6], a[7], a[8], a[9], a[10]};
}

// n, u, T, q of a state (evlb_moments): T is the moment temperature; one
// wavefront per node
__global__ __launch_bounds__(256) void moments_kernel(Dev D, const double* __restrict__ f, double* __restrict__ out6,
                                                      const double* __restrict__ vel) {
  const long long node = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (node >= D.ntot) return;
  const Raw m = velocity_sums(D, f, vel, node, threadIdx.x & 63);
  if ((threadIdx.x & 63) == 0) finish_moments(m, out6, D.ntot, node, D.status, 0.0);
}

// raw velocity sums [11][ntot] of a state, the input of a stage's fields
__global__ __launch_bounds__(256) void raw_sums_kernel(Dev D, const double* __restrict__ f, double* __restrict__ raw,
                                                       const double* __restrict__ vel) {
  const long long node = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (node >= D.ntot) return;
  const Raw m = velocity_sums(D, f, vel, node, threadIdx.x & 63);
  const long long N = D.ntot;
  const double v[11] = {m.n, m.jx, m.jy, m.pxx, m.pxy, m.pyy, m.rx, m.ry, m.g0, m.hx, m.hy};
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 11; ++i)
    if (lane == i) raw[i * N + node] = v[i];
}

// Hermite equilibrium of one velocity component at unit density:
// a_0 = 1, a_1 = u, a_{m+1} = u a_m + m (T - 1) a_{m-1};  e_k = sum_m meq[k][m] a_m.
__device__ __forceinline__ void hermite_coeffs(double u, double T, double* a) {
  a[0] = 1.0;
  a[1] = u;
#pragma unroll
  for (int m = 1; m < Q - 1; ++m) a[m + 1] = u * a[m] + (double)m * (T - 1.0) * a[m - 1];
}

// one wavefront per node: lane L writes the velocities L + 64 m, i.e. the
// rows k = L / 16 + 4 m of column l = L % 16
__global__ __launch_bounds__(256) void equilibrium_kernel(Dev D, const double* __restrict__ n_in,
                                                          const double* __restrict__ u_in,
                                                          const double* __restrict__ T_in, double* __restrict__ f,
                                                          const double* __restrict__ meq) {
  const long long node = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (node >= D.ntot) return;
  const int lane = threadIdx.x & 63, l = lane & 15;
  const long long N = D.ntot;
  const double n = n_in[node], ux = u_in[node], uy = u_in[N + node], T = T_in[node];
  double ax[Q], ay[Q];
  hermite_coeffs(ux, T, ax);
  hermite_coeffs(uy, T, ay);
  double ey = 0.0;
#pragma unroll
  for (int m = 0; m < Q; ++m) ey += meq[l * Q + m] * ay[m];
  double* F = f + node * V;
  double* G = f + (N + node) * V;
#pragma unroll
  for (int mm = 0; mm < 4; ++mm) {
    const int k = (lane >> 4) + 4 * mm;
    double ex = 0.0;
#pragma unroll
    for (int m = 0; m < Q; ++m) ex += meq[k * Q + m] * ax[m];
    const double E = n * ex * ey;
    F[lane + 64 * mm] = E;
    G[lane + 64 * mm] = 0.5 * T * E;
  }
}

// ---------------------------------------------------------------------------
// node fields
// ---------------------------------------------------------------------------
constexpr int FTX = 32, FTY = 8, FNT = FTX * FTY;
constexpr int GX = FTX + 4, GY = FTY + 4;  // tile +-2 (gradient stencil)

// u_x, u_y and T from the raw sums of a node (3/2 n T = sum |xi|^2/2 F + G);
// an isothermal run sees its fixed temperature
__device__ __forceinline__ void flow_of(const double* __restrict__ raw, long long N, long long node, double T_iso,
                                        double& ux, double& uy, double& T) {
  const double n = raw[node];
  ux = raw[N + node] / n;
  uy = raw[2 * N + node] / n;
  const double e = 0.5 * (raw[3 * N + node] + raw[5 * N + node]) + raw[8 * N + node];
  T = T_iso > 0.0 ? T_iso : (2.0 / 3.0) * (e - 0.5 * n * (ux * ux + uy * uy)) / n;
}

__global__ __launch_bounds__(FNT) void fields_kernel(Dev D, const double* __restrict__ raw, double* __restrict__ fld,
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
    sn[i] = raw[(long long)wrap(y0 - H + r, D.ny) * D.nx + wrap(x0 - H + c, D.nx)];
  }
  for (int i = tid; i < GX * GY; i += FNT) {
    const int r = i / GX, c = i - r * GX;
    const long long node = (long long)wrap(y0 - 2 + r, D.ny) * D.nx + wrap(x0 - 2 + c, D.nx);
    flow_of(raw, N, node, D.T_iso, sux[i], suy[i], sT[i]);
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
  // heat flux and the status check of this node from its raw sums
  Raw m;
  m.n = n;
  m.jx = raw[N + node];
  m.jy = raw[2 * N + node];
  m.pxx = raw[3 * N + node];
  m.pxy = raw[4 * N + node];
  m.pyy = raw[5 * N + node];
  m.rx = raw[6 * N + node];
  m.ry = raw[7 * N + node];
  m.g0 = raw[8 * N + node];
  m.hx = raw[9 * N + node];
  m.hy = raw[10 * N + node];
  double q6[6];
  finish_moments(m, q6, 1, 0, D.status, D.T_iso);
  const double vals[NF] = {n, ux, uy, T, s * q6[4], s * q6[5], nu, -bn * chi, Fx, Fy,
                           Ax, Ay, Bx, By, Uxx, Uxy, Uyx, Uyy};
#pragma unroll
  for (int i = 0; i < NF; ++i) fld[i * N + node] = vals[i];
}

// ---------------------------------------------------------------------------
// fused stage: one workgroup of sixteen wavefronts owns a strip of 8
// columns, one distribution (F or G) and all 256 velocities, and marches
// down a segment of rows
// ---------------------------------------------------------------------------
// Thread (wavefront w, lane L): column c = L & 7 of the strip and r = L >> 3;
// it holds the two velocities (k, l) = (w, r) and (w, r + 8).  In the
// node-major state a wavefront's 16 velocities of a node are one 128-byte
// line, read as two halves by consecutive loads.  Every wavefront sees one
// sign of p_k (k < 8: p_k < 0) and every register slot one sign of p_l, so
// both upwind choices are uniform.
//
// One barrier per row.  Iteration y is
//  pre(y)   (each wavefront on its own 16 velocities, no data of another
//           wavefront): the row to LDS with three halo columns each side;
//           WENO-5 faces along y from a ring of five rows per velocity in
//           registers; WENO-5 faces along x from the LDS row (each lane the
//           face on its left, the one on its right from the next lane by
//           DPP); (I x Dp) f on the f64 MFMA, every other row for that row
//           and the one before it (whose term goes into acc(y - 1)); the
//           Shakhov + J1 collision terms as a polynomial in xi_x and xi_y per
//           node; everything but the (Dp x I) f term and the strip-edge face
//           folded into acc(y).
//  barrier
//  post(y)  the work that reads other wavefronts' rows or writes what they
//           read: f^(s) of row y - 1 from acc(y - 1), the (Dp x I) f term and
//           the strip-edge face of row y - 1, its store and its per-wavefront
//           terms of the raw velocity sums (a weight matrix times the row's
//           16 x 8 values on the MFMA);
//           wavefront 0 the raw velocity sums of row y - 2, 1 the Hermite
//           coefficients a_m(u, T) of row y + 3, 2 the expansions e_k(u_x),
//           e_l(u_y) of row y + 2 (one MFMA chain over 8 nodes x 2 axes), 3
//           the per-node collision coefficients of row y + 3, 4 - 7 the
//           strip-edge faces of row y, 8 - 15 (Dp x I) f of row y
//           (v_mfma_f64_16x16x4 takes B element [c][col] from lane col + 16 c
//           and returns row 4 j + c, column col in register j of that lane;
//           col = (column, l parity)).
// What one wavefront writes and another reads crosses exactly one barrier,
// and every such buffer is double (quadruple for the collision
// coefficients, read a full iteration after they are written), so that a
// wavefront one half-iteration ahead never overwrites what a slower one
// still reads.  The ring's next row, f^n and the halo columns of the next
// row and the node fields of row y + 4 are in flight across an iteration.
constexpr int SW = 8;            // columns per strip
constexpr int SNW = 16;          // wavefronts per workgroup
constexpr int SNT = 64 * SNW;    // threads per workgroup
constexpr int NRAW = 11;         // raw velocity sums per node: 8 of F, 3 of G
// LDS strides (doubles).  A lane (c, r) reads plane r + 8 j at column c + i:
// a plane stride of 8 (mod 16) puts the 16 lanes of one LDS pass, and of 32
// lanes, on distinct banks.
constexpr int TS = 24;                 // T: columns x0 - 3 .. x0 + 10 at 0 .. 13, (I x Dp) f at 14 .. 21,
                                       // the strip-edge face of rows of parity 0 / 1 at 22 / 23
constexpr int FIS = 16 * SW + 3 * 16;  // FI per k: 16 l x 8 interior columns, then 16 l x 3 right halo columns
// per-node coefficients of the collision terms: the row polynomial
//   nu f^S + J1 = tf n e_k e_l (P0 + xi_y (P1 + xi_y (P2 + P3 xi_y)))
// with P0 = c0 + xi_x (c1 + xi_x (c2 + c3 xi_x)), P1 = d0 + xi_x (d1 + d2 xi_x),
// P2 = e0 + c3 xi_x, P3 = d2 (a rearrangement of the reduced Shakhov and J1
// terms), plus u_x, u_y, tf n, nu, F_x, F_y
enum { CF_C0, CF_C1, CF_C2, CF_C3, CF_D0, CF_D1, CF_D2, CF_E0, CF_UX, CF_UY, CF_TFN, CF_NU, CF_FX, CF_FY, NCF };

struct FusedArgs {
  const double* fs;   // f^(s-1)
  const double* f0;   // f^n (not read when first)
  double* out;        // f^(s); may alias f0 (read pointwise before the write)
  const double* fld;  // node fields [NF][ntot]
  double* raw;        // raw velocity sums of f^(s) [NRAW][ntot] (want_mom)
  double a, b, c;     // f^(s) = a f^n + b f^(s-1) + c L(f^(s-1))
  int first, want_mom;
  int nstrip, seglen;
};

struct FusedSmem {
  double T[V * TS];             // wavefront w's row, velocity (w, l) at 16 w + l (its own)
  double FI[2][Q][FIS];         // row y: [k][8 l + (c ^ ((l >> 1) & 7))] interior (the swizzle spreads a
                                // column of 16 l over the banks), [k][128 + 3 l + h] columns x0 + 8 + h
  double DX[2][Q][16 * SW];     // (Dp x I) f^(s-1) of row y: [k][8 (l ^ 2 (k & 1)) + c] (the swizzle
                                // puts the MFMA result rows k and k + 1 on distinct banks)
  double AH[2][Q][16];          // Hermite coefficients a_m(u, T) of a row, column (node, axis)
  double EK[2][2][Q][SW];       // unit-density expansions e_k(u_x) (axis 0), e_l(u_y) (axis 1)
  double CF[4][NCF][SW];        // per-node coefficients of the collision row polynomial
  double fl[2][NF][SW];         // node fields of a row
  double mred[2][SNW][8][SW];   // per-wavefront terms of the raw velocity sums of a row (fixed k)
  double aop[4][64];            // MFMA A operands Dp[i][c + 4 b] at lane i + 16 c
  double eop[4][64];            // MFMA A operands meq[i][c + 4 b] at lane i + 16 c
  double vel[Q];
};
static_assert(sizeof(FusedSmem) <= 160 * 1024, "fused stage LDS exceeds 160 KiB");

// WENO-5 (Jiang & Shu) value at a face from the five values v0 .. v4 ordered
// from the upwind side (v2 is the node upwind of the face), written in the
// first differences e_m = v_(m+1) - v_m.  The candidates less v2 are g0 =
// (5 e1 - 2 e0) / 6, 6 g1 = e1 + 2 e2, 3 g2 = 2 e2 - e3 / 2; the
// smoothness 12 beta_r = 13 a_r^2 + 3 b_r^2 expands in the squares and
// neighbour products of the differences to 16 e0^2 - 44 e0 e1 + 40 e1^2,
// 16 e1^2 - 20 e1 e2 + 16 e2^2 and 40 e2^2 - 44 e2 e3 + 16 e3^2.  The weights
// d_r / (eps + beta_r)^2 normalised: with t_r = (12 eps + 12 beta_r)^2 and
// 10 d = (1, 6, 3) the value is v2 + (t1 t2 g0 + 6 t0 t2 g1 + 3 t0 t1 g2) /
// (t1 t2 + 6 t0 t2 + 3 t0 t1) (every common factor cancels).  The division
// goes through a hardware reciprocal refined by two Newton steps.
__device__ __forceinline__ double weno5(double v0, double v1, double v2, double v3, double v4, double eps12) {
  const double e0 = v1 - v0, e1 = v2 - v1, e2 = v3 - v2, e3 = v4 - v3;
  // eps12 enters through the squares: -eps12 / 64 on the outer two, eps12 / 32
  // on the inner two sum to eps12 in every indicator (no accumulator copy)
  const double lo = -eps12 * (1.0 / 64.0), hi = eps12 * (1.0 / 32.0);
  const double s0 = fma(e0, e0, lo), s1 = fma(e1, e1, hi), s2 = fma(e2, e2, hi), s3 = fma(e3, e3, lo);
  const double x01 = e0 * e1, x12 = e1 * e2, x23 = e2 * e3;
  double t0 = fma(16.0, s0, fma(-44.0, x01, 40.0 * s1));
  double t1 = fma(16.0, s1, fma(-20.0, x12, 16.0 * s2));
  double t2 = fma(40.0, s2, fma(-44.0, x23, 16.0 * s3));
  t0 *= t0;
  t1 *= t1;
  t2 *= t2;
  const double u0 = t1 * t2, u1 = t0 * t2, u2 = t0 * t1;
  const double g0 = fma(5.0 / 6.0, e1, (-1.0 / 3.0) * e0);
  const double g1x6 = fma(2.0, e2, e1);
  const double g2x3 = fma(2.0, e2, -0.5 * e3);
  const double num = fma(u2, g2x3, fma(u1, g1x6, u0 * g0));
  const double den = fma(3.0, u2, fma(6.0, u1, u0));
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  r = fma(r, fma(-den, r, 1.0), r);
  return fma(num, r, v2);
}

// DPP row_shl: lane i of every 16-lane row takes lane i + N's value (0 past
// the row's end)
template <int N>
__device__ __forceinline__ double row_shl(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x100 + N, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x100 + N, 0xf, 0xf, false);
  return __builtin_bit_cast(double, (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)hi << 32));
}
__device__ __forceinline__ double row_next(double v) { return row_shl<1>(v); }

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int BUF_DWORD3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const double* base) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, -1, BUF_DWORD3);
}
// A buffer of 2^31 bytes: an access at BUF_DROP (no scalar offset) is out of
// range, so a store there is dropped and a load returns 0.
constexpr unsigned BUF_DROP = 0xfffffff0u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf2g(const double* base) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)0x80000000u, BUF_DWORD3);
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
typedef unsigned u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned))));
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, 0);
}

// Hermite coefficients a_0 .. a_15 of the unit-density expansion along one
// axis at node (column c, axis): a_0 = 1, a_1 = u, a_{m+1} = u a_m +
// m (T - 1) a_{m-1}, into AH[buf][m][c + 8 axis] (the B operand layout of the
// expansion MFMA).
__device__ __forceinline__ void fused_hermite(FusedSmem& S, int fb, int t) {
  const int c = t & (SW - 1), axis = t >> 3;
  const double u = S.fl[fb][axis == 0 ? F_UX : F_UY][c], Tm1 = S.fl[fb][F_T][c] - 1.0;
  double* a = &S.AH[fb][0][t];
  double a0 = 1.0, a1 = u;
  a[0] = a0;
  a[16] = a1;
#pragma unroll
  for (int m = 1; m < Q - 1; ++m) {
    const double an = fma(u, a1, (double)m * Tm1 * a0);
    a0 = a1;
    a1 = an;
    a[16 * (m + 1)] = an;
  }
}

// Per-node coefficients of the collision row polynomial of one
// distribution (d: F or G) from the node fields of column c (fl[fb]) into
// CF[cb].
__device__ __forceinline__ void fused_coeffs(const Dev& D, FusedSmem& S, int fb, int cb, int c, int d) {
  const double* fl = &S.fl[fb][0][0];
#define FL(i) fl[(i) * SW + c]
  const bool j0 = (D.term_mask & EVLB_TERM_J0) != 0;
  const bool j1 = (D.term_mask & EVLB_TERM_J1) != 0;
  const double T = FL(F_T), invT = 1.0 / T;
  const double nu = j0 ? FL(F_NU) : 0.0;
  const double pre = j1 ? FL(F_PRE) : 0.0;
  const double th0 = d == 0 ? 4.0 : 2.0;
  const double Sx = fma(nu, FL(F_SQX), 0.3 * pre * FL(F_BX));
  const double Sy = fma(nu, FL(F_SQY), 0.3 * pre * FL(F_BY));
  const double C = 0.2 * pre * (FL(F_UXX) + FL(F_UYY));
  const double W4 = 0.4 * pre * invT;
  double* cf = &S.CF[cb][0][c];
  cf[CF_C0 * SW] = fma(-th0, C, nu);
  cf[CF_C1 * SW] = fma(-th0, Sx, pre * FL(F_AX));
  cf[CF_C2 * SW] = fma(invT, C, W4 * FL(F_UXX));
  cf[CF_C3 * SW] = invT * Sx;
  cf[CF_D0 * SW] = fma(-th0, Sy, pre * FL(F_AY));
  cf[CF_D1 * SW] = W4 * (FL(F_UXY) + FL(F_UYX));
  cf[CF_D2 * SW] = invT * Sy;
  cf[CF_E0 * SW] = fma(invT, C, W4 * FL(F_UYY));
  cf[CF_UX * SW] = FL(F_UX);
  cf[CF_UY * SW] = FL(F_UY);
  cf[CF_TFN * SW] = (j0 || j1) ? (d == 0 ? 1.0 : 0.5 * T) * FL(F_N) : 0.0;
  cf[CF_NU * SW] = nu;
  cf[CF_FX * SW] = FL(F_FX);
  cf[CF_FY * SW] = FL(F_FY);
#undef FL
}

// e_k = sum_m meq[k][m] a_m for the 16 columns (node, axis) of a row on the
// f64 MFMA (B element [c][col] = a_{c + 4 b}(col) from lane col + 16 c;
// result e_{4 j + c}(col) in register j of that lane), into EK[buf].
__device__ __forceinline__ void fused_expansions(FusedSmem& S, int fb, int L) {
  const int c4 = L >> 4, col16 = L & 15;
  dbl4 e = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int b = 0; b < 4; ++b)
    e = __builtin_amdgcn_mfma_f64_16x16x4f64(S.eop[b][L], S.AH[fb][c4 + 4 * b][col16], e, 0, 0, 0);
#pragma unroll
  for (int j = 0; j < 4; ++j) S.EK[fb][col16 >> 3][4 * j + c4][col16 & 7] = e[j];
}

// Raw velocity sum s = t / SW of row y at column t % SW: the sum over the 16
// wavefronts' terms.
__device__ __forceinline__ void fused_raw_sum(const Dev& D, const FusedArgs& A, const FusedSmem& S, int d, int t,
                                              int x0, int y) {
  const int s = t / SW, cc = t & (SW - 1);
  if (x0 + cc >= D.nx) return;
  const double* m = &S.mred[y & 1][0][s][cc];
  double v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = m[i * 8 * SW];
#pragma unroll
  for (int l = 4; l < SNW; ++l) v[l & 3] += m[l * 8 * SW];
  A.raw[(long long)((d == 0 ? 0 : 8) + s) * D.ntot + (long long)y * D.nx + x0 + cc] = (v[0] + v[1]) + (v[2] + v[3]);
}

template <int N>
struct RotC {
  static constexpr int value = N;
};

template <bool ADV, bool FRC, bool FIRST>
__global__ __launch_bounds__(SNT) void fused_kernel(Dev D, FusedArgs A, const double* __restrict__ velg,
                                                    const double* __restrict__ meqg,
                                                    const double* __restrict__ dpmg) {
  __shared__ FusedSmem S;
  const int tid0 = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid0 >> 6);
  const int L0 = tid0 & 63;
  const int nx = D.nx, ny = D.ny;
  // workgroup -> (segment, strip, distribution); contiguous ranges per XCD
  // put neighbouring strips, which share halo columns, on one L2
  const unsigned per = 2u * (unsigned)A.nstrip;
  const unsigned tb = xcd_block(blockIdx.x, gridDim.x);
  const int seg = (int)(tb / per), rr = (int)(tb - (unsigned)seg * per);
  const int strip = rr >> 1, d = rr & 1;
  const int x0 = strip * SW;
  const int ya = seg * A.seglen;
  const int yb = min(ya + A.seglen, ny);
  const double eps12 = 12.0 * D.weno_eps;

  if (tid0 < 256) {
    const int e = (tid0 & 15) * Q + ((tid0 >> 4) & 3) + 4 * (tid0 >> 6);
    S.aop[tid0 >> 6][tid0 & 63] = dpmg[e];
    S.eop[tid0 >> 6][tid0 & 63] = meqg[e];
  }
  if (tid0 < Q) S.vel[tid0] = velg[tid0];

  const long long dofs = (long long)d * V * D.ntot;
  const __amdgpu_buffer_rsrc_t rs = buf(A.fs + dofs), r0 = buf((FIRST ? A.fs : A.f0) + dofs);
  const __amdgpu_buffer_rsrc_t ro = buf2g(A.out + dofs), rf = buf(A.fld);
  auto wrapx = [&](int x) { x %= nx; return x < 0 ? x + nx : x; };
  // per-lane byte offset of velocity (w, r) at the lane's column; (w, r + 8)
  // is 64 bytes further, a row nx V doubles further
  const unsigned vo = ((unsigned)wrapx(x0 + (L0 & 7)) * (unsigned)V + 16u * (unsigned)w + (unsigned)(L0 >> 3)) * 8u;
  constexpr unsigned pso = 8u * 8u;
  const unsigned rowb = (unsigned)nx * (unsigned)V * 8u;
  // the wavefront's halo, 16 velocities x 6 columns (a 128-byte line each):
  // lane L takes l = L >> 2 of column x0 - 3, x0 - 2, x0 - 1, x0 + 8 for
  // L & 3 = 0 .. 3, and l = (L & 31) >> 1 of column x0 + 9 + (L & 1) (lanes
  // 32 - 63 repeat 0 - 31); each load still covers whole lines, and the LDS
  // writes of a 16-lane pass fall on at least 8 banks
  const unsigned hvoA = ((unsigned)wrapx((L0 & 3) < 3 ? x0 - 3 + (L0 & 3) : x0 + SW) * (unsigned)V +
                         16u * (unsigned)w + (unsigned)(L0 >> 2)) * 8u;
  const unsigned hvoB = ((unsigned)wrapx(x0 + SW + 1 + (L0 & 1)) * (unsigned)V + 16u * (unsigned)w +
                         (unsigned)((L0 & 31) >> 1)) * 8u;
  // node fields [NF][ntot]: thread t < NF SW loads field t / SW of column t % SW
  const bool fthr = tid0 < NF * SW;
  const unsigned fvo =
      fthr ? ((unsigned)(tid0 / SW) * (unsigned)D.ntot + (unsigned)wrapx(x0 + (tid0 & (SW - 1)))) * 8u : 0u;
  const unsigned rowf = (unsigned)nx * 8u;
  const double pk = velg[w];
  const double pxi = pk * D.inv_dx;
  // MFMA A operand of the raw-sum weights of this wavefront's k, for sums
  // s < 8 over l < 8 in rows i = s and over l >= 8 in rows i = 8 + s: lane
  // i + 16 c holds C[s][l = c + 4 b + 8 (i >> 3)] (p = p_k, q = p_l):
  //   F: n: 1, j_x: p, j_y: q, P_xx: p^2, P_xy: p q, P_yy: q^2,
  //      r_x: p (p^2 + q^2), r_y: q (p^2 + q^2);  G: g0: 1, h_x: p, h_y: q
  double mop[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int i = L0 & 7;
    const double q = velg[(L0 >> 4) + 4 * b + (L0 & 8)], pq2 = pk * pk + q * q;
    double cw = 0.0;
    if (i == 0) cw = 1.0;
    else if (i == 1) cw = pk;
    else if (i == 2) cw = q;
    else if (d == 0 && i == 3) cw = pk * pk;
    else if (d == 0 && i == 4) cw = pk * q;
    else if (d == 0 && i == 5) cw = q * q;
    else if (d == 0 && i == 6) cw = pk * pq2;
    else if (d == 0 && i == 7) cw = q * pq2;
    mop[b] = cw;
  }
  const bool PX = pk > 0.0;  // uniform per wavefront
  const double bb = FIRST ? A.a + A.b : A.b;  // the first stage has f^n = f^(s-1)

  // y within 4 rows of the domain (ny >= 8)
  auto wrapy = [&](int y) { return (unsigned)(y < 0 ? y + ny : (y >= ny ? y - ny : y)); };
  auto rowso = [&](int y) { return wrapy(y) * rowb; };
  auto rowsf = [&](int y) { return wrapy(y) * rowf; };

  // ---- prologue.  The ring R5[j] holds, per velocity, five consecutive
  // rows in marching order: (y - 2 .. y + 2) for j = 1 (p_l > 0), (y - 1 ..
  // y + 3) for j = 0 (p_l < 0), so that the face between rows y and y + 1 is
  // weno5(R0 .. R4), resp. weno5(R4 .. R0), and the row dropped after the
  // face is always R0.
  double R5[2][5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
#pragma unroll
    for (int j = 0; j < 2; ++j) R5[j][i] = bload(rs, vo, j * pso + rowso(ya - 1 - j + i));
  }
  double fyl[2] = {0.0, 0.0};
  if (ADV) {  // the face between rows ya - 1 and ya
    const double e0 = bload(rs, vo, rowso(ya - 2)), e1 = bload(rs, vo, pso + rowso(ya - 3));
    fyl[0] = weno5(R5[0][3], R5[0][2], R5[0][1], R5[0][0], e0, eps12);
    fyl[1] = weno5(e1, R5[1][0], R5[1][1], R5[1][2], R5[1][3], eps12);
  }
  // f^n and the halo of row ya, node fields of rows ya .. ya + 3
  double f0v[2] = {0.0, 0.0}, hv[2];
  if (!FIRST) {
#pragma unroll
    for (int j = 0; j < 2; ++j) f0v[j] = bload(r0, vo, j * pso + rowso(ya));
  }
  hv[0] = bload(rs, hvoA, rowso(ya));
  hv[1] = bload(rs, hvoB, rowso(ya));
  double fq = bload(rf, fvo, rowsf(ya + 3));
  const double fq2 = bload(rf, fvo, rowsf(ya + 2));
  if (fthr) {
    S.fl[ya & 1][tid0 / SW][tid0 & (SW - 1)] = bload(rf, fvo, rowsf(ya));
    S.fl[(ya + 1) & 1][tid0 / SW][tid0 & (SW - 1)] = bload(rf, fvo, rowsf(ya + 1));
  }
  __syncthreads();
  // Hermite and collision coefficients of rows ya, ya + 1
  if (w == 1 && L0 < 32) fused_hermite(S, (ya + (L0 >> 4)) & 1, L0 & 15);
  if (w == 3 && L0 < 16) fused_coeffs(D, S, (ya + (L0 >> 3)) & 1, (ya + (L0 >> 3)) & 3, L0 & 7, d);
  __syncthreads();
  // their expansions; the node fields of row ya + 2 replace those of row ya
  if (w == 1) fused_expansions(S, ya & 1, L0);
  if (w == 2) fused_expansions(S, (ya + 1) & 1, L0);
  if (fthr) S.fl[ya & 1][tid0 / SW][tid0 & (SW - 1)] = fq2;
  __syncthreads();
  if (w == 1 && L0 < 16) fused_hermite(S, ya & 1, L0);
  if (w == 3 && L0 < 8) fused_coeffs(D, S, ya & 1, (ya + 2) & 3, L0, d);
  __syncthreads();

  const int nsum = d == 0 ? 8 : 3;
  double accP[2] = {0.0, 0.0}, cfxP = 0.0;  // acc and c F_x of the row before
  // Byte offsets in the shared block of this lane's writes of row y into FI
  // (slot 0; l = r, r + 8) and of its halo values into T and FI, formed once
  // and held opaque, so that the compiler keeps them in registers instead of
  // deriving them again every row.
  unsigned ofi[2], oh[4];
  {
    const int r0 = L0 >> 3, c0 = L0 & 7;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int l = r0 + 8 * j;
      ofi[j] = (unsigned)offsetof(FusedSmem, FI) + 8u * (unsigned)(w * FIS + 8 * l + (c0 ^ ((l >> 1) & 7)));
    }
    const int lA = L0 >> 2, hA = L0 & 3, lB = (L0 & 31) >> 1, hB = 4 + (L0 & 1);
    oh[0] = (unsigned)offsetof(FusedSmem, T) + 8u * (unsigned)((16 * w + lA) * TS + (hA < 3 ? hA : SW + hA));
    oh[1] = (unsigned)offsetof(FusedSmem, FI) + 8u * (unsigned)(w * FIS + 16 * SW + 3 * lA);
    oh[2] = (unsigned)offsetof(FusedSmem, T) + 8u * (unsigned)((16 * w + lB) * TS + SW + hB);
    oh[3] = (unsigned)offsetof(FusedSmem, FI) + 8u * (unsigned)(w * FIS + 16 * SW + 3 * lB + hB - 3);
  }
  asm volatile("" : "+v"(ofi[0]), "+v"(ofi[1]), "+v"(oh[0]), "+v"(oh[1]), "+v"(oh[2]), "+v"(oh[3]));
  char* const Sb = (char*)&S;
  auto lds = [&](unsigned o) -> double& { return *(double*)(Sb + o); };
  // One row of the march.  The ring is not shifted: row y uses the slots
  // rotated by ROT = (y - ya) mod 5 (slot (i + ROT) mod 5 holds ring entry
  // i), and the march is unrolled five rows at a time so that every slot
  // index is a constant.
  auto row = [&](auto rotc, const int y) {
    constexpr int ROT = decltype(rotc)::value;
    auto R = [&](int j, int i) -> double& { return R5[j][(i + ROT) % 5]; };
    // Opaque per-row copies of the thread indices: every LDS address and
    // table value below is derived from them inside the row, so that the
    // compiler does not hoist them out of the loop and hold (or spill) them
    // across it.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int L = tid & 63, col = L & (SW - 1), r = L >> 3;
    const int yp = y & 1;
    double accN[2] = {0.0, 0.0}, cfxN = 0.0;
    // ---------------- pre(y) ----------------
    double* Tw = &S.T[16 * w * TS];  // this wavefront's 16 velocities
    const double* cf = &S.CF[y & 3][0][col];
    double part[2] = {0.0, 0.0}, base[2] = {0.0, 0.0};
    if (y < yb) {
      const unsigned fslot = (unsigned)yp * (unsigned)(Q * FIS * 8);  // FI[yp]
      const double nu = cf[CF_NU * SW];
      double cur[2];
      cur[0] = R(0, 1);  // row y
      cur[1] = R(1, 2);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        Tw[(r + 8 * j) * TS + 3 + col] = cur[j];
        lds(ofi[j] + fslot) = cur[j];  // FI[yp][w][8 l + (col ^ ((l >> 1) & 7))]
        base[j] = fma(A.a, f0v[j], bb * cur[j]);
        part[j] = -nu * cur[j];
      }
      // the halo: T of columns x0 - 3 .. x0 - 1, x0 + 8 .. x0 + 10, FI of
      // columns x0 + 8 .. x0 + 10
      lds(oh[0]) = hv[0];
      if ((L & 3) == 3) lds(oh[1] + fslot) = hv[0];
      lds(oh[2]) = hv[1];
      lds(oh[3] + fslot) = hv[1];
      if (tid < NF * SW) S.fl[(y + 3) & 1][tid / SW][tid & (SW - 1)] = fq;
      if (ADV) {
        // y faces: j = 0 upwind from above, j = 1 from below
        const double fyr0 = weno5(R(0, 4), R(0, 3), R(0, 2), R(0, 1), R(0, 0), eps12);
        const double fyr1 = weno5(R(1, 0), R(1, 1), R(1, 2), R(1, 3), R(1, 4), eps12);
        part[0] = fma(D.inv_dx * S.vel[r], fyl[0] - fyr0, part[0]);
        part[1] = fma(D.inv_dx * S.vel[r + 8], fyl[1] - fyr1, part[1]);
        fyl[0] = fyr0;
        fyl[1] = fyr1;
      }
    }
    // in flight across the rest of this iteration: node fields of row y + 4
    // (issued first: the wait for it in the next iteration then leaves the
    // later loads in flight), the ring's next row (into the slot just
    // dropped), f^n and the halo of row y + 1.  Outside the condition, and
    // past the segment too: a load under a condition would make the
    // compiler copy the register at the loop latch, which waits for every
    // load in flight.
    fq = bload(rf, fvo, rowsf(y + 4));
#pragma unroll
    for (int j = 0; j < 2; ++j) R(j, 0) = bload(rs, vo, j * pso + rowso(y + 4 - j));  // row (y + 1) + 3 - j
    {
      const unsigned so1 = rowso(y + 1);
      if (!FIRST) {
#pragma unroll
        for (int j = 0; j < 2; ++j) f0v[j] = bload(r0, vo, j * pso + so1);
      }
      hv[0] = bload(rs, hvoA, so1);
      hv[1] = bload(rs, hvoB, so1);
    }
    if (y < yb) {
      if (ADV) {
        // x faces from this wavefront's LDS row: each lane the face on its
        // left, the face on its right from the next lane (the last column:
        // the strip-edge face, added in post(y + 1))
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double* t = &Tw[(r + 8 * j) * TS + col];
          const double lf = PX ? weno5(t[0], t[1], t[2], t[3], t[4], eps12)
                               : weno5(t[5], t[4], t[3], t[2], t[1], eps12);
          // every lane runs the DPP move (a lane masked off would read as 0
          // to its neighbour), then the last column drops what it read
          const double nb = row_next(lf);
          const double rf = col == SW - 1 ? 0.0 : nb;
          part[j] = fma(pxi, lf - rf, part[j]);
        }
      }
      double dy[2] = {0.0, 0.0};
      const bool odd = ((y - ya) & 1) != 0;
      if (FRC && (odd || y == yb - 1)) {
        // (I x Dp) f for k = w of two rows at once: B[c][col16] = f(w, l =
        // c + 4 b) at column col16 & 7 of row y - 1 (col16 < 8) or row y
        // (col16 >= 8), both from this wavefront's interior of FI (the slot
        // of row y - 1 is rewritten only in pre(y + 1)).  Row l' = 4 j + c of
        // the result goes through columns 14 - 21 of T to the lanes that own
        // it: row y's into this row's sum, row y - 1's (odd rows of the
        // segment; the even rows before them ran no MFMA) into the sum of the
        // row before.
        const int c4 = L >> 4, c8 = L & 7;
        const bool hi = (L & 8) != 0;
        const double* fp = &S.FI[hi ? yp : 1 - yp][w][0];
        const int x = c8 ^ (c4 >> 1);  // the swizzle of l = c4 + 4 b is x ^ 2 b
        dbl4 dd = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < 4; ++b)
          dd = __builtin_amdgcn_mfma_f64_16x16x4f64(S.aop[b][L], fp[8 * (c4 + 4 * b) + (x ^ (2 * b))], dd, 0, 0, 0);
        if (hi) {
#pragma unroll
          for (int j = 0; j < 4; ++j) Tw[(4 * j + c4) * TS + 14 + c8] = dd[j];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) dy[j] = Tw[(r + 8 * j) * TS + 14 + col];
        if (odd) {
          if (!hi) {
#pragma unroll
            for (int j = 0; j < 4; ++j) Tw[(4 * j + c4) * TS + 14 + c8] = dd[j];
          }
          // the lanes that wrote nothing still read what the others wrote:
          // keep the compiler from reusing the values read above
          asm volatile("" ::: "memory");
          const double fyp = A.c * S.CF[(y - 1) & 3][CF_FY][col];
#pragma unroll
          for (int j = 0; j < 2; ++j) accP[j] = fma(-fyp, Tw[(r + 8 * j) * TS + 14 + col], accP[j]);
        }
      }
      // collision terms: with xi_x = p_k - u_x fixed per wavefront, the row
      // polynomial in xi_y = p_l - u_y
      const double xx = pk - cf[CF_UX * SW];
      const double c3 = cf[CF_C3 * SW], d2 = cf[CF_D2 * SW];
      const double P0 = fma(xx, fma(xx, fma(c3, xx, cf[CF_C2 * SW]), cf[CF_C1 * SW]), cf[CF_C0 * SW]);
      const double P1 = fma(xx, fma(d2, xx, cf[CF_D1 * SW]), cf[CF_D0 * SW]);
      const double P2 = fma(c3, xx, cf[CF_E0 * SW]);
      const double tfe = cf[CF_TFN * SW] * S.EK[yp][0][w][col];  // tf n e_k(u_x)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int l = r + 8 * j;
        const double xy = S.vel[l] - cf[CF_UY * SW];
        double Lc = tfe * S.EK[yp][1][l][col] * fma(xy, fma(xy, fma(d2, xy, P2), P1), P0);
        if (FRC) Lc = fma(-cf[CF_FY * SW], dy[j], Lc);
        accN[j] = fma(A.c, part[j] + Lc, base[j]);
      }
      if (FRC) cfxN = A.c * cf[CF_FX * SW];
    }
    __syncthreads();
    // ---------------- post(y) ----------------
    {
      // f^(s) of row y - 1 (y > ya).  The stores run every iteration, those
      // with nothing to store at an offset past the buffer, so that every
      // iteration issues the same vector memory operations and the wait for
      // a load issued before them never has to drain them.
      const int pb = (y - 1) & 1;
      const bool live = y > ya;
      const unsigned so = live && x0 + col < nx ? vo + rowso(y - 1) : BUF_DROP;
      double* Tw = &S.T[16 * w * TS];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int l = r + 8 * j;
        double o = accP[j];
        if (live) {
          if (FRC) o = fma(-cfxP, S.DX[pb][w][8 * (l ^ (2 * (w & 1))) + col], o);
          if (ADV && col == SW - 1) o = fma(-A.c * pxi, S.T[(16 * w + l) * TS + 22 + pb], o);
        }
        bstore(o, ro, so == BUF_DROP ? BUF_DROP : so + j * pso, 0);
        Tw[l * TS + 14 + col] = o;  // free until pre(y + 1)
      }
      if (live && A.want_mom) {
        // this wavefront's terms of the raw sums, C f^(s) with C[s][l] the
        // weights of sum s (mop), on the MFMA: B[c][col16] = f^(s)(w, l =
        // c + 4 b + 8 h) at column col16 & 7, h = col16 >> 3.  Sum s = 4 j + c
        // of a column is row s of the result at col16 < 8 (over l < 8) plus
        // row 8 + s at col16 + 8 (over l >= 8), eight lanes further.
        const int c4 = L >> 4, c8 = L & 7;
        dbl4 dd = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < 2; ++b)
          dd = __builtin_amdgcn_mfma_f64_16x16x4f64(mop[b], Tw[(c4 + 4 * b + (L & 8)) * TS + 14 + c8], dd, 0, 0, 0);
        const double s0 = dd[0] + row_shl<8>(dd[2]), s1 = dd[1] + row_shl<8>(dd[3]);
        if ((L & 8) == 0) {
          S.mred[pb][w][c4][c8] = s0;
          S.mred[pb][w][4 + c4][c8] = s1;
        }
      }
    }
    // the serial chains on the oldest wavefront of each SIMD (the arbiter
    // issues the oldest first), the strip-edge faces (VALU) on the next
    // oldest, the MFMA work on the two youngest
    if (w == 0) {
      if (A.want_mom && y - 2 >= ya && L < nsum * SW) fused_raw_sum(D, A, S, d, L, x0, y - 2);
    } else if (w == 1) {
      // Hermite coefficients of row y + 3
      if (y + 3 < yb && L < 16) fused_hermite(S, (y + 3) & 1, L);
    } else if (w == 2) {
      if (y + 2 < yb) fused_expansions(S, (y + 2) & 1, L);
    } else if (w == 3) {
      // collision coefficients of row y + 3
      if (y + 3 < yb && L < SW) fused_coeffs(D, S, (y + 3) & 1, (y + 3) & 3, L, d);
    } else if (w >= 8) {
      if (FRC && y < yb) {
        // (Dp x I) f for l = 2 (w - 8) + lh: B[c][col16] = f(k = c + 4 b, l),
        // col16 = (column, lh)
        const int c4 = L >> 4, lq = 2 * (w - 8) + ((L >> 3) & 1);
        dbl4 dd = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int b = 0; b < 4; ++b)
          dd = __builtin_amdgcn_mfma_f64_16x16x4f64(S.aop[b][L], S.FI[yp][c4 + 4 * b][8 * lq + (col ^ ((lq >> 1) & 7))],
                                                    dd, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = 4 * j + c4;
          S.DX[yp][k][8 * (lq ^ (2 * (k & 1))) + col] = dd[j];
        }
      }
    } else {  // wavefronts 4 - 7
      if (ADV && y < yb) {
        // the strip-edge face of velocity (k, l), q = 16 k + l, from the
        // interior columns 5 - 7 and the right halo of FI, into the owner's T
        const int q = 64 * (w - 4) + L, k = q >> 4, l = q & 15;
        const double* fi = &S.FI[yp][k][8 * l];
        const int sw = (l >> 1) & 7;
        const double i5 = fi[5 ^ sw], i6 = fi[6 ^ sw], i7 = fi[7 ^ sw];
        fi = &S.FI[yp][k][0];
        const double h0 = fi[16 * SW + 3 * l], h1 = fi[16 * SW + 3 * l + 1], h2 = fi[16 * SW + 3 * l + 2];
        const bool px = k >= 8;
        S.T[q * TS + 22 + yp] = weno5(px ? i5 : h2, px ? i6 : h1, px ? i7 : h0, px ? h0 : i7, px ? h1 : i6, eps12);
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) accP[j] = accN[j];
    cfxP = cfxN;
  };
  for (int y = ya; y <= yb; y += 5) {
    row(RotC<0>(), y);
    if (y + 1 > yb) break;
    row(RotC<1>(), y + 1);
    if (y + 2 > yb) break;
    row(RotC<2>(), y + 2);
    if (y + 3 > yb) break;
    row(RotC<3>(), y + 3);
    if (y + 4 > yb) break;
    row(RotC<4>(), y + 4);
  }
  // velocity sums of the last row
  __syncthreads();
  if (A.want_mom && w == 0 && L0 < nsum * SW) fused_raw_sum(D, A, S, d, L0, x0, yb - 1);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t tab_d, tab_i, f1, f2, mom, raw, fld, status, total;
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
  L.raw = off; off += align256(sizeof(double) * NRAW * (size_t)N);
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
  if (N > (1ll << 20)) return EVLB_EINVAL;  // 32-bit byte offsets within one distribution's 256 planes
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

int launch_raw(Ctx* c, const double* f, hipStream_t st) {
  const unsigned nb = (unsigned)((c->N + 3) / 4);  // one wavefront per node
  hipLaunchKernelGGL(raw_sums_kernel, dim3(nb), dim3(256), 0, st, c->dev, f, (double*)(c->ws + c->L.raw), c->vel);
  return launched();
}

int launch_fields(Ctx* c, hipStream_t st) {
  const dim3 grid((c->nx + FTX - 1) / FTX, (c->ny + FTY - 1) / FTY);
  hipLaunchKernelGGL(fields_kernel, grid, dim3(FNT), fields_lds_bytes(c->L.halo), st, c->dev,
                     (const double*)(c->ws + c->L.raw), (double*)(c->ws + c->L.fld), c->avg_ofs, c->avg_w,
                     c->pair_ofs, c->pair_cx, c->pair_cy);
  return launched();
}

// Strips of SW columns, two distributions, and enough segments of rows for
// about one workgroup per CU (at least 16 rows each: a segment re-reads the
// six rows of its ring prologue).
void fused_shape(const Ctx* c, int* nstrip, int* nseg, int* seglen) {
  *nstrip = (c->nx + SW - 1) / SW;
  int s = (256 + 2 * *nstrip - 1) / (2 * *nstrip);
  const int smax = c->ny / 16 > 1 ? c->ny / 16 : 1;
  if (s > smax) s = smax;
  if (s < 1) s = 1;
  *seglen = (c->ny + s - 1) / s;
  *nseg = (c->ny + *seglen - 1) / *seglen;  // every segment non-empty
}

template <bool ADV, bool FRC>
void launch_fused(Ctx* c, const FusedArgs& A, dim3 grid, int first, hipStream_t st) {
  if (first)
    hipLaunchKernelGGL((fused_kernel<ADV, FRC, true>), grid, dim3(SNT), 0, st, c->dev, A, c->vel, c->meq, c->dpm);
  else
    hipLaunchKernelGGL((fused_kernel<ADV, FRC, false>), grid, dim3(SNT), 0, st, c->dev, A, c->vel, c->meq, c->dpm);
}

// one evaluation: the fields of the raw sums in the workspace, then
// out = a f0 + b fs + c L(fs) and (want_mom) the raw sums of out
int stage(Ctx* c, const double* fs, const double* f0, double* out, double a, double b, double cc, int first,
          int want_mom, hipStream_t st) {
  int rc = launch_fields(c, st);
  if (rc) return rc;
  int nstrip, nseg, seglen;
  fused_shape(c, &nstrip, &nseg, &seglen);
  FusedArgs A{fs, f0, out, (const double*)(c->ws + c->L.fld), (double*)(c->ws + c->L.raw), a, b, cc, first,
              want_mom, nstrip, seglen};
  const dim3 grid((unsigned)(2 * nstrip * nseg));
  const bool adv = (c->dev.term_mask & EVLB_TERM_ADV) != 0, frc = (c->dev.term_mask & EVLB_TERM_FORCE) != 0;
  if (adv && frc)
    launch_fused<true, true>(c, A, grid, first, st);
  else if (adv)
    launch_fused<true, false>(c, A, grid, first, st);
  else if (frc)
    launch_fused<false, true>(c, A, grid, first, st);
  else
    launch_fused<false, false>(c, A, grid, first, st);
  return launched();
}

}  // namespace

int set_equilibrium(Ctx* c, const double* n, const double* u, const double* T, double* f, hipStream_t st) {
  const unsigned nb = (unsigned)((c->N + 3) / 4);  // one wavefront per node
  hipLaunchKernelGGL(equilibrium_kernel, dim3(nb), dim3(256), 0, st, c->dev, n, u, T, f, c->meq);
  return launched();
}

int step(Ctx* c, double* f, int nsteps, hipStream_t st) {
  static const double RKA[3] = {0.0, 0.75, 1.0 / 3.0};
  static const double RKB[3] = {1.0, 0.25, 2.0 / 3.0};
  double* f1 = (double*)(c->ws + c->L.f1);
  double* f2 = (double*)(c->ws + c->L.f2);
  int rc = launch_raw(c, f, st);
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
  int rc = launch_raw(c, f, st);
  if (rc) return rc;
  return stage(c, f, f, L, 0.0, 0.0, 1.0, 1, 0, st);
}

int moments(Ctx* c, const double* f, double* n, double* u, double* T, double* q, hipStream_t st) {
  double* m = (double*)(c->ws + c->L.mom);
  const unsigned nb = (unsigned)((c->N + 3) / 4);  // one wavefront per node
  hipLaunchKernelGGL(moments_kernel, dim3(nb), dim3(256), 0, st, c->dev, f, m, c->vel);
  if (launched()) return EVLB_EHIP;
  const size_t bytes = sizeof(double) * (size_t)c->N;
  if (hipMemcpyAsync(n, m, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(u, m + c->N, 2 * bytes, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(T, m + 3 * c->N, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return EVLB_EHIP;
  if (q && hipMemcpyAsync(q, m + 4 * c->N, 2 * bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return EVLB_EHIP;
  return EVLB_OK;
}

}  // namespace evlb2d
