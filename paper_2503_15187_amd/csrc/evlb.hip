// EV-FDLB time step for MI355X (gfx950): fused HIP kernels and the C ABI
// declared in include/evlb.h.
//
// One TVD-RK3 stage is ONE kernel.  A workgroup owns a tile of W = 64
// consecutive nodes of one periodic system and all q velocities:
//   1. load     F, G rows of the tile plus a 3-node halo (WENO-5) into LDS;
//               the density window (force / averaged density halo) and
//               u, T (gradient halo) from the moments of the previous stage.
//   2. fields   averaged density and contact value (eq:carnstar, Sec. II A)
//               on the tile +-2; WENO-5 face values of every row.
//   3. fields   Vlasov force (eq:F1 / eq:F2), transport (eq:viscosity,
//               eq:tau, eq:prandtl), J1 gradients (eq:J1) per node.
//   4. update   lanes = nodes, wavefront = group of velocities: Hermite
//               equilibrium, momentum derivative, Shakhov term, J1, advection,
//               RK3 combine; partial velocity moments of the new state.
//   5. reduce   moments (n, u, T, q) of the new state -> global, read by the
//               next stage.
// Global state is structure-of-arrays [2][q][n_tot] (node fastest), so every
// row load and store of a wavefront is one contiguous 512-byte segment.
//
// Tile shapes: wide tiles (64 nodes, groups of velocities per wavefront,
// tables through the scalar cache), narrow tiles (16 nodes, one update per
// thread, the velocity-space contractions on the f64 MFMA) for grids too
// small to fill the chip, and column tiles (one wavefront of 63 nodes, a
// node's whole velocity column in registers) for large grids.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/evlb.h"
#include "evlb2d.h"
#include "tables.h"

namespace {

constexpr int W = 64;          // nodes per tile == lanes of a wavefront
constexpr int HF = 3;          // distribution halo of the WENO-5 faces
constexpr int MS_MAX = 16;     // max sigma/dx
constexpr int MF_MAX = 64;     // max r_cut/dx
constexpr int HN_MAX = MF_MAX; // density window half width
constexpr int NFIELD = 10;

enum { NF_N, NF_U, NF_T, NF_NU, NF_S, NF_PRE, NF_A, NF_B, NF_U1, NF_FX };

struct DevParams {
  const double* vel;   // [q]
  const double* meq;   // [q][q]
  const double* dpm;   // [q][q]
  const double* savg;  // [2 ms + 1]
  const double* cfor;  // [mf]
  const double* cphi;  // [mf] d cfor / d phi_sigma
  const double* csig;  // [mf] d cfor / d sigma
  const double* ssig;  // [2 ms + 1] d savg / d sigma
  const int4* tiles;   // {system offset, system nodes, tile start, 0}
  int ntiles;
  int single;          // one system: tile t starts at node t * width
  int ms, mf, hn;
  long long ntot;
  double dx, inv_dx, dt;
  double b;        // 2 pi sigma^3 / 3
  double eta_c;    // pi sigma^3 / 6
  double mu0c;     // 5 / (16 sigma^2 sqrt(pi)):  mu0 = mu0c sqrt(T)
  double sigma;
  double weno_eps, g_ext, two_a, kappa;
  double T_iso;    // > 0: isothermal, the temperature the next stage sees
  const double* tiso;  // per node: the isothermal temperature of its system (0 = thermal), or null
  int force_model, term_mask;
  int* status;     // [0] non-finite latch, [1] barrier abort latch
  unsigned* bar;   // [0] arrival count, [1] generation
};

struct StageArgs {
  const double* f_prev;  // f^(s-1)
  const double* f_n;     // f^n (RK3 base)
  double* f_out;         // f^(s), or L(f) in rhs mode
  const double* mom_in;  // [4][ntot] n, u, T, q of f_prev
  double* mom_out;       // [4][ntot] of f_out
  double alpha, beta;    // f_out = alpha f_n + beta (f_prev + dt L)
  int first;             // f_n == f_prev
  int rhs_mode;          // write L(f_prev) instead of a stage
};

// 1/x from the hardware reciprocal and two Newton steps r <- r (2 - x r):
// within an ulp or two of the quotient, with a shorter dependency chain
// than the correctly rounded division
__device__ __forceinline__ double rcpn(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// Lane i takes lane i + 1's value across the whole wavefront (DPP wave_shl:1;
// lane 63 gets 0).  Two VALU moves, where a shuffle is an LDS-crossbar round
// trip.
__device__ __forceinline__ double wave_next(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0x130, 0xf, 0xf, false);
  return __builtin_bit_cast(double, (unsigned long long)(unsigned)lo | ((unsigned long long)(unsigned)hi << 32));
}

// Classical WENO-5 (Jiang & Shu) face value from the five upwind-ordered
// values v0..v4 = f_{i-2}..f_{i+2}; alpha_r = d_r/(eps+beta_r)^2 combined
// over a common denominator (one reciprocal).
//
// Two arithmetic forms of the same function.  LEAN works in the first
// differences e_m = v_(m+1) - v_m: the candidates less v2 are g0 = (5 e1 -
// 2 e0) / 6, 6 g1 = e1 + 2 e2, 3 g2 = 2 e2 - e3 / 2; the smoothness
// indicators 12 beta_r (against 12 eps) expand in the squares and neighbour
// products of the differences to 16 e0^2 - 44 e0 e1 + 40 e1^2, 16 e1^2 -
// 20 e1 e2 + 16 e2^2 and 40 e2^2 - 44 e2 e3 + 16 e3^2; with the linear
// weights as 10 d_r = (1, 6, 3) the value is v2 plus the normalised
// weighted corrections -- about fifteen fewer operations per face: the
// column and wide tiles, whose faces are throughput work, use it.  The
// narrow tile's faces sit on its critical path, and there the textbook form
// measures slightly faster.
template <bool LEAN>
__device__ __forceinline__ double weno5(double v0, double v1, double v2, double v3, double v4,
                                        double eps) {
  if constexpr (LEAN) {
    const double eps12 = 12.0 * eps;
    const double d0 = v1 - v0, d1 = v2 - v1, d2 = v3 - v2, d3 = v4 - v3;
    // eps12 enters through the squares: -eps12 / 64 on the outer two, eps12 / 32
    // on the inner two sum to eps12 in every indicator (no accumulator copy)
    const double lo = -eps12 * (1.0 / 64.0), hi = eps12 * (1.0 / 32.0);
    const double s0 = fma(d0, d0, lo), s1 = fma(d1, d1, hi), s2 = fma(d2, d2, hi), s3 = fma(d3, d3, lo);
    const double x01 = d0 * d1, x12 = d1 * d2, x23 = d2 * d3;
    double t0 = fma(16.0, s0, fma(-44.0, x01, 40.0 * s1));
    double t1 = fma(16.0, s1, fma(-20.0, x12, 16.0 * s2));
    double t2 = fma(40.0, s2, fma(-44.0, x23, 16.0 * s3));
    t0 *= t0;
    t1 *= t1;
    t2 *= t2;
    const double u0 = t1 * t2, u1 = t0 * t2, u2 = t0 * t1;
    const double g0 = fma(5.0 / 6.0, d1, (-1.0 / 3.0) * d0);
    const double g1x6 = fma(2.0, d2, d1);
    const double g2x3 = fma(2.0, d2, -0.5 * d3);
    const double num = fma(u2, g2x3, fma(u1, g1x6, u0 * g0));
    const double den = fma(3.0, u2, fma(6.0, u1, u0));
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    r = fma(r, fma(-den, r, 1.0), r);
    return fma(num, r, v2);
  }
  const double c0 = v0 - 2.0 * v1 + v2, e0 = v0 - 4.0 * v1 + 3.0 * v2;
  const double c1 = v1 - 2.0 * v2 + v3, e1 = v1 - v3;
  const double c2 = v2 - 2.0 * v3 + v4, e2 = 3.0 * v2 - 4.0 * v3 + v4;
  const double q0 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) * (1.0 / 6.0);
  const double q1 = (-v1 + 5.0 * v2 + 2.0 * v3) * (1.0 / 6.0);
  const double q2 = (2.0 * v2 + 5.0 * v3 - v4) * (1.0 / 6.0);
  const double b0 = (13.0 / 12.0) * c0 * c0 + 0.25 * e0 * e0;
  const double b1 = (13.0 / 12.0) * c1 * c1 + 0.25 * e1 * e1;
  const double b2 = (13.0 / 12.0) * c2 * c2 + 0.25 * e2 * e2;
  double t0 = eps + b0; t0 *= t0;
  double t1 = eps + b1; t1 *= t1;
  double t2 = eps + b2; t2 *= t2;
  const double w0 = 0.1 * t1 * t2;
  const double w1 = 0.6 * t0 * t2;
  const double w2 = 0.3 * t0 * t1;
  // divide through the hardware reciprocal and two Newton steps r <- r (2 - d r)
  const double den = w0 + w1 + w2;
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  r = fma(r, fma(-den, r, 1.0), r);
  return (w0 * q0 + w1 * q1 + w2 * q2) * r;
}

// Launch shape of the wide stage kernel: tiles of W = 64 nodes, NG groups of
// velocities (thread = node j x group g, NT = W * NG threads).  A velocity
// group is uniform over a wavefront, so the constant tables are read through
// the scalar cache.  (The 16-node shape has its own tile function,
// stage_tile_narrow.)
template <int Q, int W, int NG>
struct Shape {
  static constexpr int NT = W * NG;
  static constexpr int VPT = Q / NG;
  static_assert(W % 64 == 0, "a velocity group spans whole wavefronts");
  static_assert(Q % NG == 0, "velocity groups must divide q");
  static_assert(NG >= 2, "two node groups are needed for the field phase");
  static_assert(NT <= 1024, "workgroup too large");
};

template <int Q, int W, int NG>
struct Smem {
  double f[2 * Q][W + 2 * HF];     // F rows then G rows, tile + WENO halo
  union {
    double flux[2 * Q][W + 1];     // WENO-5 face values
    double red[NG][6][W];          // partial velocity moments
  };
  double n[W + 2 * HN_MAX];        // density window
  double u[W + 4], T[W + 4], X[W + 4], chi[W + 4];
  double a[Q][W];                  // Hermite moments of the local Maxwellian
  union {
    double fpart[NG][W];           // partial force sums
    double msum[6][W];             // velocity moments of the new state
  };
  double nf[NFIELD][W];
  double sav[2 * MS_MAX + 1];      // averaging weights
  double cf[MF_MAX];               // EV1 force taps
};

__device__ __forceinline__ int wrapi(int i, int n) {
  while (i < 0) i += n;
  while (i >= n) i -= n;
  return i;
}

// The averaging weights and force taps into LDS.  All loads are issued
// before the first LDS write, so the copy costs one memory round trip.
template <int Q, int W, int NG>
__device__ __forceinline__ void load_tables(const DevParams& P, Smem<Q, W, NG>& S) {
  constexpr int NT = Shape<Q, W, NG>::NT;
  constexpr int NSAV = 2 * MS_MAX + 1;
  constexpr int NALL = NSAV + MF_MAX;
  constexpr int L = (NALL + NT - 1) / NT;
  const int tid = threadIdx.x;
  double v[L];
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int e = tid + i * NT;
    // one load per entry through a selected pointer (separate loads in the
    // branches would be serialised by the register they share)
    const double* src = nullptr;
    int si = 0;
    if (e < 2 * P.ms + 1) { src = P.savg; si = e; }
    else if (e >= NSAV && e < NSAV + P.mf) { src = P.cfor; si = e - NSAV; }
    v[i] = src ? src[si] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int e = tid + i * NT;
    if (e < NSAV) S.sav[e] = v[i];
    else if (e < NALL) S.cf[e - NSAV] = v[i];
  }
  __syncthreads();
}

// One stage over one tile (see file header).
template <int Q, int W, int NG>
__device__ void stage_tile(const DevParams& P, const StageArgs& A, int tile, Smem<Q, W, NG>& S) {
  using SH = Shape<Q, W, NG>;
  constexpr int NT = SH::NT;
  constexpr int VPT = SH::VPT;
  const int tid = threadIdx.x;
  const int4 td = P.tiles[tile];
  const int off = td.x, nsys = td.y, i0 = td.z;
  const long long ntot = P.ntot;
  const int hn = P.hn;
  const int j = tid % W;
  const int g = __builtin_amdgcn_readfirstlane(tid / W);
  const int kbase = g * VPT;
  const bool valid = (i0 + j) < nsys;
  const long long gnode = off + i0 + j;

  // ---- 1. load ----------------------------------------------------------
  // RK3 base values of this thread's velocities, fetched first so that their
  // latency overlaps the tile staging
  double Fn[VPT], Gn[VPT];
  const bool need_base = !A.first && !A.rhs_mode && valid;
#pragma unroll
  for (int v = 0; v < VPT; ++v) {
    Fn[v] = 0.0;
    Gn[v] = 0.0;
    if (need_base) {
      Fn[v] = A.f_n[(long long)(kbase + v) * ntot + gnode];
      Gn[v] = A.f_n[(long long)(Q + kbase + v) * ntot + gnode];
    }
  }
  // tile + WENO halo of F and G, the density window, u and T on the tile +-2:
  // every load is issued before the first LDS write (one round trip)
  constexpr int FW = W + 2 * HF;
  constexpr int NFV = 2 * Q * FW;
  constexpr int LF = (NFV + NT - 1) / NT;
  double fv[LF];
#pragma unroll
  for (int i = 0; i < LF; ++i) {
    const int idx = tid + i * NT;
    fv[i] = 0.0;
    if (idx < NFV) {
      const int r = idx / FW;
      const int c = idx - r * FW;
      fv[i] = A.f_prev[(long long)r * ntot + off + wrapi(i0 - HF + c, nsys)];
    }
  }
  const double* mn = A.mom_in;
  constexpr int LN = (W + 2 * HN_MAX + NT - 1) / NT;
  const int nwin = W + 2 * hn;
  double nv[LN];
#pragma unroll
  for (int i = 0; i < LN; ++i) {
    const int c = tid + i * NT;
    nv[i] = 0.0;
    if (c < nwin) nv[i] = mn[off + wrapi(i0 - hn + c, nsys)];
  }
  static_assert(NT >= W + 4, "one thread per node of the tile +-2");
  double uv = 0.0, Tv = 0.0;
  if (tid < W + 4) {
    const int node = off + wrapi(i0 - 2 + tid, nsys);
    uv = mn[ntot + node];
    Tv = mn[2 * ntot + node];
  }
  double qj = 0.0;
  if (tid >= W && tid < 2 * W) qj = mn[3 * ntot + off + wrapi(i0 + j, nsys)];
  // isothermal temperature of the own node's system, read with the tile
  double tiso = P.T_iso;
  if (P.tiso && tid < W && valid) tiso = P.tiso[gnode];
#pragma unroll
  for (int i = 0; i < LF; ++i) {
    const int idx = tid + i * NT;
    if (idx < NFV) {
      const int r = idx / FW;
      S.f[r][idx - r * FW] = fv[i];
    }
  }
#pragma unroll
  for (int i = 0; i < LN; ++i) {
    const int c = tid + i * NT;
    if (c < nwin) S.n[c] = nv[i];
  }
  if (tid < W + 4) {
    S.u[tid] = uv;
    S.T[tid] = Tv;
  }
  __syncthreads();

  // ---- 2. contact value, Hermite moments, force partial sums, WENO faces ---
  {
    // contact value chi(nbar) and X = n^2 chi T on the tile +-2
    for (int c = tid; c < W + 4; c += NT) {
      const int cn = c + hn - 2;
      double s0 = 0.0, s1 = 0.0;
      int jj = -P.ms;
      for (; jj + 1 <= P.ms; jj += 2) {
        s0 += S.sav[jj + P.ms] * S.n[cn + jj];
        s1 += S.sav[jj + 1 + P.ms] * S.n[cn + jj + 1];
      }
      if (jj <= P.ms) s0 += S.sav[jj + P.ms] * S.n[cn + jj];
      const double eta = P.eta_c * (s0 + s1);
      const double om = 1.0 - eta;
      const double chi = (2.0 - eta) / (2.0 * om * om * om);
      const double nn = S.n[cn];
      S.chi[c] = chi;
      S.X[c] = nn * nn * chi * S.T[c];
    }
    // Hermite moments a_0 = n, a_1 = n u, a_{l+1} = u a_l + l (T - 1) a_{l-1}
    if (tid >= NT - W) {
      const int jn = tid - (NT - W);
      const double n = S.n[jn + hn], u = S.u[jn + 2], tm1 = S.T[jn + 2] - 1.0;
      double am = n, a = n * u;
      S.a[0][jn] = am;
      S.a[1][jn] = a;
#pragma unroll
      for (int l = 1; l < Q - 1; ++l) {
        const double an = u * a + (double)l * tm1 * am;
        am = a;
        a = an;
        S.a[l + 1][jn] = a;
      }
    }
    // EV1 force: node j, chunk g of the paired taps
    if (P.force_model == EVLB_FORCE_EV1) {
      const int ch = (P.mf + NG - 1) / NG;
      const int m0 = 1 + g * ch;
      const int m1 = min(P.mf, m0 + ch - 1);
      const int cn = j + hn;
      double s0 = 0.0, s1 = 0.0;
      int m = m0;
      for (; m + 1 <= m1; m += 2) {
        s0 += S.cf[m - 1] * (S.n[cn + m] - S.n[cn - m]);
        s1 += S.cf[m] * (S.n[cn + m + 1] - S.n[cn - m - 1]);
      }
      if (m <= m1) s0 += S.cf[m - 1] * (S.n[cn + m] - S.n[cn - m]);
      S.fpart[g][j] = s0 + s1;
    }
    if (P.term_mask & EVLB_TERM_ADV) {
      for (int idx = tid; idx < 2 * Q * (W + 1); idx += NT) {
        const int r = idx / (W + 1);
        const int jf = idx - r * (W + 1);      // face i0 + jf - 1/2
        const int k = r < Q ? r : r - Q;
        const bool pos = k >= Q / 2;             // p_k > 0: upwind from the left
        const double* fr = &S.f[r][0];
        const int b0 = pos ? jf : jf + 5;
        const int st = pos ? 1 : -1;
        S.flux[r][jf] = weno5<true>(fr[b0], fr[b0 + st], fr[b0 + 2 * st], fr[b0 + 3 * st], fr[b0 + 4 * st],
                              P.weno_eps);
      }
    }
  }
  __syncthreads();

  // ---- 3. node fields: force and gradients (group 0), transport (group 1) --
  if (tid < W) {
    const int c = j + 2;
    const int cn = j + hn;
    const double idx12 = P.inv_dx * (1.0 / 12.0);
    double Fx = P.g_ext;
    if (P.force_model == EVLB_FORCE_EV1) {
      double s = 0.0;
#pragma unroll
      for (int gg = 0; gg < NG; ++gg) s += S.fpart[gg][j];
      Fx += s;
    } else if (P.force_model == EVLB_FORCE_EV2) {
      const double d1 = (S.n[cn - 2] - 8.0 * S.n[cn - 1] + 8.0 * S.n[cn + 1] - S.n[cn + 2]) * idx12;
      const double d3 = (-S.n[cn - 2] + 2.0 * S.n[cn - 1] - 2.0 * S.n[cn + 1] + S.n[cn + 2]) *
                        (0.5 * P.inv_dx * P.inv_dx * P.inv_dx);
      Fx += P.two_a * d1 + P.kappa * d3;
    }
    const double T = S.T[c];
    S.nf[NF_A][j] = (S.X[c - 2] - 8.0 * S.X[c - 1] + 8.0 * S.X[c + 1] - S.X[c + 2]) * idx12 / S.X[c];
    S.nf[NF_B][j] = (S.T[c - 2] - 8.0 * S.T[c - 1] + 8.0 * S.T[c + 1] - S.T[c + 2]) * idx12 / T;
    S.nf[NF_U1][j] = (S.u[c - 2] - 8.0 * S.u[c - 1] + 8.0 * S.u[c + 1] - S.u[c + 2]) * idx12;
    S.nf[NF_FX][j] = Fx;
    S.nf[NF_N][j] = S.n[cn];
    S.nf[NF_U][j] = S.u[c];
    S.nf[NF_T][j] = T;
  } else if (tid < 2 * W) {
    // transport: mu (eq:viscosity), tau (eq:tau), Pr (eq:prandtl); rate chi/tau
    const int c = j + 2;
    const double n = S.n[j + hn];
    const double T = S.T[c];
    const double chi = S.chi[c];
    const double bn = P.b * n;
    const double y = bn * chi;
    const double mu0 = P.mu0c * sqrt(T);
    const double c12 = 0.16 * (1.0 + 12.0 / M_PI);
    const double c32 = 0.36 * (1.0 + 32.0 / (9.0 * M_PI));
    const double mu = mu0 * (1.0 / chi + 0.8 * bn + c12 * bn * bn * chi);
    S.nf[NF_NU][j] = chi * n * T * (1.0 + 0.4 * y) / mu;
    const double Pr = (2.0 / 3.0) * (1.0 + 0.6 * y) * (1.0 + 0.8 * y + c12 * y * y) /
                      ((1.0 + 0.4 * y) * (1.0 + 1.2 * y + c32 * y * y));
    S.nf[NF_S][j] = (1.0 - Pr) * qj / (5.0 * n * T * T);
    S.nf[NF_PRE][j] = -bn * chi;
  }
  __syncthreads();

  // ---- 4. update -----------------------------------------------------------
  const double* meq = P.meq;
  const double* dpm = P.dpm;
  const double* vel = P.vel;
  double pm[6] = {0, 0, 0, 0, 0, 0};
  {
    const double u = S.nf[NF_U][j], T = S.nf[NF_T][j];
    const double nu = S.nf[NF_NU][j], sS = S.nf[NF_S][j], pre = S.nf[NF_PRE][j];
    const double Ag = S.nf[NF_A][j], Bg = S.nf[NF_B][j], Ug = S.nf[NF_U1][j];
    const double Fx = S.nf[NF_FX][j];
    const double invT = 1.0 / T;
    // Hermite equilibrium E_k = sum_l meq[k][l] a_l
    double E[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v) E[v] = 0.0;
#pragma unroll
    for (int l = 0; l < Q; ++l) {
      const double al = S.a[l][j];
#pragma unroll
      for (int v = 0; v < VPT; ++v) E[v] += meq[(kbase + v) * Q + l] * al;
    }
    // momentum derivative (Dp F)_k, (Dp G)_k
    double dF[VPT], dG[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v) { dF[v] = 0.0; dG[v] = 0.0; }
    if (P.term_mask & EVLB_TERM_FORCE) {
#pragma unroll
      for (int kp = 0; kp < Q; ++kp) {
        const double fk = S.f[kp][j + HF];
        const double gk = S.f[Q + kp][j + HF];
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
          const double d = dpm[(kbase + v) * Q + kp];
          dF[v] += d * fk;
          dG[v] += d * gk;
        }
      }
    }
#pragma unroll
    for (int v = 0; v < VPT; ++v) {
      const int k = kbase + v;
      const double pk = vel[k];
      const double F = S.f[k][j + HF];
      const double G = S.f[Q + k][j + HF];
      const double xi = pk - u;
      const double th = xi * xi * invT;
      double LF = 0.0, LG = 0.0;
      if (P.term_mask & EVLB_TERM_ADV) {
        LF = -pk * (S.flux[k][j + 1] - S.flux[k][j]) * P.inv_dx;
        LG = -pk * (S.flux[Q + k][j + 1] - S.flux[Q + k][j]) * P.inv_dx;
      }
      if (P.term_mask & EVLB_TERM_FORCE) {
        LF -= Fx * dF[v];
        LG -= Fx * dG[v];
      }
      if (P.term_mask & EVLB_TERM_J0) {
        const double FS = E[v] * (1.0 + sS * xi * (th - 3.0));
        const double GS = T * E[v] * (1.0 + sS * xi * (th - 1.0));
        LF -= nu * (F - FS);
        LG -= nu * (G - GS);
      }
      if (P.term_mask & EVLB_TERM_J1) {
        LF += pre * E[v] * (xi * (Ag + 0.3 * (th - 3.0) * Bg) + 0.6 * (th - 1.0) * Ug);
        LG += pre * T * E[v] * (xi * (Ag + 0.3 * (th - 1.0) * Bg) + 0.2 * (3.0 * th - 1.0) * Ug);
      }
      double Fo, Go;
      if (A.rhs_mode) {
        Fo = LF;
        Go = LG;
      } else {
        const double Fb = A.first ? F : Fn[v];
        const double Gb = A.first ? G : Gn[v];
        Fo = A.alpha * Fb + A.beta * (F + P.dt * LF);
        Go = A.alpha * Gb + A.beta * (G + P.dt * LG);
      }
      if (valid) {
        A.f_out[(long long)k * ntot + gnode] = Fo;
        A.f_out[(long long)(Q + k) * ntot + gnode] = Go;
      }
      const double p2 = pk * pk;
      pm[0] += Fo;
      pm[1] += pk * Fo;
      pm[2] += p2 * Fo;
      pm[3] += p2 * pk * Fo;
      pm[4] += Go;
      pm[5] += pk * Go;
    }
  }
  __syncthreads();  // faces (aliased by red) fully consumed
  if (A.rhs_mode) return;
#pragma unroll
  for (int m = 0; m < 6; ++m) S.red[g][m][j] = pm[m];
  __syncthreads();

  // ---- 5. moments of the new state --------------------------------------
  for (int t = tid; t < 6 * W; t += NT) {
    const int m = t / W, jj = t - m * W;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int gg = 0; gg + 1 < NG; gg += 2) {
      s0 += S.red[gg][m][jj];
      s1 += S.red[gg + 1][m][jj];
    }
    if (NG & 1) s0 += S.red[NG - 1][m][jj];
    S.msum[m][jj] = s0 + s1;
  }
  __syncthreads();
  if (tid < W && valid) {
    const double n = S.msum[0][tid];
    const double u = S.msum[1][tid] / n;
    const double T = (2.0 / 3.0) * (0.5 * S.msum[2][tid] + S.msum[4][tid] - 0.5 * n * u * u) / n;
    const double x3 = S.msum[3][tid] - 3.0 * u * S.msum[2][tid] + 3.0 * u * u * S.msum[1][tid] - u * u * u * n;
    const double q = 0.5 * x3 + S.msum[5][tid] - u * S.msum[4][tid];
    A.mom_out[gnode] = n;
    A.mom_out[ntot + gnode] = u;
    A.mom_out[2 * ntot + gnode] = tiso > 0.0 ? tiso : T;
    A.mom_out[3 * ntot + gnode] = q;
    if (!(n > 0.0) || !(T > 0.0) || !isfinite(n) || !isfinite(T) || !isfinite(q) || !isfinite(u))
      P.status[0] = 1;
  }
  __syncthreads();
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Narrow shape: WN = 16 nodes x Q velocities, one update per thread
// (tid = k * 16 + j), Q / 4 wavefronts.  Built for grids too small to fill
// the chip, where a stage is a chain of latencies: every global load of a
// tile goes out in one batch, and the velocity-space contractions
//   E_k = sum_l meq[k][l] a_l,  (Dp F)_k = sum_k' dpm[k][k'] F_k'  (and G)
// run on v_mfma_f64_16x16x4 as (Q x Q) x (Q x 16 nodes) products (A operand
// [i][c] from lane i + 16 c, B operand [c][col] from lane col + 16 c, result
// [4 r + c][col] in register r of lane col + 16 c), so an update reads three
// LDS values instead of 3 Q.  The Dp chains need only the tile and run with
// the contact values and faces; the equilibrium chains wait for the Hermite
// moments and run with the node fields, on wavefronts other than the one
// that computes the fields.
// ---------------------------------------------------------------------------
constexpr int WN = 16;

// Sum of v over the four lanes j, j + 16, j + 32, j + 48 (every lane gets
// it): the cross-row swaps of gfx950 exchange 16-lane rows (pairs 0-1, 2-3)
// and 32-lane halves on the VALU.
__device__ __forceinline__ double row4_sum(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  const auto l16 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h16 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double a = __builtin_bit_cast(double, (unsigned long long)l16[0] | ((unsigned long long)h16[0] << 32));
  const double c = __builtin_bit_cast(double, (unsigned long long)l16[1] | ((unsigned long long)h16[1] << 32));
  const double s = a + c;  // rows 0 + 1 in rows 0, 1; rows 2 + 3 in rows 2, 3
  const unsigned long long sb = __builtin_bit_cast(unsigned long long, s);
  const unsigned slo = (unsigned)sb, shi = (unsigned)(sb >> 32);
  const auto l32 = __builtin_amdgcn_permlane32_swap(slo, slo, false, false);
  const auto h32 = __builtin_amdgcn_permlane32_swap(shi, shi, false, false);
  const double x = __builtin_bit_cast(double, (unsigned long long)l32[0] | ((unsigned long long)h32[0] << 32));
  const double y = __builtin_bit_cast(double, (unsigned long long)l32[1] | ((unsigned long long)h32[1] << 32));
  return x + y;
}

template <int Q>
struct SmemN {
  double f[2 * Q][WN + 2 * HF];  // F rows then G rows, tile + WENO halo
  double flux[2 * Q][WN + 1];    // WENO-5 face values
  double n[WN + 2 * HN_MAX];     // density window
  double u[WN + 4], T[WN + 4], X[WN + 4], chi[WN + 4];
  double a[Q][WN];               // Hermite moments of the local Maxwellian
  double fpart[Q][WN];           // EV1 partial force sums
  double ctr[3][Q][WN];          // E, Dp F, Dp G
  double nf[NFIELD][WN];
  double red[Q / 4][6][WN];      // per-wavefront velocity moments
  double sav[2 * MS_MAX + 1];
  double cf[MF_MAX];
};

template <int Q>
__device__ void stage_tile_narrow(const DevParams& P, const StageArgs& A, int tile, SmemN<Q>& S) {
  constexpr int W = WN, NT = W * Q, NW = Q / 4;
  constexpr int RB = (Q + 15) / 16;  // row blocks of 16 output rows
  constexpr int KC = Q / 4;          // contraction steps of 4
  static_assert(2 * RB <= NW, "one Dp chain per wavefront");
  static_assert(NT >= 2 * MS_MAX + 1 + MF_MAX, "one thread per table entry");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int j = tid % W, k = tid / W;
  int off, nsys, i0;
  if (P.single) {
    off = 0;
    nsys = (int)P.ntot;
    i0 = tile * W;
  } else {
    const int4 td = P.tiles[tile];
    off = td.x;
    nsys = td.y;
    i0 = td.z;
  }
  const long long ntot = P.ntot;
  const int hn = P.hn;
  const bool valid = (i0 + j) < nsys;
  const long long gnode = off + i0 + j;

  // MFMA chains of this wavefront: Dp chain i < 2 RB (F then G, row block
  // i mod RB) and equilibrium chain rb < RB run on wavefront (1 + i) mod NW
  // and (1 + rb) mod NW (wavefront 0 computes the node fields)
  int chD = -1, chE = -1;
#pragma unroll
  for (int i = 0; i < 2 * RB; ++i)
    if ((1 + i) % NW == wave) chD = i;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
    if ((1 + rb) % NW == wave) chE = rb;
  const bool dchain = chD >= 0 && (P.term_mask & EVLB_TERM_FORCE);

  // ---- 1. load: one batch of global loads, then the LDS writes ----------
  double aD[KC], aE[KC];  // MFMA A operands: table rows 16 rb + (lane & 15)
  {
    const int rowD = 16 * (chD % RB) + (lane & 15), rowE = 16 * chE + (lane & 15);
#pragma unroll
    for (int b = 0; b < KC; ++b) {
      const int col = 4 * b + (lane >> 4);
      aD[b] = dchain && rowD < Q ? P.dpm[rowD * Q + col] : 0.0;
      aE[b] = chE >= 0 && rowE < Q ? P.meq[rowE * Q + col] : 0.0;
    }
  }
  const double pk = P.vel[k];
  double Fn = 0.0, Gn = 0.0;
  if (!A.first && !A.rhs_mode && valid) {
    Fn = A.f_n[(long long)k * ntot + gnode];
    Gn = A.f_n[(long long)(Q + k) * ntot + gnode];
  }
  constexpr int FW = W + 2 * HF;
  constexpr int NFV = 2 * Q * FW;
  constexpr int LF = (NFV + NT - 1) / NT;
  double fv[LF];
#pragma unroll
  for (int i = 0; i < LF; ++i) {
    const int idx = tid + i * NT;
    fv[i] = 0.0;
    if (idx < NFV) {
      const int r = idx / FW;
      fv[i] = A.f_prev[(long long)r * ntot + off + wrapi(i0 - HF + idx - r * FW, nsys)];
    }
  }
  const double* mn = A.mom_in;
  constexpr int LN = (W + 2 * HN_MAX + NT - 1) / NT;
  const int nwin = W + 2 * hn;
  double nv[LN];
#pragma unroll
  for (int i = 0; i < LN; ++i) {
    const int c = tid + i * NT;
    nv[i] = c < nwin ? mn[off + wrapi(i0 - hn + c, nsys)] : 0.0;
  }
  // thread c < W + 4 owns node i0 - 2 + c: u, T, q
  double uv = 0.0, Tv = 0.0, qv = 0.0;
  if (tid < W + 4) {
    const int node = off + wrapi(i0 - 2 + tid, nsys);
    uv = mn[ntot + node];
    Tv = mn[2 * ntot + node];
    qv = mn[3 * ntot + node];
  }
  // isothermal temperature of the own node's system (moment threads)
  double tiso = P.T_iso;
  if (P.tiso && tid < W && valid) tiso = P.tiso[gnode];
  // averaging weights and force taps: threads NT - 97 .. NT - 1
  constexpr int NSAV = 2 * MS_MAX + 1;
  const int e = tid - (NT - NSAV - MF_MAX);
  const double* src = nullptr;
  int si = 0;
  if (e >= 0 && e < 2 * P.ms + 1) { src = P.savg; si = e; }
  else if (e >= NSAV && e < NSAV + P.mf) { src = P.cfor; si = e - NSAV; }
  const double tv = src ? src[si] : 0.0;
#pragma unroll
  for (int i = 0; i < LF; ++i) {
    const int idx = tid + i * NT;
    if (idx < NFV) {
      const int r = idx / FW;
      S.f[r][idx - r * FW] = fv[i];
    }
  }
#pragma unroll
  for (int i = 0; i < LN; ++i) {
    const int c = tid + i * NT;
    if (c < nwin) S.n[c] = nv[i];
  }
  if (tid < W + 4) {
    S.u[tid] = uv;
    S.T[tid] = Tv;
  }
  if (e >= 0 && e < NSAV) S.sav[e] = tv;
  else if (e >= NSAV) S.cf[e - NSAV] = tv;
  __syncthreads();

  // ---- 2. contact value, transport, Hermite moments, force sums, faces ----
  // B operands of this wavefront's Dp chain, read before the faces
  double bD[KC];
#pragma unroll
  for (int b = 0; b < KC; ++b) bD[b] = 0.0;
  if (dchain) {
    const int brow = chD / RB == 1 ? Q : 0;
#pragma unroll
    for (int b = 0; b < KC; ++b) bD[b] = S.f[brow + 4 * b + (lane >> 4)][(lane & 15) + HF];
  }
  if (tid < W + 4) {
    // chi(nbar) and X = n^2 chi T on the tile +-2 (eq:carnstar)
    const int c = tid, cn = c + hn - 2;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int jj = -P.ms;
    for (; jj + 3 <= P.ms; jj += 4) {
      s0 += S.sav[jj + P.ms] * S.n[cn + jj];
      s1 += S.sav[jj + 1 + P.ms] * S.n[cn + jj + 1];
      s2 += S.sav[jj + 2 + P.ms] * S.n[cn + jj + 2];
      s3 += S.sav[jj + 3 + P.ms] * S.n[cn + jj + 3];
    }
    for (; jj <= P.ms; ++jj) s0 += S.sav[jj + P.ms] * S.n[cn + jj];
    const double eta = P.eta_c * ((s0 + s1) + (s2 + s3));
    const double om = 1.0 - eta;
    const double chi = (2.0 - eta) * rcpn(2.0 * om * om * om);
    const double nn = S.n[cn];
    S.chi[c] = chi;
    S.X[c] = nn * nn * chi * Tv;
    if (c >= 2 && c < W + 2) {
      // transport of the own node: mu (eq:viscosity), tau (eq:tau), Pr (eq:prandtl)
      const double bn = P.b * nn;
      const double y = bn * chi;
      const double mu0 = P.mu0c * sqrt(Tv);
      const double c12 = 0.16 * (1.0 + 12.0 / M_PI);
      const double c32 = 0.36 * (1.0 + 32.0 / (9.0 * M_PI));
      const double mu = mu0 * (rcpn(chi) + 0.8 * bn + c12 * bn * bn * chi);
      S.nf[NF_NU][c - 2] = chi * nn * Tv * (1.0 + 0.4 * y) * rcpn(mu);
      const double Pr = (2.0 / 3.0) * (1.0 + 0.6 * y) * (1.0 + 0.8 * y + c12 * y * y) *
                        rcpn((1.0 + 0.4 * y) * (1.0 + 1.2 * y + c32 * y * y));
      const double iT = rcpn(Tv);
      S.nf[NF_S][c - 2] = (1.0 - Pr) * qv * (0.2 * iT * iT) * rcpn(nn);
      S.nf[NF_PRE][c - 2] = -bn * chi;
    }
  }
  if (tid >= NT - W) {
    // Hermite moments a_0 = n, a_1 = n u, a_{l+1} = u a_l + l (T - 1) a_{l-1}
    const int jn = tid - (NT - W);
    const double n = S.n[jn + hn], u = S.u[jn + 2], tm1 = S.T[jn + 2] - 1.0;
    double am = n, a = n * u;
    S.a[0][jn] = am;
    S.a[1][jn] = a;
#pragma unroll
    for (int l = 1; l < Q - 1; ++l) {
      const double an = u * a + (double)l * tm1 * am;
      am = a;
      a = an;
      S.a[l + 1][jn] = a;
    }
  }
  if (P.force_model == EVLB_FORCE_EV1) {
    // node j, chunk k of the paired taps
    const int ch = (P.mf + Q - 1) / Q;
    const int m0 = 1 + k * ch;
    const int m1 = min(P.mf, m0 + ch - 1);
    const int cn = j + hn;
    double s0 = 0.0, s1 = 0.0;
    int m = m0;
    for (; m + 1 <= m1; m += 2) {
      s0 += S.cf[m - 1] * (S.n[cn + m] - S.n[cn - m]);
      s1 += S.cf[m] * (S.n[cn + m + 1] - S.n[cn - m - 1]);
    }
    if (m <= m1) s0 += S.cf[m - 1] * (S.n[cn + m] - S.n[cn - m]);
    S.fpart[k][j] = s0 + s1;
  }
  // WENO faces on the threads without contact-value or Hermite work.  With
  // six or more wavefronts the contact-value wavefront takes none, wavefronts
  // 1 .. NW-2 take FM faces per thread and the Hermite wavefront's other lanes
  // the rest, so that no wavefront runs many faces and the recurrence too.
  // Each face index is clamped into range and only the store is guarded, so
  // the faces of a thread are independent straight-line code.
  if (P.term_mask & EVLB_TERM_ADV) {
    constexpr int NFACE = 2 * Q * (W + 1);
    constexpr bool SPLIT = NT >= 384;
    constexpr int WS = SPLIT ? 64 : W + 4;            // first face thread
    constexpr int NMAIN = SPLIT ? 64 * (NW - 2) : NT - W - WS;
    constexpr int FM = SPLIT ? NFACE / NMAIN : (NFACE + NMAIN - 1) / NMAIN;
    constexpr int NREST = SPLIT ? NFACE - FM * NMAIN : 0;  // faces for the last wavefront
    static_assert(!SPLIT || NREST <= 64 - W, "the remaining faces fit the last wavefront");
    int base = -1, nf = 0, stride = 0;
    if (tid >= WS && tid < WS + NMAIN) {
      base = tid - WS;
      nf = FM;
      stride = NMAIN;
    } else if (SPLIT && tid >= 64 * (NW - 1) && tid < 64 * (NW - 1) + NREST) {
      base = FM * NMAIN + tid - 64 * (NW - 1);
      nf = 1;
      stride = 0;
    }
    // face idx of row r = idx / (W + 1): face i0 + jf - 1/2, upwind by the sign of p_k
    auto face = [&](int idx, bool keep) {
      const int r = idx / (W + 1);
      const int jf = idx - r * (W + 1);
      const int kr = r < Q ? r : r - Q;
      const bool pos = kr >= Q / 2;  // p_k > 0: upwind from the left
      const double* fr = &S.f[r][0];
      const int b0 = pos ? jf : jf + 5;
      const int st = pos ? 1 : -1;
      const double h = weno5<false>(fr[b0], fr[b0 + st], fr[b0 + 2 * st], fr[b0 + 3 * st], fr[b0 + 4 * st], P.weno_eps);
      if (keep) S.flux[r][jf] = h;
    };
    if (nf == FM) {  // whole wavefronts take this branch or the next
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int want = base + i * stride;
        const bool keep = want < NFACE;
        face(keep ? want : base, keep);
      }
    } else if (nf == 1) {
      face(base, true);
    }
  }
  if (dchain) {
    // (Dp F) or (Dp G) for one row block on the MFMA, as two independent
    // accumulation chains (even and odd contraction steps)
    const int p = 1 + chD / RB, rb = chD % RB;
    const int col = lane & 15, c = lane >> 4;
    dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < KC; b += 2) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(aD[b], bD[b], acc0, 0, 0, 0);
      if (b + 1 < KC) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(aD[b + 1], bD[b + 1], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * rb + 4 * r + c;
      if (row < Q) S.ctr[p][row][col] = acc0[r] + acc1[r];
    }
  }
  __syncthreads();

  // ---- 3. force and gradients (threads < 16); equilibrium (MFMA) ----------
  if (tid < W) {
    const int c = j + 2, cn = j + hn;
    const double idx12 = P.inv_dx * (1.0 / 12.0);
    double Fx = P.g_ext;
    if (P.force_model == EVLB_FORCE_EV1) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int g = 0; g + 1 < Q; g += 2) {
        s0 += S.fpart[g][j];
        s1 += S.fpart[g + 1][j];
      }
      Fx += s0 + s1;
    } else if (P.force_model == EVLB_FORCE_EV2) {
      const double d1 = (S.n[cn - 2] - 8.0 * S.n[cn - 1] + 8.0 * S.n[cn + 1] - S.n[cn + 2]) * idx12;
      const double d3 = (-S.n[cn - 2] + 2.0 * S.n[cn - 1] - 2.0 * S.n[cn + 1] + S.n[cn + 2]) *
                        (0.5 * P.inv_dx * P.inv_dx * P.inv_dx);
      Fx += P.two_a * d1 + P.kappa * d3;
    }
    const double T = S.T[c];
    S.nf[NF_A][j] = (S.X[c - 2] - 8.0 * S.X[c - 1] + 8.0 * S.X[c + 1] - S.X[c + 2]) * idx12 * rcpn(S.X[c]);
    S.nf[NF_B][j] = (S.T[c - 2] - 8.0 * S.T[c - 1] + 8.0 * S.T[c + 1] - S.T[c + 2]) * idx12 * rcpn(T);
    S.nf[NF_U1][j] = (S.u[c - 2] - 8.0 * S.u[c - 1] + 8.0 * S.u[c + 1] - S.u[c + 2]) * idx12;
    S.nf[NF_FX][j] = Fx;
    S.nf[NF_N][j] = S.n[cn];
    S.nf[NF_U][j] = S.u[c];
    S.nf[NF_T][j] = T;
  }
  if (chE >= 0) {
    const int col = lane & 15, c = lane >> 4;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < KC; ++b)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aE[b], S.a[4 * b + c][col], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * chE + 4 * r + c;
      if (row < Q) S.ctr[0][row][col] = acc[r];
    }
  }
  __syncthreads();

  // ---- 4. update -----------------------------------------------------------
  double pm[6];
  {
    const double u = S.nf[NF_U][j], T = S.nf[NF_T][j];
    const double nu = S.nf[NF_NU][j], sS = S.nf[NF_S][j], pre = S.nf[NF_PRE][j];
    const double Ag = S.nf[NF_A][j], Bg = S.nf[NF_B][j], Ug = S.nf[NF_U1][j];
    const double Fx = S.nf[NF_FX][j];
    const double invT = rcpn(T);
    const double E = S.ctr[0][k][j];
    const double F = S.f[k][j + HF];
    const double G = S.f[Q + k][j + HF];
    const double xi = pk - u;
    const double th = xi * xi * invT;
    double LF = 0.0, LG = 0.0;
    if (P.term_mask & EVLB_TERM_ADV) {
      LF = -pk * (S.flux[k][j + 1] - S.flux[k][j]) * P.inv_dx;
      LG = -pk * (S.flux[Q + k][j + 1] - S.flux[Q + k][j]) * P.inv_dx;
    }
    if (P.term_mask & EVLB_TERM_FORCE) {
      LF -= Fx * S.ctr[1][k][j];
      LG -= Fx * S.ctr[2][k][j];
    }
    if (P.term_mask & EVLB_TERM_J0) {
      const double FS = E * (1.0 + sS * xi * (th - 3.0));
      const double GS = T * E * (1.0 + sS * xi * (th - 1.0));
      LF -= nu * (F - FS);
      LG -= nu * (G - GS);
    }
    if (P.term_mask & EVLB_TERM_J1) {
      LF += pre * E * (xi * (Ag + 0.3 * (th - 3.0) * Bg) + 0.6 * (th - 1.0) * Ug);
      LG += pre * T * E * (xi * (Ag + 0.3 * (th - 1.0) * Bg) + 0.2 * (3.0 * th - 1.0) * Ug);
    }
    double Fo, Go;
    if (A.rhs_mode) {
      Fo = LF;
      Go = LG;
    } else {
      const double Fb = A.first ? F : Fn;
      const double Gb = A.first ? G : Gn;
      Fo = A.alpha * Fb + A.beta * (F + P.dt * LF);
      Go = A.alpha * Gb + A.beta * (G + P.dt * LG);
    }
    if (valid) {
      A.f_out[(long long)k * ntot + gnode] = Fo;
      A.f_out[(long long)(Q + k) * ntot + gnode] = Go;
    }
    const double p2 = pk * pk;
    pm[0] = Fo;
    pm[1] = pk * Fo;
    pm[2] = p2 * Fo;
    pm[3] = p2 * pk * Fo;
    pm[4] = Go;
    pm[5] = pk * Go;
  }
  if (A.rhs_mode) {
    __syncthreads();  // LDS is reused by the next tile
    return;
  }
  // the four velocities of a node within a wavefront: lanes j, j + 16, j + 32, j + 48
#pragma unroll
  for (int m = 0; m < 6; ++m) pm[m] = row4_sum(pm[m]);
  if (lane < W) {
#pragma unroll
    for (int m = 0; m < 6; ++m) S.red[wave][m][j] = pm[m];
  }
  __syncthreads();

  // ---- 5. moments of the new state --------------------------------------
  if (tid < W && valid) {
    double ms[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int w = 0; w + 1 < NW; w += 2) {
        s0 += S.red[w][m][tid];
        s1 += S.red[w + 1][m][tid];
      }
      if (NW & 1) s0 += S.red[NW - 1][m][tid];
      ms[m] = s0 + s1;
    }
    const double n = ms[0];
    const double in = rcpn(n);
    const double u = ms[1] * in;
    const double T = (2.0 / 3.0) * (0.5 * ms[2] + ms[4] - 0.5 * n * u * u) * in;
    const double x3 = ms[3] - 3.0 * u * ms[2] + 3.0 * u * u * ms[1] - u * u * u * n;
    const double q = 0.5 * x3 + ms[5] - u * ms[4];
    A.mom_out[gnode] = n;
    A.mom_out[ntot + gnode] = u;
    A.mom_out[2 * ntot + gnode] = tiso > 0.0 ? tiso : T;
    A.mom_out[3 * ntot + gnode] = q;
    if (!(n > 0.0) || !(T > 0.0) || !isfinite(n) || !isfinite(T) || !isfinite(q) || !isfinite(u))
      P.status[0] = 1;
  }
  __syncthreads();
}

// Workgroups go to the eight XCDs in turn (workgroup b to XCD b mod 8), and
// each XCD has its own L2.  xcd_tile gives XCD x the contiguous tiles
// x q + min(x, r) + i (ntiles = 8 q + r), so that tiles sharing halo and
// window lines, and a tile's own lines from one stage to the next, meet in
// one L2.  It is a bijection of 0 .. ntiles - 1.
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  const int q = ntiles >> 3, r = ntiles & 7;
  const int x = b & 7, i = b >> 3;
  return x * q + min(x, r) + i;
}

template <int Q, int W, int NG>
__global__ __launch_bounds__(W * NG) void stage_kernel(DevParams P, StageArgs A) {
  if constexpr (W == WN) {
    static_assert(NG == Q, "narrow tiles take one velocity per thread");
    __shared__ SmemN<Q> S;
    // every kernel argument into SGPRs before the first branch: one scalar
    // round trip at entry instead of one at each first use
    asm volatile("" ::"s"(P.meq), "s"(P.dpm), "s"(P.vel), "s"(P.savg), "s"(P.cfor), "s"(P.tiles), "s"(P.status),
                 "s"(P.ntiles), "s"(P.single), "s"(P.ms), "s"(P.mf), "s"(P.hn), "s"(P.ntot), "s"(P.force_model),
                 "s"(P.term_mask));
    asm volatile("" ::"s"(P.inv_dx), "s"(P.dt), "s"(P.b), "s"(P.eta_c), "s"(P.mu0c), "s"(P.weno_eps), "s"(P.g_ext),
                 "s"(P.two_a), "s"(P.kappa), "s"(P.T_iso), "s"(P.tiso));
    asm volatile("" ::"s"(A.f_prev), "s"(A.f_n), "s"(A.f_out), "s"(A.mom_in), "s"(A.mom_out), "s"(A.alpha),
                 "s"(A.beta), "s"(A.first), "s"(A.rhs_mode));
    // one tile per workgroup (the grid is the tile count): no loop, so no
    // wait at a loop head for loads still in flight
    if ((int)blockIdx.x < P.ntiles) stage_tile_narrow<Q>(P, A, xcd_tile(blockIdx.x, P.ntiles), S);
  } else {
    __shared__ Smem<Q, W, NG> S;
    load_tables<Q, W, NG>(P, S);
    if ((int)blockIdx.x < P.ntiles) stage_tile<Q, W, NG>(P, A, xcd_tile(blockIdx.x, P.ntiles), S);
  }
}

// ---------------------------------------------------------------------------
// Column shape: one wavefront per tile of WC = 63 nodes, thread = node.  Each
// thread keeps its node's F, G columns and Hermite moments in registers, so
// the q x q contractions (equilibrium, momentum derivative) need no LDS
// traffic and the velocity moments of the new state are a per-thread sum.
// The 64 lanes compute the 64 WENO-5 faces of a row (face j between nodes
// j-1 and j); a node's right face comes from the next lane by a shuffle.
// ---------------------------------------------------------------------------
constexpr int WC = 63;

// The density window is dead once the contact values and the forces are
// formed, and u, T and X of nodes -2..64 take its place: the tile then fits
// eight workgroups per CU (Q = 16).
template <int Q>
struct SmemCol {
  double f[2 * Q][WC + 2 * HF];      // columns: node i0 - 3 + c, c = 0..68
  union {
    double n[WC + 2 * HN_MAX];
    struct {
      double u[WC + 4], T[WC + 4], X[WC + 4];
    } g;
  } w;
  double sav[2 * MS_MAX + 1];        // averaging weights
  double cf[MF_MAX];                 // EV1 force taps
};

template <int Q>
__device__ void stage_tile_col(const DevParams& P, const StageArgs& A, int tile, SmemCol<Q>& S,
                               const double* __restrict__ vel, const double* __restrict__ meq,
                               const double* __restrict__ dpm) {
  const int lane = threadIdx.x;  // 0..63
  const int4 td = P.tiles[tile];
  const int off = td.x, nsys = td.y, i0 = td.z;
  const long long ntot = P.ntot;
  const int hn = P.hn;
  const bool valid = lane < WC && (i0 + lane) < nsys;
  const long long gnode = off + i0 + lane;

  // ---- 1. load: own column to registers and LDS, halo columns to LDS ----
  double Fc[Q], Gc[Q];
  {
    const long long gown = off + wrapi(i0 + lane, nsys);  // lane 63: right halo node 63
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      Fc[k] = A.f_prev[(long long)k * ntot + gown];
      Gc[k] = A.f_prev[(long long)(Q + k) * ntot + gown];
    }
    // halo columns 0, 1, 2 (nodes -3..-1) and 67, 68 (nodes 64, 65) of all
    // 2Q rows, spread over the lanes: a few loads per lane instead of 2Q on
    // five lanes
    constexpr int NH = 5 * 2 * Q, LH = (NH + 63) / 64;
    double hv[LH];
#pragma unroll
    for (int i = 0; i < LH; ++i) {
      const int idx = lane + 64 * i;
      hv[i] = 0.0;
      if (idx < NH) {
        const int r = idx / 5, h = idx - 5 * r;
        const int c = h < 3 ? h : h + 64;
        hv[i] = A.f_prev[(long long)r * ntot + off + wrapi(i0 - HF + c, nsys)];
      }
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      S.f[k][lane + HF] = Fc[k];
      S.f[Q + k][lane + HF] = Gc[k];
    }
#pragma unroll
    for (int i = 0; i < LH; ++i) {
      const int idx = lane + 64 * i;
      if (idx < NH) {
        const int r = idx / 5, h = idx - 5 * r;
        S.f[r][h < 3 ? h : h + 64] = hv[i];
      }
    }
  }
  // density window, u and T on nodes -2..64, the averaging and force tables:
  // all loads issued before the first LDS write
  const double* mn = A.mom_in;
  constexpr int LN = (WC + 2 * HN_MAX + 63) / 64;
  constexpr int LU = (WC + 4 + 63) / 64;
  static_assert(LU == 2, "nodes -2..64 on one or two values per lane");
  constexpr int NSAV = 2 * MS_MAX + 1;
  constexpr int LT = (NSAV + MF_MAX + 63) / 64;
  const int nwin = WC + 2 * hn;
  double nv[LN], uv[LU], Tv[LU], tv[LT];
#pragma unroll
  for (int i = 0; i < LN; ++i) {
    const int c = lane + 64 * i;
    nv[i] = c < nwin ? mn[off + wrapi(i0 - hn + c, nsys)] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < LU; ++i) {
    const int c = lane + 64 * i;
    uv[i] = 0.0;
    Tv[i] = 0.0;
    if (c < WC + 4) {
      const int node = off + wrapi(i0 - 2 + c, nsys);
      uv[i] = mn[ntot + node];
      Tv[i] = mn[2 * ntot + node];
    }
  }
#pragma unroll
  for (int i = 0; i < LT; ++i) {
    const int e = lane + 64 * i;
    const double* src = nullptr;
    int si = 0;
    if (e < 2 * P.ms + 1) { src = P.savg; si = e; }
    else if (e >= NSAV && e < NSAV + P.mf) { src = P.cfor; si = e - NSAV; }
    tv[i] = src ? src[si] : 0.0;
  }
  const double qj = valid ? mn[3 * ntot + gnode] : 0.0;
  const double tiso = P.tiso && valid ? P.tiso[gnode] : P.T_iso;
#pragma unroll
  for (int i = 0; i < LN; ++i) {
    const int c = lane + 64 * i;
    if (c < nwin) S.w.n[c] = nv[i];
  }
#pragma unroll
  for (int i = 0; i < LT; ++i) {
    const int e = lane + 64 * i;
    if (e < NSAV) S.sav[e] = tv[i];
    else if (e < NSAV + MF_MAX) S.cf[e - NSAV] = tv[i];
  }
  __syncthreads();

  // ---- 2. contact value and X = n^2 chi T on nodes -2..64 (c = lane, and
  // c = lane + 64 on lanes 0..2), kept in registers ------------------------
  double chv[LU], Xv[LU];
#pragma unroll
  for (int i = 0; i < LU; ++i) {
    const int cc = lane + 64 * i;
    chv[i] = 1.0;
    Xv[i] = 1.0;
    if (cc < WC + 4) {
      const int cn = cc + hn - 2;
      double s0 = 0.0, s1 = 0.0;
      int jj = -P.ms;
      for (; jj + 1 <= P.ms; jj += 2) {
        s0 += S.sav[jj + P.ms] * S.w.n[cn + jj];
        s1 += S.sav[jj + 1 + P.ms] * S.w.n[cn + jj + 1];
      }
      if (jj <= P.ms) s0 += S.sav[jj + P.ms] * S.w.n[cn + jj];
      const double eta = P.eta_c * (s0 + s1);
      const double om = 1.0 - eta;
      chv[i] = (2.0 - eta) * rcpn(2.0 * om * om * om);
      const double nn = S.w.n[cn];
      Xv[i] = nn * nn * chv[i] * Tv[i];
    }
  }

  // ---- 3. node fields of the own node -------------------------------------
  const int jw = lane < WC ? lane : WC - 1;  // lane 63 mirrors lane 62 (no node)
  const int c = jw + 2, cn = jw + hn;
  const double n = S.w.n[cn];
  const double idx12 = P.inv_dx * (1.0 / 12.0);
  double Fx = P.g_ext;
  if (P.force_model == EVLB_FORCE_EV1) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int m = 1;
    for (; m + 3 <= P.mf; m += 4) {
      s0 += S.cf[m - 1] * (S.w.n[cn + m] - S.w.n[cn - m]);
      s1 += S.cf[m] * (S.w.n[cn + m + 1] - S.w.n[cn - m - 1]);
      s2 += S.cf[m + 1] * (S.w.n[cn + m + 2] - S.w.n[cn - m - 2]);
      s3 += S.cf[m + 2] * (S.w.n[cn + m + 3] - S.w.n[cn - m - 3]);
    }
    for (; m <= P.mf; ++m) s0 += S.cf[m - 1] * (S.w.n[cn + m] - S.w.n[cn - m]);
    Fx += (s0 + s1) + (s2 + s3);
  } else if (P.force_model == EVLB_FORCE_EV2) {
    const double d1 = (S.w.n[cn - 2] - 8.0 * S.w.n[cn - 1] + 8.0 * S.w.n[cn + 1] - S.w.n[cn + 2]) * idx12;
    const double d3 = (-S.w.n[cn - 2] + 2.0 * S.w.n[cn - 1] - 2.0 * S.w.n[cn + 1] + S.w.n[cn + 2]) *
                      (0.5 * P.inv_dx * P.inv_dx * P.inv_dx);
    Fx += P.two_a * d1 + P.kappa * d3;
  }
  __syncthreads();  // the density window is dead: u, T and X take its place
#pragma unroll
  for (int i = 0; i < LU; ++i) {
    const int cc = lane + 64 * i;
    if (cc < WC + 4) {
      S.w.g.u[cc] = uv[i];
      S.w.g.T[cc] = Tv[i];
      S.w.g.X[cc] = Xv[i];
    }
  }
  // chi of the own node (c = jw + 2) from the lane that formed it
  const int csrc = c < 64 ? c : c - 64;
  const double chA = __shfl(chv[0], csrc), chB = __shfl(chv[LU - 1], csrc);
  const double chi = c < 64 ? chA : chB;
  __syncthreads();
  const double u = S.w.g.u[c], T = S.w.g.T[c];
  const double invT = rcpn(T);
  const double* Xs = S.w.g.X;
  const double* Ts = S.w.g.T;
  const double* us = S.w.g.u;
  const double Ag = (Xs[c - 2] - 8.0 * Xs[c - 1] + 8.0 * Xs[c + 1] - Xs[c + 2]) * idx12 * rcpn(Xs[c]);
  const double Bg = (Ts[c - 2] - 8.0 * Ts[c - 1] + 8.0 * Ts[c + 1] - Ts[c + 2]) * idx12 * invT;
  const double Ug = (us[c - 2] - 8.0 * us[c - 1] + 8.0 * us[c + 1] - us[c + 2]) * idx12;
  const double bn = P.b * n;
  const double y = bn * chi;
  const double c12 = 0.16 * (1.0 + 12.0 / M_PI);
  const double c32 = 0.36 * (1.0 + 32.0 / (9.0 * M_PI));
  const double mu = P.mu0c * sqrt(T) * (rcpn(chi) + 0.8 * bn + c12 * bn * bn * chi);
  const double nu = chi * n * T * (1.0 + 0.4 * y) * rcpn(mu);
  const double Pr = (2.0 / 3.0) * (1.0 + 0.6 * y) * (1.0 + 0.8 * y + c12 * y * y) *
                    rcpn((1.0 + 0.4 * y) * (1.0 + 1.2 * y + c32 * y * y));
  const double sS = (1.0 - Pr) * qj * (0.2 * invT * invT) * rcpn(n);
  const double pre = -bn * chi;
  // Hermite moments a_0 = n, a_1 = n u, a_{l+1} = u a_l + l (T - 1) a_{l-1}
  double a[Q];
  a[0] = n;
  a[1] = n * u;
#pragma unroll
  for (int l = 1; l < Q - 1; ++l) a[l + 1] = u * a[l] + (double)l * (T - 1.0) * a[l - 1];

  // ---- 4. update, velocity by velocity -----------------------------------
  double pm[6] = {0, 0, 0, 0, 0, 0};
  const bool adv = P.term_mask & EVLB_TERM_ADV;
  const bool frc = P.term_mask & EVLB_TERM_FORCE;
  const bool j0 = P.term_mask & EVLB_TERM_J0;
  const bool j1 = P.term_mask & EVLB_TERM_J1;
  // Shakhov relaxation and J1 of velocity k: -nu f_k + E_k c(xi) with
  // xi = p_k - u and a cubic c per node and distribution.  For F,
  //   nu (1 + sS xi (xi^2/T - 3)) + pre (xi (A + 0.3 (xi^2/T - 3) B) + 0.6 (xi^2/T - 1) U),
  // for G,
  //   nu T (1 + sS xi (xi^2/T - 1)) + pre T (xi (A + 0.3 (xi^2/T - 1) B) + 0.2 (3 xi^2/T - 1) U),
  // expanded in powers of xi.
  const double nu0 = j0 ? nu : 0.0, sv = j0 ? nu * sS : 0.0;
  const double pA = j1 ? pre * Ag : 0.0, pB = j1 ? pre * Bg : 0.0, pU = j1 ? pre * Ug : 0.0;
  const double cF0 = nu0 - 0.6 * pU, cF1 = pA - 3.0 * sv - 0.9 * pB;
  const double cF2 = 0.6 * pU * invT, cF3 = (sv + 0.3 * pB) * invT;
  const double cG0 = T * (nu0 - 0.2 * pU), cG1 = T * (pA - sv - 0.3 * pB);
  const double cG2 = 0.6 * pU, cG3 = sv + 0.3 * pB;
#pragma unroll 1
  for (int k = 0; k < Q; ++k) {
    double Fb = 0.0, Gb = 0.0;
    if (!A.first && !A.rhs_mode && valid) {
      Fb = A.f_n[(long long)k * ntot + gnode];
      Gb = A.f_n[(long long)(Q + k) * ntot + gnode];
    }
    const double pk = vel[k];
    double LF = 0.0, LG = 0.0;
    if (adv) {
      // face `lane` of rows k (F) and Q + k (G); upwind by the sign of p_k
      const bool pos = k >= Q / 2;
      const int b0 = pos ? lane : lane + 5;
      const int st = pos ? 1 : -1;
      const double* fr = &S.f[k][0];
      const double* gr = &S.f[Q + k][0];
      const double hF = weno5<true>(fr[b0], fr[b0 + st], fr[b0 + 2 * st], fr[b0 + 3 * st], fr[b0 + 4 * st], P.weno_eps);
      const double hG = weno5<true>(gr[b0], gr[b0 + st], gr[b0 + 2 * st], gr[b0 + 3 * st], gr[b0 + 4 * st], P.weno_eps);
      const double hFr = wave_next(hF);  // lane 63's faces are not used
      const double hGr = wave_next(hG);
      LF = -pk * (hFr - hF) * P.inv_dx;
      LG = -pk * (hGr - hG) * P.inv_dx;
    }
    double E0 = 0.0, E1 = 0.0;
    const double* mrow = meq + k * Q;
#pragma unroll
    for (int l = 0; l < Q; l += 2) {
      E0 += mrow[l] * a[l];
      E1 += mrow[l + 1] * a[l + 1];
    }
    const double E = E0 + E1;
    const double Fk = S.f[k][lane + HF];
    const double Gk = S.f[Q + k][lane + HF];
    if (frc) {
      const double* drow = dpm + k * Q;
      double dF0 = 0.0, dF1 = 0.0, dG0 = 0.0, dG1 = 0.0;
#pragma unroll
      for (int kk = 0; kk < Q; kk += 2) {
        dF0 += drow[kk] * Fc[kk];
        dF1 += drow[kk + 1] * Fc[kk + 1];
        dG0 += drow[kk] * Gc[kk];
        dG1 += drow[kk + 1] * Gc[kk + 1];
      }
      LF -= Fx * (dF0 + dF1);
      LG -= Fx * (dG0 + dG1);
    }
    const double xi = pk - u;
    const double qF = fma(fma(fma(cF3, xi, cF2), xi, cF1), xi, cF0);
    const double qG = fma(fma(fma(cG3, xi, cG2), xi, cG1), xi, cG0);
    LF = fma(E, qF, fma(-nu0, Fk, LF));
    LG = fma(E, qG, fma(-nu0, Gk, LG));
    double Fo, Go;
    if (A.rhs_mode) {
      Fo = LF;
      Go = LG;
    } else {
      if (A.first) {
        Fb = Fk;
        Gb = Gk;
      }
      Fo = A.alpha * Fb + A.beta * (Fk + P.dt * LF);
      Go = A.alpha * Gb + A.beta * (Gk + P.dt * LG);
    }
    if (valid) {
      A.f_out[(long long)k * ntot + gnode] = Fo;
      A.f_out[(long long)(Q + k) * ntot + gnode] = Go;
    }
    const double p2 = pk * pk;
    pm[0] += Fo;
    pm[1] += pk * Fo;
    pm[2] += p2 * Fo;
    pm[3] += p2 * pk * Fo;
    pm[4] += Go;
    pm[5] += pk * Go;
  }

  // ---- 5. moments of the new state ----------------------------------------
  if (!A.rhs_mode && valid) {
    const double n1 = pm[0];
    const double in1 = rcpn(n1);
    const double u1 = pm[1] * in1;
    const double T1 = (2.0 / 3.0) * (0.5 * pm[2] + pm[4] - 0.5 * n1 * u1 * u1) * in1;
    const double x3 = pm[3] - 3.0 * u1 * pm[2] + 3.0 * u1 * u1 * pm[1] - u1 * u1 * u1 * n1;
    const double q1 = 0.5 * x3 + pm[5] - u1 * pm[4];
    A.mom_out[gnode] = n1;
    A.mom_out[ntot + gnode] = u1;
    A.mom_out[2 * ntot + gnode] = tiso > 0.0 ? tiso : T1;
    A.mom_out[3 * ntot + gnode] = q1;
    if (!(n1 > 0.0) || !(T1 > 0.0) || !isfinite(n1) || !isfinite(T1) || !isfinite(q1) || !isfinite(u1))
      P.status[0] = 1;
  }
  __syncthreads();
}

template <int Q>
__global__ __launch_bounds__(64) void stage_kernel_col(DevParams P, StageArgs A, const double* __restrict__ vel,
                                                       const double* __restrict__ meq,
                                                       const double* __restrict__ dpm) {
  __shared__ SmemCol<Q> S;
  // one tile per workgroup (the grid is the tile count)
  if ((int)blockIdx.x < P.ntiles) stage_tile_col<Q>(P, A, xcd_tile(blockIdx.x, P.ntiles), S, vel, meq, dpm);
}

// Grid-wide barrier for the persistent kernel (all workgroups co-resident:
// cooperative launch).  A monotonically increasing arrival counter: barrier
// number e completes when the counter reaches (e + 1) * nblocks.  An
// agent-scope release fence before the arrival and an acquire fence after
// the wait make each stage's global writes, from every XCD, visible to all
// workgroups.  The wait is bounded: on time-out the abort latch is set and
// every workgroup leaves its step loop.
__device__ bool grid_barrier(const DevParams& P, unsigned nblocks, unsigned epoch) {
  __syncthreads();
  __shared__ int s_ok;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(P.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = (epoch + 1u) * nblocks;
    int ok = 1;
    long long spins = 0;
    while ((int)(__hip_atomic_load(P.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 1023) == 0) {
        if (spins > (1ll << 24) ||
            __hip_atomic_load(P.status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          __hip_atomic_store(P.status + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Resets the barrier counter and the abort latch (a kernel rather than a
// memset so that the sequence stays valid under stream capture).
__global__ void clear_barrier_kernel(DevParams P) {
  if (threadIdx.x == 0) {
    P.bar[0] = 0u;
    P.bar[1] = 0u;
    P.status[1] = 0;
  }
}

struct PersistArgs {
  double* f;            // f^n in/out
  double* f1;
  double* f2;
  double* momA;
  double* momB;         // momA holds the moments of f on entry
  int nsteps;
};

// Persistent kernel: all stages of nsteps steps in one cooperative launch,
// workgroups separated by grid barriers between stages.
template <int Q, int W, int NG>
struct GroupShape {
  static constexpr int NT = W * NG;
  typedef std::conditional_t<W == WN, SmemN<Q>, Smem<Q, W, NG>> Shared;
  __device__ static void prologue(const DevParams& P, Shared& S) {
    if constexpr (W != WN) load_tables<Q, W, NG>(P, S);
  }
  __device__ static void tile(const DevParams& P, const StageArgs& A, int t, Shared& S, const double*,
                              const double*, const double*) {
    if constexpr (W == WN) stage_tile_narrow<Q>(P, A, t, S);
    else stage_tile<Q, W, NG>(P, A, t, S);
  }
};

template <int Q>
struct ColumnShape {
  static constexpr int NT = 64;
  typedef SmemCol<Q> Shared;
  __device__ static void prologue(const DevParams&, Shared&) {}
  __device__ static void tile(const DevParams& P, const StageArgs& A, int t, Shared& S,
                              const double* __restrict__ vel, const double* __restrict__ meq,
                              const double* __restrict__ dpm) {
    stage_tile_col<Q>(P, A, t, S, vel, meq, dpm);
  }
};

template <class SHAPE>
__global__ __launch_bounds__(SHAPE::NT) void persistent_kernel(DevParams P, PersistArgs R,
                                                               const double* __restrict__ vel,
                                                               const double* __restrict__ meq,
                                                               const double* __restrict__ dpm) {
  __shared__ typename SHAPE::Shared S;
  SHAPE::prologue(P, S);
  const double a_s[3] = {0.0, 0.75, 1.0 / 3.0};
  const double b_s[3] = {1.0, 0.25, 2.0 / 3.0};
  unsigned epoch = 0;
  for (int step = 0; step < R.nsteps; ++step) {
    for (int s = 0; s < 3; ++s) {
      StageArgs A;
      A.f_prev = s == 0 ? R.f : (s == 1 ? R.f1 : R.f2);
      A.f_n = R.f;
      A.f_out = s == 0 ? R.f1 : (s == 1 ? R.f2 : R.f);
      const int parity = (step * 3 + s) & 1;
      A.mom_in = parity ? R.momB : R.momA;
      A.mom_out = parity ? R.momA : R.momB;
      A.alpha = a_s[s];
      A.beta = b_s[s];
      A.first = s == 0;
      A.rhs_mode = 0;
      for (int b = blockIdx.x; b < P.ntiles; b += gridDim.x) SHAPE::tile(P, A, xcd_tile(b, P.ntiles), S, vel, meq, dpm);
      if (!grid_barrier(P, gridDim.x, epoch++)) return;
    }
  }
}

// Moments of a state, one thread per node (also the entry moments of a step).
template <int Q>
__global__ __launch_bounds__(256) void moments_kernel(DevParams P, const double* __restrict__ f,
                                                      double* __restrict__ n_out, double* __restrict__ u_out,
                                                      double* __restrict__ T_out, double* __restrict__ q_out,
                                                      int stage_input) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.ntot) return;
  const long long nt = P.ntot;
  double F[Q], G[Q];
  double n = 0.0, m1 = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    F[k] = f[k * nt + i];
    G[k] = f[(Q + k) * nt + i];
    n += F[k];
    m1 += P.vel[k] * F[k];
  }
  const double u = m1 / n;
  double e = 0.0, q = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const double xi = P.vel[k] - u;
    const double ek = 0.5 * xi * xi * F[k] + G[k];
    e += ek;
    q += xi * ek;
  }
  const double T = (2.0 / 3.0) * e / n;
  n_out[i] = n;
  u_out[i] = u;
  // as the input of a stage, an isothermal run sees its fixed temperature
  const double tiso = stage_input ? (P.tiso ? P.tiso[i] : P.T_iso) : 0.0;
  T_out[i] = tiso > 0.0 ? tiso : T;
  if (q_out) q_out[i] = q;
}

// Reduced Maxwellian F = E(n, u, T), G = T E, one thread per node.
template <int Q>
__global__ __launch_bounds__(256) void equilibrium_kernel(DevParams P, const double* __restrict__ n_in,
                                                          const double* __restrict__ u_in,
                                                          const double* __restrict__ T_in,
                                                          double* __restrict__ f) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.ntot) return;
  const long long nt = P.ntot;
  const double n = n_in[i], u = u_in[i], T = T_in[i];
  double a[Q];
  a[0] = n;
  a[1] = n * u;
#pragma unroll
  for (int l = 1; l < Q - 1; ++l) a[l + 1] = u * a[l] + (double)l * (T - 1.0) * a[l - 1];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    double E = 0.0;
#pragma unroll
    for (int l = 0; l < Q; ++l) E += P.meq[k * Q + l] * a[l];
    f[k * nt + i] = E;
    f[(Q + k) * nt + i] = T * E;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

#include "adjoint.inc"

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int WIDE = 64;    // tile width for large grids
constexpr int NARROW = WN;  // tile width for grids too small to fill the chip

struct Layout {
  size_t tables, tiles_wide, tiles_narrow, tiles_col, tiles_adj, f1, f2, momA, momB, status, tiso;
  size_t adj_g, adj_mu2, adj_mu1, adj_fa, adj_fb, adj_mom, adj_part, adj_lam, total;
  long long ntot;
  int ntiles_wide, ntiles_narrow, ntiles_col, ntiles_adj, ms, mf;
  size_t ntables;
};

int count_tiles(const evlb_params* p, int w) {
  int t = 0;
  for (int s = 0; s < p->n_sys; ++s) t += (p->nx[s] + w - 1) / w;
  return t;
}

bool is_even_multiple(double a, double dx, int* m, double tol = 1e-9) {
  const double r = a / dx;
  const long long k = llround(r);
  if (k <= 0 || std::fabs(r - (double)k) > tol * r || (k & 1)) return false;
  *m = (int)k;
  return true;
}

int validate(const evlb_params* p) {
  if (!p) return EVLB_EINVAL;
  if (p->abi_version != EVLB_ABI_VERSION) return EVLB_EINVAL;
  if (p->dim == 2) return p->T_iso_sys ? EVLB_EUNSUPPORTED : evlb2d::validate(p);
  if (p->dim != 1) return EVLB_EUNSUPPORTED;
  if (p->n_sys < 1 || !p->nx) return EVLB_EINVAL;
  long long ntot = 0;
  for (int s = 0; s < p->n_sys; ++s) {
    if (p->nx[s] < 8) return EVLB_EINVAL;
    ntot += p->nx[s];
  }
  if (ntot > (1ll << 31) - 1) return EVLB_EINVAL;
  if (p->q != 8 && p->q != 16 && p->q != 24) return EVLB_EUNSUPPORTED;
  if (!(p->dx > 0) || !(p->dt > 0) || !std::isfinite(p->dx) || !std::isfinite(p->dt)) return EVLB_EINVAL;
  if (!(p->sigma > 0) || !(p->phi_sigma >= 0) || !std::isfinite(p->phi_sigma)) return EVLB_EINVAL;
  if (!(p->gamma > 3.0)) return EVLB_EINVAL;
  if (p->force_model == EVLB_FORCE_EV2 && !(p->gamma > 5.0)) return EVLB_EINVAL;
  if (p->force_model < 0 || p->force_model > 2) return EVLB_EINVAL;
  if (p->term_mask & ~EVLB_TERM_ALL) return EVLB_EINVAL;
  if (!(p->weno_eps > 0) || !std::isfinite(p->g_ext)) return EVLB_EINVAL;
  if (p->exec_mode < 0 || p->exec_mode > 2) return EVLB_EINVAL;
  if (p->adjoint != 0 && p->adjoint != 1) return EVLB_EINVAL;
  if (p->adjoint && p->force_model == EVLB_FORCE_EV2) return EVLB_EUNSUPPORTED;
  if (!(p->T_iso >= 0.0) || !std::isfinite(p->T_iso)) return EVLB_EINVAL;
  if (p->adjoint && p->T_iso > 0.0) return EVLB_EUNSUPPORTED;
  if (p->T_iso_sys) {
    for (int s = 0; s < p->n_sys; ++s) {
      const double t = p->T_iso_sys[s];
      if (!(t >= 0.0) || !std::isfinite(t)) return EVLB_EINVAL;
      if (p->adjoint && t > 0.0) return EVLB_EUNSUPPORTED;
    }
  }
  if (p->tile_nodes != 0 && p->tile_nodes != WIDE && p->tile_nodes != NARROW && p->tile_nodes != WC)
    return EVLB_EINVAL;
  int ms, mf = 0;
  // the averaging window is the nearest even number of cells; sigma may sit
  // slightly off it (derivatives with respect to sigma at a fixed window)
  if (!is_even_multiple(p->sigma, p->dx, &ms, 1e-3) || ms > MS_MAX) return EVLB_EINVAL;
  if (p->force_model == EVLB_FORCE_EV1) {
    if (!is_even_multiple(p->r_cut, p->dx, &mf) || mf > MF_MAX) return EVLB_EINVAL;
  }
  // stability of WENO-5 + TVD-RK3 advection: CFL number <= 1
  std::vector<double> v, w;
  evlb::gauss_hermite_nodes(p->q, v, w);
  if (p->dt * v.back() / p->dx > 1.0) return EVLB_ECFL;
  return EVLB_OK;
}

Layout make_layout(const evlb_params* p) {
  Layout L{};
  L.ntot = 0;
  for (int s = 0; s < p->n_sys; ++s) L.ntot += p->nx[s];
  L.ntiles_wide = count_tiles(p, WIDE);
  L.ntiles_narrow = count_tiles(p, NARROW);
  L.ntiles_col = count_tiles(p, WC);
  L.ntiles_adj = count_tiles(p, WA);
  L.ms = (int)llround(p->sigma / p->dx);
  L.mf = p->force_model == EVLB_FORCE_EV1 ? (int)llround(p->r_cut / p->dx) : 0;
  const int q = p->q;
  size_t off = 0;
  L.tables = off;
  const int mfa = L.mf > 0 ? L.mf : 1;
  L.ntables = (size_t)(q + 2 * q * q + 2 * (2 * L.ms + 1) + 3 * mfa);
  off += align256(sizeof(double) * L.ntables);
  L.tiles_wide = off;
  off += align256(sizeof(int4) * (size_t)L.ntiles_wide);
  L.tiles_narrow = off;
  off += align256(sizeof(int4) * (size_t)L.ntiles_narrow);
  L.tiles_col = off;
  off += align256(sizeof(int4) * (size_t)L.ntiles_col);
  L.tiles_adj = off;
  off += align256(sizeof(int4) * (size_t)L.ntiles_adj);
  const size_t fbytes = align256(sizeof(double) * 2 * (size_t)q * (size_t)L.ntot);
  L.f1 = off; off += fbytes;
  L.f2 = off; off += fbytes;
  const size_t mbytes = align256(sizeof(double) * 4 * (size_t)L.ntot);
  L.momA = off; off += mbytes;
  L.momB = off; off += mbytes;
  L.status = off; off += 256;
  L.tiso = 0;
  if (p->T_iso_sys) {
    L.tiso = off;
    off += align256(sizeof(double) * (size_t)L.ntot);
  }
  if (p->adjoint) {
    L.adj_g = off; off += fbytes;
    L.adj_mu2 = off; off += fbytes;
    L.adj_mu1 = off; off += fbytes;
    L.adj_fa = off; off += align256(sizeof(double) * NFA * (size_t)L.ntot);
    L.adj_fb = off; off += align256(sizeof(double) * NFB * (size_t)L.ntot);
    L.adj_mom = off; off += mbytes;
    // parameter partials: per VJP one slot per field-adjoint tile (16 nodes) and per node tile, for two
    // steps (a step's partials are summed while the next step runs)
    L.adj_part = off; off += align256(sizeof(double) * 2 * 2 * 3 * (size_t)(L.ntiles_narrow + L.ntiles_adj));
    L.adj_lam = off; off += fbytes;
  }
  L.total = off;
  return L;
}

}  // namespace

struct evlb_ctx {
  evlb_params p;
  std::vector<int32_t> nx;
  std::vector<double> vel;
  std::vector<double> tiso;  // per-system isothermal temperatures (copy of T_iso_sys)
  Layout L;
  DevParams dp;  // tiles/ntiles of the wide shape; launches patch them
  char* ws;
  int device;
  int cus;
  evlb2d::Ctx* c2 = nullptr;  // dim = 2 path
};

namespace {

#define EVLB_HIP(call)                         \
  do {                                         \
    if ((call) != hipSuccess) return EVLB_EHIP; \
  } while (0)

// launch shapes per quadrature order: wide tiles (64 nodes, NG groups) and
// narrow tiles (16 nodes, one velocity per thread)
template <int Q> struct WideNG;
template <> struct WideNG<8> { static constexpr int v = 4; };
template <> struct WideNG<16> { static constexpr int v = 8; };
template <> struct WideNG<24> { static constexpr int v = 8; };

DevParams params_for(const evlb_ctx* c, int w) {
  DevParams P = c->dp;
  if (w == NARROW) {
    P.tiles = (const int4*)(c->ws + c->L.tiles_narrow);
    P.ntiles = c->L.ntiles_narrow;
  } else if (w == WC) {
    P.tiles = (const int4*)(c->ws + c->L.tiles_col);
    P.ntiles = c->L.ntiles_col;
  } else {
    P.tiles = (const int4*)(c->ws + c->L.tiles_wide);
    P.ntiles = c->L.ntiles_wide;
  }
  return P;
}

template <int Q, int W, int NG>
int launch_stage(evlb_ctx* c, const StageArgs& A, hipStream_t st) {
  const DevParams P = params_for(c, W);
  hipLaunchKernelGGL((stage_kernel<Q, W, NG>), dim3(P.ntiles), dim3(W * NG), 0, st, P, A);
  return hipGetLastError() == hipSuccess ? EVLB_OK : EVLB_EHIP;
}

template <int Q>
int launch_stage_col(evlb_ctx* c, const StageArgs& A, hipStream_t st) {
  const DevParams P = params_for(c, WC);
  hipLaunchKernelGGL((stage_kernel_col<Q>), dim3(P.ntiles), dim3(64), 0, st, P, A, P.vel, P.meq, P.dpm);
  return hipGetLastError() == hipSuccess ? EVLB_OK : EVLB_EHIP;
}

template <class SHAPE>
int launch_persistent(evlb_ctx* c, int width, double* f, int nsteps, hipStream_t st) {
  int per_cu = 0;
  EVLB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_kernel<SHAPE>, SHAPE::NT, 0));
  if (per_cu < 1) return EVLB_EHIP;
  DevParams P = params_for(c, width);
  int grid = per_cu * c->cus;
  if (grid > P.ntiles) grid = P.ntiles;
  PersistArgs R;
  R.f = f;
  R.f1 = (double*)(c->ws + c->L.f1);
  R.f2 = (double*)(c->ws + c->L.f2);
  R.momA = (double*)(c->ws + c->L.momA);
  R.momB = (double*)(c->ws + c->L.momB);
  R.nsteps = nsteps;
  hipLaunchKernelGGL(clear_barrier_kernel, dim3(1), dim3(64), 0, st, P);
  EVLB_HIP(hipGetLastError());
  const double* vel = P.vel;
  const double* meq = P.meq;
  const double* dpm = P.dpm;
  void* args[] = {&P, &R, &vel, &meq, &dpm};
  EVLB_HIP(hipLaunchCooperativeKernel((const void*)persistent_kernel<SHAPE>, dim3(grid), dim3(SHAPE::NT), args, 0, st));
  return EVLB_OK;
}

template <int Q>
int run_moments(evlb_ctx* c, const double* f, double* n, double* u, double* T, double* q, hipStream_t st,
                int stage_input = 1) {
  const long long nt = c->L.ntot;
  const int blocks = (int)((nt + 255) / 256);
  hipLaunchKernelGGL((moments_kernel<Q>), dim3(blocks), dim3(256), 0, st, c->dp, f, n, u, T, q, stage_input);
  return hipGetLastError() == hipSuccess ? EVLB_OK : EVLB_EHIP;
}

// tile shape: explicit, or the column shape when it yields at least four
// wavefronts per CU, else the narrow shape (small grids, latency bound)
int pick_width(const evlb_ctx* c) {
  if (c->p.tile_nodes) return c->p.tile_nodes;
  return c->L.ntiles_col >= 4 * c->cus ? WC : NARROW;
}

StageArgs stage_args(double* f, double* f1, double* f2, double* momA, double* momB, int step, int s) {
  const double a_s[3] = {0.0, 0.75, 1.0 / 3.0};
  const double b_s[3] = {1.0, 0.25, 2.0 / 3.0};
  StageArgs A;
  A.f_prev = s == 0 ? f : (s == 1 ? f1 : f2);
  A.f_n = f;
  A.f_out = s == 0 ? f1 : (s == 1 ? f2 : f);
  const int parity = (step * 3 + s) & 1;
  A.mom_in = parity ? momB : momA;
  A.mom_out = parity ? momA : momB;
  A.alpha = a_s[s];
  A.beta = b_s[s];
  A.first = s == 0;
  A.rhs_mode = 0;
  return A;
}

template <int Q>
int launch_stage_w(evlb_ctx* c, int w, const StageArgs& A, hipStream_t st) {
  if (w == NARROW) return launch_stage<Q, NARROW, Q>(c, A, st);
  if (w == WC) return launch_stage_col<Q>(c, A, st);
  return launch_stage<Q, WIDE, WideNG<Q>::v>(c, A, st);
}

template <int Q>
int run_step(evlb_ctx* c, double* f, int nsteps, hipStream_t st) {
  const long long nt = c->L.ntot;
  double* momA = (double*)(c->ws + c->L.momA);
  double* momB = (double*)(c->ws + c->L.momB);
  int rc = run_moments<Q>(c, f, momA, momA + nt, momA + 2 * nt, momA + 3 * nt, st);
  if (rc) return rc;
  const int w = pick_width(c);
  int mode = c->p.exec_mode;
  if (mode == EVLB_EXEC_AUTO) mode = EVLB_EXEC_PER_STAGE;
  if (mode == EVLB_EXEC_PERSISTENT) {
    if (w == NARROW) return launch_persistent<GroupShape<Q, NARROW, Q>>(c, w, f, nsteps, st);
    if (w == WC) return launch_persistent<ColumnShape<Q>>(c, w, f, nsteps, st);
    return launch_persistent<GroupShape<Q, WIDE, WideNG<Q>::v>>(c, w, f, nsteps, st);
  }
  double* f1 = (double*)(c->ws + c->L.f1);
  double* f2 = (double*)(c->ws + c->L.f2);
  for (int step = 0; step < nsteps; ++step) {
    for (int s = 0; s < 3; ++s) {
      rc = launch_stage_w<Q>(c, w, stage_args(f, f1, f2, momA, momB, step, s), st);
      if (rc) return rc;
    }
  }
  return EVLB_OK;
}

template <int Q>
int run_rhs(evlb_ctx* c, const double* f, double* L, hipStream_t st) {
  const long long nt = c->L.ntot;
  double* momA = (double*)(c->ws + c->L.momA);
  double* momB = (double*)(c->ws + c->L.momB);
  int rc = run_moments<Q>(c, f, momA, momA + nt, momA + 2 * nt, momA + 3 * nt, st);
  if (rc) return rc;
  StageArgs A;
  A.f_prev = f;
  A.f_n = f;
  A.f_out = L;
  A.mom_in = momA;
  A.mom_out = momB;
  A.alpha = 0.0;
  A.beta = 1.0;
  A.first = 1;
  A.rhs_mode = 1;
  return launch_stage_w<Q>(c, pick_width(c), A, st);
}

template <int Q>
int run_equilibrium(evlb_ctx* c, const double* n, const double* u, const double* T, double* f, hipStream_t st) {
  const int blocks = (int)((c->L.ntot + 255) / 256);
  hipLaunchKernelGGL((equilibrium_kernel<Q>), dim3(blocks), dim3(256), 0, st, c->dp, n, u, T, f);
  return hipGetLastError() == hipSuccess ? EVLB_OK : EVLB_EHIP;
}


// ---- adjoint step -----------------------------------------------------------

DevParams params_adj(const evlb_ctx* c) {
  DevParams P = c->dp;
  P.tiles = (const int4*)(c->ws + c->L.tiles_adj);
  P.ntiles = c->L.ntiles_adj;
  return P;
}

// g = (dL/df)^T v at state f (moments mom), written as
// out = cc (v + dt g) + a1 X1 + a2 X2; parameter partials weighted by pw into
// the slot range vjp_index of the partial buffer (one slot per field-adjoint
// tile, then one per node tile).
template <int Q>
int launch_vjp(evlb_ctx* c, const double* f, const double* mom, const double* v, double* out, const double* X1,
               const double* X2, double cc, double a1, double a2, double pw, int vjp_index, hipStream_t st,
               double* vinj = nullptr, const double* obs = nullptr, const double* wts = nullptr, int j = 0,
               bool final_reduce = false, double* dparams = nullptr, int par = 0, bool sum_prev = false) {
  const DevParams P = params_adj(c);
  AdjArgs A;
  A.f = f;
  A.mom = mom;
  A.v = v;
  A.gdir = (double*)(c->ws + c->L.adj_g);
  A.fa = (double*)(c->ws + c->L.adj_fa);
  A.fb = (double*)(c->ws + c->L.adj_fb);
  A.out = out;
  A.X1 = X1;
  A.X2 = X2;
  A.c = cc;
  A.a1 = a1;
  A.a2 = a2;
  A.pw = pw;
  A.vinj = vinj;
  A.obs = obs;
  A.w = wts;
  A.j = j;
  const int nta = P.ntiles;
  const DevParams Pn = params_for(c, NARROW);
  const int ntn = Pn.ntiles;
  const int nslots = 3 * (ntn + nta);  // one step: three VJPs
  // slots of step parity par, VJP i: ntn field-adjoint tiles, then nta node tiles
  double* part = (double*)(c->ws + c->L.adj_part) + (size_t)par * 2 * nslots;
  // with sum_prev, one extra field workgroup sums the other parity's slots
  // (the previous step, complete by stream order) into dparams
  A.rpart = sum_prev ? (const double*)(c->ws + c->L.adj_part) + (size_t)(par ^ 1) * 2 * nslots : nullptr;
  A.rslots = nslots;
  A.rdp = dparams;
  A.part = part + (size_t)vjp_index * 2 * (ntn + nta);
  hipLaunchKernelGGL((adj_fields_kernel<Q>), dim3(ntn + (sum_prev ? 1 : 0)), dim3(WN * Q), 0, st, Pn, A);
  EVLB_HIP(hipGetLastError());
  A.rpart = nullptr;
  A.part = part + ((size_t)vjp_index * (ntn + nta) + ntn) * 2;
  hipLaunchKernelGGL((adj_column_kernel<Q>), dim3(nta * (2 * Q / NCW)), dim3(64 * NCW), 0, st, P, A,
                     final_reduce ? 1 : 0, (const double*)part, nslots, dparams);
  EVLB_HIP(hipGetLastError());
  return EVLB_OK;
}

// One adjoint step given the step's states f^n, f1, f2 and their moments.
template <int Q>
int adjoint_core(evlb_ctx* c, const double* fn, const double* mn, const double* f1, const double* m1,
                 const double* f2, const double* m2, const double* lam3, double* lam0, double* dparams,
                 hipStream_t st, double* lam3_inject = nullptr, const double* obs = nullptr,
                 const double* wts = nullptr, int j = 0, int par = 0, bool sum_prev = false,
                 bool final_reduce = true) {
  double* mu2 = (double*)(c->ws + c->L.adj_mu2);
  double* mu1 = (double*)(c->ws + c->L.adj_mu1);
  const double dt = c->p.dt;
  // f^{n+1} = 1/3 f^n + 2/3 (f2 + dt L(f2)):   mu2 = 2/3 (lam3 + dt J(f2)^T lam3)
  // (with an observable: lam3 += w[j] obs first, stored back into lam3)
  // (with sum_prev, the previous step's parameter partials are summed into
  // dparams beside the first kernel)
  int rc = launch_vjp<Q>(c, f2, m2, lam3, mu2, nullptr, nullptr, 2.0 / 3.0, 0.0, 0.0, dt * 2.0 / 3.0, 0, st,
                         lam3_inject, obs, wts, j, false, dparams, par, sum_prev);
  if (rc) return rc;
  // f2 = 3/4 f^n + 1/4 (f1 + dt L(f1)):          mu1 = 1/4 (mu2 + dt J(f1)^T mu2)
  rc = launch_vjp<Q>(c, f1, m1, mu2, mu1, nullptr, nullptr, 0.25, 0.0, 0.0, dt * 0.25, 1, st, nullptr, nullptr,
                     nullptr, 0, false, nullptr, par);
  if (rc) return rc;
  // f1 = f^n + dt L(f^n):  lam^n = mu1 + dt J(f^n)^T mu1 + 1/3 lam3 + 3/4 mu2
  // (with final_reduce its last kernel adds the step's parameter derivatives
  // to dparams; otherwise the next step's first kernel does)
  return launch_vjp<Q>(c, fn, mn, mu1, lam0, lam3, mu2, 1.0, 1.0 / 3.0, 0.75, dt, 2, st, nullptr, nullptr, nullptr, 0,
                       final_reduce, dparams, par);
}

template <int Q>
int run_adjoint(evlb_ctx* c, const double* fn, const double* lam3, double* lam0, double* dparams, hipStream_t st) {
  const long long nt = c->L.ntot;
  double* momA = (double*)(c->ws + c->L.momA);
  double* momB = (double*)(c->ws + c->L.momB);
  double* f1 = (double*)(c->ws + c->L.f1);
  double* f2 = (double*)(c->ws + c->L.f2);
  double* amom = (double*)(c->ws + c->L.adj_mom);
  // recompute the two inner stages: f1 (moments in momB), f2 (moments in momA)
  int rc = run_moments<Q>(c, fn, amom, amom + nt, amom + 2 * nt, amom + 3 * nt, st);
  if (rc) return rc;
  const int w = pick_width(c);
  StageArgs A0 = stage_args(const_cast<double*>(fn), f1, f2, momA, momB, 0, 0);
  A0.mom_in = amom;
  rc = launch_stage_w<Q>(c, w, A0, st);
  if (rc) return rc;
  rc = launch_stage_w<Q>(c, w, stage_args(const_cast<double*>(fn), f1, f2, momA, momB, 0, 1), st);
  if (rc) return rc;
  return adjoint_core<Q>(c, fn, amom, f1, momB, f2, momA, lam3, lam0, dparams, st);
}

// Record layout of one step j: f^j, f1^j, f2^j ([2][q][n] each), then the
// moments of the three ([4][n] each).
size_t record_doubles(const evlb_ctx* c) {
  const size_t fs = 2 * (size_t)c->p.q * (size_t)c->L.ntot;
  return 3 * fs + 3 * 4 * (size_t)c->L.ntot;
}

template <int Q>
int run_step_record(evlb_ctx* c, const double* f0, int nsteps, double* rec, hipStream_t st) {
  const size_t fs = 2 * (size_t)Q * (size_t)c->L.ntot;
  const size_t R = record_doubles(c);
  const long long nt = c->L.ntot;
  EVLB_HIP(hipMemcpyAsync(rec, f0, fs * sizeof(double), hipMemcpyDeviceToDevice, st));
  double* m0 = rec + 3 * fs;
  int rc = run_moments<Q>(c, rec, m0, m0 + nt, m0 + 2 * nt, m0 + 3 * nt, st);
  if (rc) return rc;
  const int w = pick_width(c);
  const double a_s[3] = {0.0, 0.75, 1.0 / 3.0};
  const double b_s[3] = {1.0, 0.25, 2.0 / 3.0};
  for (int j = 0; j < nsteps; ++j) {
    double* r = rec + (size_t)j * R;
    double* rn = rec + (size_t)(j + 1) * R;
    double* fj[3] = {r, r + fs, r + 2 * fs};
    double* mj[3] = {r + 3 * fs, r + 3 * fs + 4 * nt, r + 3 * fs + 8 * nt};
    for (int s = 0; s < 3; ++s) {
      StageArgs A;
      A.f_prev = fj[s];
      A.f_n = fj[0];
      A.f_out = s < 2 ? fj[s + 1] : rn;
      A.mom_in = mj[s];
      A.mom_out = s < 2 ? mj[s + 1] : rn + 3 * fs;
      A.alpha = a_s[s];
      A.beta = b_s[s];
      A.first = s == 0;
      A.rhs_mode = 0;
      rc = launch_stage_w<Q>(c, w, A, st);
      if (rc) return rc;
    }
  }
  return EVLB_OK;
}

template <int Q>
int run_adjoint_record(evlb_ctx* c, const double* rec, int nsteps, double* lam, const double* obs, const double* wts,
                       double* dparams, hipStream_t st) {
  const size_t fs = 2 * (size_t)Q * (size_t)c->L.ntot;
  const size_t R = record_doubles(c);
  const long long nt = c->L.ntot;
  double* other = (double*)(c->ws + c->L.adj_lam);
  double* cur = lam;
  for (int j = nsteps - 1; j >= 0; --j) {
    const double* r = rec + (size_t)j * R;
    double* nxt = cur == lam ? other : lam;
    const bool inj = obs && wts;
    // step s of the pass keeps its parameter partials in parity s & 1; the
    // next step sums them beside its first kernel, and the last step sums its
    // own in its last kernel
    const int s = nsteps - 1 - j;
    int rc = adjoint_core<Q>(c, r, r + 3 * fs, r + fs, r + 3 * fs + 4 * nt, r + 2 * fs, r + 3 * fs + 8 * nt, cur, nxt,
                             dparams, st, inj ? cur : nullptr, obs, wts, j, s & 1, s > 0, j == 0);
    if (rc) return rc;
    cur = nxt;
  }
  if (cur != lam) EVLB_HIP(hipMemcpyAsync(lam, cur, fs * sizeof(double), hipMemcpyDeviceToDevice, st));
  return EVLB_OK;
}

template <int Q>
int run_equilibrium_adjoint(evlb_ctx* c, const double* n, const double* u, const double* T, const double* lam,
                            double* nb, double* ub, double* Tb, hipStream_t st) {
  const int blocks = (int)((c->L.ntot + 255) / 256);
  hipLaunchKernelGGL((equilibrium_adjoint_kernel<Q>), dim3(blocks), dim3(256), 0, st, c->dp, n, u, T, lam, nb, ub,
                     Tb);
  return hipGetLastError() == hipSuccess ? EVLB_OK : EVLB_EHIP;
}

#define EVLB_DISPATCH_Q(q, fn, ...)              \
  switch (q) {                                   \
    case 8: return fn<8>(__VA_ARGS__);           \
    case 16: return fn<16>(__VA_ARGS__);         \
    case 24: return fn<24>(__VA_ARGS__);         \
    default: return EVLB_EUNSUPPORTED;           \
  }

bool device_matches(const evlb_ctx* c) {
  int d = -1;
  return hipGetDevice(&d) == hipSuccess && d == c->device;
}

}  // namespace

// The workspace of evlb_init_noalloc: one array per device, loaded with the
// code object.  Host code reaches it only through the address that
// hipGetSymbolAddress returns with that device current (the array's name in
// host code is a host-side stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[EVLB_NOALLOC_MAX_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` per device (null: not looked up yet)

int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return EVLB_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return EVLB_EHIP;
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return EVLB_OK;
}
}  // namespace

extern "C" {

int evlb_validate(const evlb_params* params) { return validate(params); }

size_t evlb_workspace_bytes(const evlb_params* params) {
  if (validate(params) != EVLB_OK) return 0;
  if (params->dim == 2) return evlb2d::workspace_bytes(params);
  return make_layout(params).total;
}

int evlb_init_noalloc(const evlb_params* params, void* hip_stream, evlb_ctx** out) {
  if (!out) return EVLB_EINVAL;
  *out = nullptr;
  const int rc = validate(params);
  if (rc) return rc;
  if (evlb_workspace_bytes(params) > EVLB_NOALLOC_MAX_BYTES) return EVLB_EWORKSPACE;
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess) return EVLB_EHIP;
  void* ws = nullptr;
  const int sc = scratch_address(device, &ws);
  if (sc) return sc;
  return evlb_init(params, ws, EVLB_NOALLOC_MAX_BYTES, hip_stream, out);
}

int evlb_init(const evlb_params* params, void* d_workspace, size_t ws_bytes, void* hip_stream, evlb_ctx** out) {
  if (!out) return EVLB_EINVAL;
  *out = nullptr;
  int rc = validate(params);
  if (rc) return rc;
  if (params->dim == 2) {
    const size_t need = evlb2d::workspace_bytes(params);
    if (!d_workspace || ws_bytes < need || ((uintptr_t)d_workspace & 255)) return EVLB_EWORKSPACE;
    evlb_ctx* c = new (std::nothrow) evlb_ctx();
    if (!c) return EVLB_EINVAL;
    c->p = *params;
    c->nx.assign(params->nx, params->nx + 1);
    c->p.nx = c->nx.data();
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return EVLB_EHIP; }
    rc = evlb2d::init(params, (char*)d_workspace, ws_bytes, (hipStream_t)hip_stream, &c->c2);
    if (rc) { delete c; return rc; }
    c->ws = (char*)d_workspace;
    c->vel = evlb2d::velocities(c->c2);
    c->L.ntot = evlb2d::node_count(c->c2);
    c->dp.status = evlb2d::status_word(c->c2);
    *out = c;
    return EVLB_OK;
  }
  const Layout L = make_layout(params);
  if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace & 255)) return EVLB_EWORKSPACE;
  evlb_ctx* c = new (std::nothrow) evlb_ctx();
  if (!c) return EVLB_EINVAL;
  c->p = *params;
  c->nx.assign(params->nx, params->nx + params->n_sys);
  c->p.nx = c->nx.data();
  if (params->T_iso_sys) c->tiso.assign(params->T_iso_sys, params->T_iso_sys + params->n_sys);
  c->p.T_iso_sys = params->T_iso_sys ? c->tiso.data() : nullptr;
  c->L = L;
  c->ws = (char*)d_workspace;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return EVLB_EHIP; }
  if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
    delete c;
    return EVLB_EHIP;
  }
  evlb::TableParams tp{params->q, params->dx, params->sigma, params->phi_sigma, params->gamma, params->r_cut};
  evlb::HostTables t;
  evlb::build_tables(tp, t);
  if (params->force_model != EVLB_FORCE_EV1) {
    t.cfor.assign(1, 0.0);
    t.cphi.assign(1, 0.0);
    t.csig.assign(1, 0.0);
  }
  c->vel = t.vel;
  const int q = params->q;
  std::vector<double> host;
  host.insert(host.end(), t.vel.begin(), t.vel.end());
  host.insert(host.end(), t.meq.begin(), t.meq.end());
  host.insert(host.end(), t.dpm.begin(), t.dpm.end());
  host.insert(host.end(), t.savg.begin(), t.savg.end());
  host.insert(host.end(), t.cfor.begin(), t.cfor.end());
  host.insert(host.end(), t.cphi.begin(), t.cphi.end());
  host.insert(host.end(), t.csig.begin(), t.csig.end());
  host.insert(host.end(), t.ssig.begin(), t.ssig.end());
  std::vector<int4> tw, tn, tc, ta;
  int off = 0;
  for (int s = 0; s < params->n_sys; ++s) {
    for (int i0 = 0; i0 < params->nx[s]; i0 += WIDE) tw.push_back(make_int4(off, params->nx[s], i0, 0));
    for (int i0 = 0; i0 < params->nx[s]; i0 += NARROW) tn.push_back(make_int4(off, params->nx[s], i0, 0));
    for (int i0 = 0; i0 < params->nx[s]; i0 += WC) tc.push_back(make_int4(off, params->nx[s], i0, 0));
    for (int i0 = 0; i0 < params->nx[s]; i0 += WA) ta.push_back(make_int4(off, params->nx[s], i0, 0));
    off += params->nx[s];
  }
  hipStream_t st = (hipStream_t)hip_stream;
  double* tab = (double*)(c->ws + L.tables);
  // the per-system temperatures expanded to one value per node
  std::vector<double> tn_node;
  if (params->T_iso_sys) {
    tn_node.resize((size_t)L.ntot);
    size_t o = 0;
    for (int s = 0; s < params->n_sys; ++s)
      for (int i = 0; i < params->nx[s]; ++i) tn_node[o++] = params->T_iso_sys[s];
  }
  // copies ordered on the caller's stream; the stream is synchronised before
  // returning because the host vectors die with this call
  if (hipMemcpyAsync(tab, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c->ws + L.tiles_wide, tw.data(), tw.size() * sizeof(int4), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(c->ws + L.tiles_narrow, tn.data(), tn.size() * sizeof(int4), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(c->ws + L.tiles_col, tc.data(), tc.size() * sizeof(int4), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(c->ws + L.tiles_adj, ta.data(), ta.size() * sizeof(int4), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemsetAsync(c->ws + L.status, 0, 256, st) != hipSuccess ||
      (params->T_iso_sys && hipMemcpyAsync(c->ws + L.tiso, tn_node.data(), tn_node.size() * sizeof(double),
                                           hipMemcpyHostToDevice, st) != hipSuccess) ||
      hipStreamSynchronize(st) != hipSuccess) {
    delete c;
    return EVLB_EHIP;
  }
  DevParams& d = c->dp;
  d.vel = tab;
  d.meq = tab + q;
  d.dpm = tab + q + q * q;
  d.savg = tab + q + 2 * q * q;
  const int nc = (int)t.cfor.size();
  d.cfor = tab + q + 2 * q * q + 2 * L.ms + 1;
  d.cphi = d.cfor + nc;
  d.csig = d.cphi + nc;
  d.ssig = d.csig + nc;
  d.tiles = (const int4*)(c->ws + L.tiles_wide);
  d.ntiles = L.ntiles_wide;
  d.single = params->n_sys == 1;
  d.ms = L.ms;
  d.mf = L.mf;
  d.hn = L.mf > L.ms + 2 ? L.mf : L.ms + 2;
  d.ntot = L.ntot;
  d.dx = params->dx;
  d.inv_dx = 1.0 / params->dx;
  d.dt = params->dt;
  const double sg = params->sigma;
  d.b = 2.0 * M_PI * sg * sg * sg / 3.0;
  d.eta_c = M_PI * sg * sg * sg / 6.0;
  d.mu0c = 5.0 / (16.0 * sg * sg * std::sqrt(M_PI));
  d.sigma = sg;
  d.weno_eps = params->weno_eps;
  d.g_ext = params->g_ext;
  const double g = params->gamma;
  d.two_a = 2.0 * (2.0 * M_PI * sg * sg * sg / 3.0) * params->phi_sigma * g / (g - 3.0);
  d.kappa = (2.0 * M_PI * std::pow(sg, 5) / 15.0) * params->phi_sigma * (g > 5.0 ? g / (g - 5.0) : 0.0);
  d.force_model = params->force_model;
  d.term_mask = params->term_mask;
  d.T_iso = params->T_iso;
  d.tiso = params->T_iso_sys ? (const double*)(c->ws + L.tiso) : nullptr;
  d.status = (int*)(c->ws + L.status);
  d.bar = (unsigned*)(c->ws + L.status + 64);
  *out = c;
  return EVLB_OK;
}

int evlb_set_equilibrium(evlb_ctx* ctx, const double* d_n, const double* d_u, const double* d_T, double* d_f,
                         void* hip_stream) {
  if (!ctx || !d_n || !d_u || !d_T || !d_f) return EVLB_EINVAL;
  if (!device_matches(ctx)) return EVLB_EINVAL;
  if (ctx->c2) return evlb2d::set_equilibrium(ctx->c2, d_n, d_u, d_T, d_f, (hipStream_t)hip_stream);
  EVLB_DISPATCH_Q(ctx->p.q, run_equilibrium, ctx, d_n, d_u, d_T, d_f, (hipStream_t)hip_stream);
}

int evlb_step(evlb_ctx* ctx, double* d_f, int32_t nsteps, void* hip_stream) {
  if (!ctx || !d_f || nsteps < 0) return EVLB_EINVAL;
  if (!device_matches(ctx)) return EVLB_EINVAL;
  if (nsteps == 0) return EVLB_OK;
  if (ctx->c2) return evlb2d::step(ctx->c2, d_f, nsteps, (hipStream_t)hip_stream);
  EVLB_DISPATCH_Q(ctx->p.q, run_step, ctx, d_f, nsteps, (hipStream_t)hip_stream);
}

int evlb_rhs(evlb_ctx* ctx, const double* d_f, double* d_L, void* hip_stream) {
  if (!ctx || !d_f || !d_L || d_f == d_L) return EVLB_EINVAL;
  if (!device_matches(ctx)) return EVLB_EINVAL;
  if (ctx->c2) return evlb2d::rhs(ctx->c2, d_f, d_L, (hipStream_t)hip_stream);
  EVLB_DISPATCH_Q(ctx->p.q, run_rhs, ctx, d_f, d_L, (hipStream_t)hip_stream);
}

int evlb_moments(evlb_ctx* ctx, const double* d_f, double* d_n, double* d_u, double* d_T, double* d_q,
                 void* hip_stream) {
  if (!ctx || !d_f || !d_n || !d_u || !d_T) return EVLB_EINVAL;
  if (!device_matches(ctx)) return EVLB_EINVAL;
  if (ctx->c2) return evlb2d::moments(ctx->c2, d_f, d_n, d_u, d_T, d_q, (hipStream_t)hip_stream);
  EVLB_DISPATCH_Q(ctx->p.q, run_moments, ctx, d_f, d_n, d_u, d_T, d_q, (hipStream_t)hip_stream, 0);
}

int evlb_adjoint_step(evlb_ctx* ctx, const double* d_f_n, const double* d_lam_np1, double* d_lam_n,
                      double* d_dparams, void* hip_stream) {
  if (!ctx || !d_f_n || !d_lam_np1 || !d_lam_n || !d_dparams) return EVLB_EINVAL;
  if (ctx->c2) return EVLB_EUNSUPPORTED;
  if (!ctx->p.adjoint) return EVLB_EINVAL;
  if (d_lam_n == d_lam_np1 || (const double*)d_lam_n == d_f_n) return EVLB_EINVAL;
  if (!device_matches(ctx)) return EVLB_EINVAL;
  EVLB_DISPATCH_Q(ctx->p.q, run_adjoint, ctx, d_f_n, d_lam_np1, d_lam_n, d_dparams, (hipStream_t)hip_stream);
}

int evlb_equilibrium_adjoint(evlb_ctx* ctx, const double* d_n, const double* d_u, const double* d_T,
                             const double* d_lam, double* d_nbar, double* d_ubar, double* d_Tbar, void* hip_stream) {
  if (!ctx || !d_n || !d_u || !d_T || !d_lam || !d_nbar || !d_ubar || !d_Tbar) return EVLB_EINVAL;
  if (ctx->c2) return EVLB_EUNSUPPORTED;
  if (!device_matches(ctx)) return EVLB_EINVAL;
  EVLB_DISPATCH_Q(ctx->p.q, run_equilibrium_adjoint, ctx, d_n, d_u, d_T, d_lam, d_nbar, d_ubar, d_Tbar,
                  (hipStream_t)hip_stream);
}

int64_t evlb_record_doubles(const evlb_ctx* ctx) { return ctx && !ctx->c2 ? (int64_t)record_doubles(ctx) : 0; }

int evlb_step_record(evlb_ctx* ctx, const double* d_f0, int32_t nsteps, double* d_rec, void* hip_stream) {
  if (!ctx || !d_f0 || !d_rec || nsteps < 0) return EVLB_EINVAL;
  if (ctx->c2) return EVLB_EUNSUPPORTED;
  if (!device_matches(ctx)) return EVLB_EINVAL;
  EVLB_DISPATCH_Q(ctx->p.q, run_step_record, ctx, d_f0, nsteps, d_rec, (hipStream_t)hip_stream);
}

int evlb_adjoint_record(evlb_ctx* ctx, const double* d_rec, int32_t nsteps, double* d_lam, const double* d_obs,
                        const double* d_w, double* d_dparams, void* hip_stream) {
  if (!ctx || !d_rec || !d_lam || !d_dparams || nsteps < 0) return EVLB_EINVAL;
  if (ctx->c2) return EVLB_EUNSUPPORTED;
  if (!ctx->p.adjoint || ((d_obs == nullptr) != (d_w == nullptr))) return EVLB_EINVAL;
  if (!device_matches(ctx)) return EVLB_EINVAL;
  EVLB_DISPATCH_Q(ctx->p.q, run_adjoint_record, ctx, d_rec, nsteps, d_lam, d_obs, d_w, d_dparams,
                  (hipStream_t)hip_stream);
}

int evlb_status(evlb_ctx* ctx, void* hip_stream, int32_t clear) {
  if (!ctx) return EVLB_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  int h[2] = {0, 0};
  // read (and clear) the latch in stream order, then wait for both
  if (hipMemcpyAsync(h, ctx->dp.status, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return EVLB_EHIP;
  if (clear && hipMemsetAsync(ctx->dp.status, 0, sizeof(h), st) != hipSuccess) return EVLB_EHIP;
  if (hipStreamSynchronize(st) != hipSuccess) return EVLB_EHIP;
  if (h[1]) return EVLB_EHIP;
  return h[0] ? EVLB_ENONFINITE : EVLB_OK;
}

int evlb_info(const evlb_ctx* ctx, int64_t* n_tot, double* h_velocities) {
  if (!ctx) return EVLB_EINVAL;
  if (n_tot) *n_tot = ctx->L.ntot;
  if (h_velocities) std::memcpy(h_velocities, ctx->vel.data(), ctx->vel.size() * sizeof(double));
  return EVLB_OK;
}

void evlb_destroy(evlb_ctx* ctx) {
  if (ctx && ctx->c2) evlb2d::destroy(ctx->c2);
  delete ctx;
}

const char* evlb_strerror(int code) {
  switch (code) {
    case EVLB_OK: return "ok";
    case EVLB_EINVAL: return "invalid argument or parameter";
    case EVLB_ECFL: return "time step above the advection stability limit";
    case EVLB_EWORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    case EVLB_EHIP: return "HIP runtime error";
    case EVLB_ENONFINITE: return "non-positive or non-finite density or temperature";
    case EVLB_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown error";
  }
}

}  // extern "C"
