// Host-side constant tables of the EV-FDLB step (velocity set, Hermite
// projections, stencil weights), computed once per context in long double.
//
// Velocity set: full-range Gauss-Hermite quadrature of order Q for the
// weight exp(-p^2/2)/sqrt(2 pi) (Sec. III names the quadrature; the paper
// uses Q_x = 16).  Nodes are the roots of He_Q, located by sign changes on
// a fine grid and refined by bisection and Newton steps; the weights are
// the Christoffel numbers Q!/(Q He_{Q-1}(p_k))^2.
#include "tables.h"

#include <cmath>
#include <stdexcept>
#include <vector>

namespace evlb {

namespace {

typedef long double ld;

// He_0..He_lmax at x by He_{l+1} = x He_l - l He_{l-1}.
void hermite_values(ld x, int lmax, std::vector<ld>& h) {
  h.assign(lmax + 1, 0.0L);
  h[0] = 1.0L;
  if (lmax >= 1) h[1] = x;
  for (int l = 1; l < lmax; ++l) h[l + 1] = x * h[l] - (ld)l * h[l - 1];
}

ld he(int n, ld x) {
  std::vector<ld> h;
  hermite_values(x, n, h);
  return h[n];
}

ld factorial(int n) {
  ld f = 1.0L;
  for (int i = 2; i <= n; ++i) f *= (ld)i;
  return f;
}

// composite Simpson 1/3 weight of node j in 0..m2 (m2 even intervals)
double simpson(int j, int m2) {
  if (j == 0 || j == m2) return 1.0 / 3.0;
  return (j % 2) ? 4.0 / 3.0 : 2.0 / 3.0;
}

}  // namespace

void gauss_hermite_nodes(int Q, std::vector<double>& p, std::vector<double>& w) {
  // all roots of He_Q lie in |x| < sqrt(4Q + 2)
  const ld R = std::sqrt((ld)(4 * Q + 2));
  const int M = 40000;
  std::vector<ld> roots;
  ld x0 = -R, f0 = he(Q, x0);
  for (int i = 1; i <= M && (int)roots.size() < Q; ++i) {
    ld x1 = -R + 2.0L * R * (ld)i / (ld)M;
    ld f1 = he(Q, x1);
    if (f1 == 0.0L) {
      roots.push_back(x1);
    } else if ((f0 < 0) != (f1 < 0) && f0 != 0.0L) {
      ld a = x0, b = x1, fa = f0;
      for (int it = 0; it < 200 && b - a > 0; ++it) {
        ld m = 0.5L * (a + b);
        ld fm = he(Q, m);
        if ((fm < 0) == (fa < 0)) { a = m; fa = fm; } else { b = m; }
      }
      ld r = 0.5L * (a + b);
      std::vector<ld> h;
      for (int it = 0; it < 3; ++it) {
        hermite_values(r, Q, h);
        ld d = (ld)Q * h[Q - 1];
        if (d != 0) r -= h[Q] / d;
      }
      roots.push_back(r);
    }
    x0 = x1;
    f0 = f1;
  }
  if ((int)roots.size() != Q) throw std::runtime_error("Gauss-Hermite root search failed");
  p.resize(Q);
  w.resize(Q);
  const ld qf = factorial(Q);
  std::vector<ld> wl(Q);
  for (int k = 0; k < Q; ++k) {
    ld hq1 = he(Q - 1, roots[k]);
    wl[k] = qf / (((ld)Q * hq1) * ((ld)Q * hq1));
  }
  // symmetric rule: average mirrored pairs
  for (int k = 0; k < Q; ++k) {
    ld r = 0.5L * (roots[k] - roots[Q - 1 - k]);
    ld ww = 0.5L * (wl[k] + wl[Q - 1 - k]);
    p[k] = (double)r;
    w[k] = (double)ww;
  }
}

void build_tables(const TableParams& tp, HostTables& t) {
  const int Q = tp.q;
  std::vector<double> p, w;
  gauss_hermite_nodes(Q, p, w);
  t.vel = p;
  t.wgt = w;

  // Hermite equilibrium: E_k = sum_l meq[k][l] a_l, meq = w_k He_l(p_k)/l!
  // Momentum derivative: dp[k][k'] = -w_k sum_{l<=Q-2} He_{l+1}(p_k) He_l(p_k')/l!
  t.meq.assign(Q * Q, 0.0);
  t.dpm.assign(Q * Q, 0.0);
  std::vector<std::vector<ld>> H(Q);
  for (int k = 0; k < Q; ++k) hermite_values((ld)p[k], Q, H[k]);
  for (int k = 0; k < Q; ++k) {
    for (int l = 0; l < Q; ++l) t.meq[k * Q + l] = (double)((ld)w[k] * H[k][l] / factorial(l));
    for (int kp = 0; kp < Q; ++kp) {
      ld s = 0.0L;
      for (int l = 0; l + 1 < Q; ++l) s += H[k][l + 1] * H[kp][l] / factorial(l);
      t.dpm[k * Q + kp] = (double)(-(ld)w[k] * s);
    }
  }

  // Averaged density (Sec. II A, ball of radius sigma reduced to 1D):
  // nbar_i = sum_{|j|<=ms} savg_j n_{i+j}, savg_j = 3/(4 s^3)(s^2-(j dx)^2) dx S_j
  const int ms = (int)std::lround(tp.sigma / tp.dx);
  t.ms = ms;
  t.savg.assign(2 * ms + 1, 0.0);
  t.ssig.assign(2 * ms + 1, 0.0);
  for (int j = -ms; j <= ms; ++j) {
    ld s = (ld)j * tp.dx;
    ld sg = tp.sigma;
    t.savg[j + ms] = (double)(3.0L / (4.0L * sg * sg * sg) * (sg * sg - s * s) * (ld)tp.dx *
                              (ld)simpson(j + ms, 2 * ms));
    // the node window stays fixed when sigma varies; the weights follow it
    t.ssig[j + ms] = (double)((3.0L / (2.0L * sg * sg) - 9.0L * (sg * sg - s * s) / (4.0L * sg * sg * sg * sg)) *
                              (ld)tp.dx * (ld)simpson(j + ms, 2 * ms));
  }

  // EV1 force, eq:F1 by composite Simpson on |s| <= r_cut:
  // F_i = sum_{j=1..mf} cfor_j (n_{i+j} - n_{i-j}),
  // cfor_j = K(j dx) dx S_j, K(s) = 2 pi phi s (sigma/max(sigma,|s|))^gamma
  const int mf = (int)std::lround(tp.r_cut / tp.dx);
  t.mf = mf;
  t.cfor.assign(mf, 0.0);
  t.cphi.assign(mf, 0.0);
  t.csig.assign(mf, 0.0);
  const ld pi = 3.141592653589793238462643383279502884L;
  for (int j = 1; j <= mf; ++j) {
    ld s = (ld)j * tp.dx;
    const bool outer = !(s < (ld)tp.sigma);
    ld ratio = outer ? std::pow((ld)tp.sigma / s, (ld)tp.gamma) : 1.0L;
    const ld unit = 2.0L * pi * s * ratio * (ld)tp.dx * (ld)simpson(j + mf, 2 * mf);
    t.cfor[j - 1] = (double)((ld)tp.phi * unit);
    t.cphi[j - 1] = (double)unit;
    // outer branch: K ~ sigma^gamma; inner branch independent of sigma
    t.csig[j - 1] = outer ? (double)((ld)tp.phi * unit * (ld)tp.gamma / (ld)tp.sigma) : 0.0;
  }
}

// 2D disc stencils.
//
// Averaged density: the ball average of Sec. II A integrated over z is a disc
// average with weight 2 sqrt(sigma^2 - s^2) (the chord of the ball); the
// weights of the cells with s < sigma are normalised to sum 1.
//
// Force: a line of density along z at in-plane distance s acts through the
// tail of eq:sutherland (gamma = 6) outside the hard core; with z = s tan t,
//   K(s) = 12 phi sigma^6 s^-7 I(psi),  I(psi) = int_0^psi sin^6 t dt
//        = 5 psi/16 - 15 sin(2 psi)/64 + 3 sin(4 psi)/64 - sin(6 psi)/192,
// psi = asin(s/sigma) inside the core and pi/2 outside.  The force on a node
// is sum over cells of K(s) (s_vec / s) n dx^2, taken as antisymmetric pairs
// +-s: F = sum_pairs c (n(+s) - n(-s)).
void build_disc_tables(double dx, double sigma, double phi, double r_cut, bool force, DiscTables& t) {
  const ld pi = 3.141592653589793238462643383279502884L;
  const ld h = dx, sg = sigma;
  t = DiscTables();
  const int ma = (int)std::ceil(sigma / dx);
  ld wsum = 0.0L;
  std::vector<ld> wl;
  for (int j = -ma; j <= ma; ++j) {
    for (int i = -ma; i <= ma; ++i) {
      const ld s2 = (ld)(i * i + j * j) * h * h;
      if (!(s2 < sg * sg)) continue;
      const ld w = 2.0L * std::sqrt(sg * sg - s2);
      t.avg_di.push_back(i);
      t.avg_dj.push_back(j);
      wl.push_back(w);
      wsum += w;
      if (std::abs(i) > t.avg_reach) t.avg_reach = std::abs(i);
      if (std::abs(j) > t.avg_reach) t.avg_reach = std::abs(j);
    }
  }
  for (ld w : wl) t.avg_w.push_back((double)(w / wsum));
  if (!force) return;
  const int mf = (int)std::lround(r_cut / dx);
  for (int j = -mf; j <= mf; ++j) {
    for (int i = -mf; i <= mf; ++i) {
      if (i * i + j * j > mf * mf || i * i + j * j == 0) continue;
      if (!(i > 0 || (i == 0 && j > 0))) continue;
      const ld s = h * std::sqrt((ld)(i * i + j * j));
      const ld psi = s < sg ? std::asin(s / sg) : 0.5L * pi;
      const ld I = 5.0L * psi / 16.0L - 15.0L * std::sin(2.0L * psi) / 64.0L +
                   3.0L * std::sin(4.0L * psi) / 64.0L - std::sin(6.0L * psi) / 192.0L;
      const ld sg3 = sg * sg * sg;
      const ld K = 12.0L * (ld)phi * sg3 * sg3 * I / std::pow(s, 7);
      t.pair_di.push_back(i);
      t.pair_dj.push_back(j);
      t.pair_cx.push_back((double)(K * (ld)i * h * h * h));
      t.pair_cy.push_back((double)(K * (ld)j * h * h * h));
      if (std::abs(i) > t.pair_reach) t.pair_reach = std::abs(i);
      if (std::abs(j) > t.pair_reach) t.pair_reach = std::abs(j);
    }
  }
}

}  // namespace evlb
