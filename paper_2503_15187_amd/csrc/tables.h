// Host-side constant tables of the EV-FDLB step (see tables.cpp).
#pragma once

#include <vector>

namespace evlb {

struct TableParams {
  int q;
  double dx, sigma, phi, gamma, r_cut;
};

struct HostTables {
  std::vector<double> vel, wgt;   // [q] nodes (ascending), weights (sum 1)
  std::vector<double> meq, dpm;   // [q*q], row k = velocity
  std::vector<double> savg;       // [2*ms+1]
  std::vector<double> cfor;       // [mf], j = 1..mf
  std::vector<double> cphi;       // [mf] d cfor_j / d phi
  std::vector<double> csig;       // [mf] d cfor_j / d sigma
  std::vector<double> ssig;       // [2*ms+1] d savg_j / d sigma
  int ms = 0, mf = 0;
};

// Disc stencils of the 2D extension (fluid homogeneous in z), cell-centre
// rule on the grid of spacing dx.  Offsets (di, dj) are along (x, y).
struct DiscTables {
  std::vector<int> avg_di, avg_dj;     // cells with s < sigma
  std::vector<double> avg_w;           // 2 sqrt(sigma^2 - s^2), sum 1
  std::vector<int> pair_di, pair_dj;   // one cell of each +-s pair, s <= r_cut
  std::vector<double> pair_cx, pair_cy;  // K(s) s_vec dx^2 / s
  int avg_reach = 0, pair_reach = 0;   // max |di|, |dj| of each stencil
};

void gauss_hermite_nodes(int q, std::vector<double>& p, std::vector<double>& w);
void build_tables(const TableParams& tp, HostTables& t);
void build_disc_tables(double dx, double sigma, double phi, double r_cut, bool force, DiscTables& t);

}  // namespace evlb
