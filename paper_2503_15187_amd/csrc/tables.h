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

void gauss_hermite_nodes(int q, std::vector<double>& p, std::vector<double>& w);
void build_tables(const TableParams& tp, HostTables& t);

}  // namespace evlb
