// Host interface of the 2D path (dim = 2) behind the C ABI of evlb.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "../../include/evlb.h"

namespace evlb2d {

struct Ctx;

int validate(const evlb_params* p);
size_t workspace_bytes(const evlb_params* p);
int init(const evlb_params* p, char* ws, size_t bytes, hipStream_t st, Ctx** out);
void destroy(Ctx* c);

long long node_count(const Ctx* c);
const std::vector<double>& velocities(const Ctx* c);
int* status_word(const Ctx* c);

int set_equilibrium(Ctx* c, const double* n, const double* u, const double* T, double* f, hipStream_t st);
int step(Ctx* c, double* f, int nsteps, hipStream_t st);
int rhs(Ctx* c, const double* f, double* L, hipStream_t st);
int moments(Ctx* c, const double* f, double* n, double* u, double* T, double* q, hipStream_t st);

}  // namespace evlb2d
