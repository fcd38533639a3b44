// Host-side set-up of a plan that needs no device: descriptor validation,
// the stability bound, the PML profile and the linear-interpolation sensor
// operator (gather taps per grid row and the transposed operator grouped by
// node).  Plain C++ with no HIP dependency, so that it also builds on its
// own for host-only checks (sanitizers).
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/pat.h"

namespace pat {

// Linear-interpolation tap of one sensor in one grid row:
// partial[slot] = w0 * p[row][x0] + w1 * p[row][x0 + 1]
struct GTap {
  int32_t x0;
  int32_t slot;
  float w0, w1;
};

// Transposed sensor operator, grouped by node: a row's groups have distinct
// x, each summing its taps w * h[s] in a fixed order.
struct SGroup {
  int32_t x;
  int32_t beg, end;
};
struct STap {
  int32_t s;
  float w;
};

// The sensor operator of one plan in CSR form.
//   slot_ptr[s] .. slot_ptr[s+1]  partial-sum slots of sensor s (one per grid
//                                 row it touches with non-zero weight)
//   g_ptr[row] .. g_ptr[row+1]    gather taps of a grid row
//   s_ptr[row] .. s_ptr[row+1]    node groups of a grid row (scatter W^T)
struct SensorOps {
  std::vector<int32_t> g_ptr, s_ptr, slot_ptr;
  std::vector<GTap> g_tap;
  std::vector<SGroup> s_grp;
  std::vector<STap> s_tap;
  int nslots = 0;
};

// PAT_OK or PAT_EINVAL: ranges of every descriptor field (pat.h).
int validate_desc(const pat_desc* d, bool lossy);

// Time step of the plan: d.dt, or cfl * min dx / c_max when d.dt <= 0.
double plan_dt(const pat_desc& d, double c_max);

// PAT_OK, or PAT_EUNSTABLE when c_max dt / min dx exceeds 1 / sqrt(ndim).
int check_stability(const pat_desc& d, double c_max, double dt);

// PML factor exp(-sigma dt / 2) at node i (stag: at i + 1/2) of an axis of n
// points with L layer points per side; sigma = alpha (c_ref / dx) (depth / L)^4.
double pml_factor(int n, int L, double alpha, double c_ref, double dx, double dt, int i, bool stag);

// The sensor operator of the n_sensors positions pos[s * ndim + j] (physical
// coordinates).  PAT_EINVAL if a grid coordinate lies outside [0, n_j - 1]
// or is not finite.
int build_sensors(const pat_desc& d, const double* pos, SensorOps& so);

}  // namespace pat
