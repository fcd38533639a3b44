// Host-side plan set-up without a device (see host_plan.h).
#include "host_plan.h"

#include <algorithm>
#include <cmath>

namespace pat {

namespace {
bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
}  // namespace

int validate_desc(const pat_desc* d, bool lossy) {
  if (!d) return PAT_EINVAL;
  if (d->ndim != 2 && d->ndim != 3) return PAT_EINVAL;
  for (int j = 0; j < d->ndim; ++j) {
    const int lim = d->ndim == 3 ? 256 : 1024;
    if (!is_pow2(d->n[j]) || d->n[j] < 16 || d->n[j] > lim) return PAT_EINVAL;
    if (!(d->dx[j] > 0) || !std::isfinite(d->dx[j]) || !std::isfinite(d->origin[j])) return PAT_EINVAL;
    if (d->pml_size[j] < 0 || 2 * d->pml_size[j] >= d->n[j]) return PAT_EINVAL;
  }
  if (d->nt < 1) return PAT_EINVAL;
  if (!std::isfinite(d->dt) || !std::isfinite(d->cfl)) return PAT_EINVAL;
  if (d->dt <= 0 && !(d->cfl > 0)) return PAT_EINVAL;
  if (!(d->pml_alpha >= 0) || !std::isfinite(d->pml_alpha)) return PAT_EINVAL;
  if (lossy && !(d->alpha_power > 0 && d->alpha_power < 3 && d->alpha_power != 1.0)) return PAT_EINVAL;
  if (d->n_sensors < 1) return PAT_EINVAL;
  if (d->flags & ~(PAT_NO_PML | PAT_CHECK_FINITE | PAT_SMOOTH_P0 | PAT_EOS_INIT)) return PAT_EINVAL;
  return PAT_OK;
}

double plan_dt(const pat_desc& d, double c_max) {
  double dxmin = d.dx[0];
  for (int j = 1; j < d.ndim; ++j) dxmin = std::min(dxmin, d.dx[j]);
  return d.dt > 0 ? d.dt : d.cfl * dxmin / c_max;
}

int check_stability(const pat_desc& d, double c_max, double dt) {
  double dxmin = d.dx[0];
  for (int j = 1; j < d.ndim; ++j) dxmin = std::min(dxmin, d.dx[j]);
  if (!(c_max > 0) || !std::isfinite(c_max) || !(dt > 0) || !std::isfinite(dt)) return PAT_EINVAL;
  if (c_max * dt / dxmin > (1.0 / std::sqrt((double)d.ndim)) * (1.0 + 1e-12)) return PAT_EUNSTABLE;
  return PAT_OK;
}

double pml_factor(int n, int L, double alpha, double c_ref, double dx, double dt, int i, bool stag) {
  if (L <= 0) return 1.0;
  const double s = i + (stag ? 0.5 : 0.0);
  double depth = 0.0;
  if (s < L) depth = L - s;
  if (s > (n - 1 - L)) depth = s - (n - 1 - L);
  const double sigma = alpha * (c_ref / dx) * std::pow(depth / L, 4.0);
  return std::exp(-sigma * dt / 2.0);
}

// Linear-interpolation sensor operator: one gather tap per (sensor, row)
// with non-zero row weight; the transposed operator grouped by node.
int build_sensors(const pat_desc& d, const double* pos, SensorOps& so) {
  const int nd = d.ndim, ns = d.n_sensors;
  const int ny = d.n[1], nz = nd == 3 ? d.n[2] : 1;
  const int nrows = ny * nz;
  struct RowTap {
    int row, x0, slot, s;
    double w0, w1;
  };
  std::vector<RowTap> taps;
  so.slot_ptr.assign(ns + 1, 0);
  int slot = 0;
  for (int s = 0; s < ns; ++s) {
    int lo[3] = {0, 0, 0};
    double fr[3] = {0, 0, 0};
    for (int j = 0; j < nd; ++j) {
      const double g = (pos[(size_t)s * nd + j] - d.origin[j]) / d.dx[j];
      if (!(g >= 0.0) || !(g <= (double)(d.n[j] - 1))) return PAT_EINVAL;
      const int i0 = std::min((int)std::floor(g), d.n[j] - 2);
      lo[j] = i0;
      fr[j] = g - i0;
    }
    so.slot_ptr[s] = slot;
    const int nrow_taps = nd == 3 ? 4 : 2;
    for (int b = 0; b < nrow_taps; ++b) {
      const int by = b & 1, bz = (b >> 1) & 1;
      double w = by ? fr[1] : 1.0 - fr[1];
      if (nd == 3) w *= bz ? fr[2] : 1.0 - fr[2];
      if (w == 0.0) continue;
      const int row = (lo[1] + by) + (nd == 3 ? (lo[2] + bz) * ny : 0);
      taps.push_back(RowTap{row, lo[0], slot, s, w * (1.0 - fr[0]), w * fr[0]});
      ++slot;
    }
    if (slot == so.slot_ptr[s]) return PAT_EINVAL;  // cannot happen: weights sum to 1
  }
  so.slot_ptr[ns] = slot;
  so.nslots = slot;

  // gather: CSR by row
  std::stable_sort(taps.begin(), taps.end(), [](const RowTap& a, const RowTap& b) { return a.row < b.row; });
  so.g_ptr.assign(nrows + 1, 0);
  so.g_tap.clear();
  for (const auto& t : taps) {
    so.g_ptr[t.row + 1]++;
    so.g_tap.push_back(GTap{t.x0, t.slot, (float)t.w0, (float)t.w1});
  }
  for (int r = 0; r < nrows; ++r) so.g_ptr[r + 1] += so.g_ptr[r];

  // scatter: per row, node groups sorted by x, taps by sensor
  struct NodeTap {
    int row, x, s;
    double w;
  };
  std::vector<NodeTap> nt;
  for (const auto& t : taps) {
    if (t.w0 != 0.0) nt.push_back(NodeTap{t.row, t.x0, t.s, t.w0});
    if (t.w1 != 0.0) nt.push_back(NodeTap{t.row, t.x0 + 1, t.s, t.w1});
  }
  std::sort(nt.begin(), nt.end(), [](const NodeTap& a, const NodeTap& b) {
    if (a.row != b.row) return a.row < b.row;
    if (a.x != b.x) return a.x < b.x;
    return a.s < b.s;
  });
  so.s_ptr.assign(nrows + 1, 0);
  so.s_grp.clear();
  so.s_tap.clear();
  for (size_t i = 0; i < nt.size();) {
    size_t j = i;
    const int beg = (int)so.s_tap.size();
    while (j < nt.size() && nt[j].row == nt[i].row && nt[j].x == nt[i].x) {
      so.s_tap.push_back(STap{nt[j].s, (float)nt[j].w});
      ++j;
    }
    so.s_grp.push_back(SGroup{nt[i].x, beg, (int)so.s_tap.size()});
    so.s_ptr[nt[i].row + 1]++;
    i = j;
  }
  for (int r = 0; r < nrows; ++r) so.s_ptr[r + 1] += so.s_ptr[r];
  return PAT_OK;
}

}  // namespace pat

extern "C" int pat_desc_check(const pat_desc* desc, int32_t lossy, const double* sensor_pos, double c_max) {
  int rc = pat::validate_desc(desc, lossy != 0);
  if (rc) return rc;
  if (!sensor_pos) return PAT_EINVAL;
  if (c_max > 0) {  // c_max <= 0: the medium is not known yet, no stability check
    if (!std::isfinite(c_max)) return PAT_EINVAL;
    if ((rc = pat::check_stability(*desc, c_max, pat::plan_dt(*desc, c_max)))) return rc;
  }
  pat::SensorOps so;
  return pat::build_sensors(*desc, sensor_pos, so);
}
