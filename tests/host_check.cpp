// Host-only exercise of the plan set-up code (host_plan.cpp) for the
// sanitizer test: descriptor validation over valid and broken descriptors,
// the stability bound, and the sensor operator's CSR tables on random,
// edge and corner sensor positions in 2D and 3D, with their invariants:
//   * g_ptr / s_ptr monotone, ending at the tap / group counts;
//   * every slot appears in exactly one gather tap, slots of a sensor
//     contiguous, the weights of a sensor summing to one;
//   * the scatter tables are the transpose of the gather tables:
//     <W p, h> = <p, W^T h> for random p and h (float64 sums).
// Exit code 0 when every check holds; prints the first failure otherwise.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_1603_02329_amd/csrc/host_plan.h"

using namespace pat;

static int fails = 0;
#define CHECK(c, ...)                                   \
  do {                                                  \
    if (!(c)) {                                         \
      if (fails++ < 10) {                               \
        std::printf("FAIL line %d: ", __LINE__);        \
        std::printf(__VA_ARGS__);                       \
        std::printf("\n");                              \
      }                                                 \
    }                                                   \
  } while (0)

static pat_desc base_desc(int nd, const int* n) {
  pat_desc d{};
  d.ndim = nd;
  for (int j = 0; j < 3; ++j) {
    d.n[j] = j < nd ? n[j] : 1;
    d.dx[j] = 1e-4;
    d.origin[j] = -1e-3 * j;
    d.pml_size[j] = j < nd ? 2 : 0;
  }
  d.nt = 10;
  d.dt = 0.0;
  d.cfl = 0.3;
  d.pml_alpha = 2.0;
  d.alpha_power = 1.5;
  d.n_sensors = 1;
  d.flags = 0;
  return d;
}

static void check_sensors(const pat_desc& d, const std::vector<double>& pos, std::mt19937_64& rng) {
  SensorOps so;
  const int rc = build_sensors(d, pos.data(), so);
  CHECK(rc == PAT_OK, "build_sensors rc %d", rc);
  if (rc) return;
  const int nd = d.ndim, ns = d.n_sensors;
  const int nx = d.n[0], ny = d.n[1], nz = nd == 3 ? d.n[2] : 1;
  const int nrows = ny * nz;
  CHECK((int)so.g_ptr.size() == nrows + 1 && (int)so.s_ptr.size() == nrows + 1, "ptr sizes");
  CHECK(so.g_ptr[0] == 0 && so.g_ptr[nrows] == (int)so.g_tap.size(), "g_ptr ends");
  CHECK(so.s_ptr[0] == 0 && so.s_ptr[nrows] == (int)so.s_grp.size(), "s_ptr ends");
  for (int r = 0; r < nrows; ++r) {
    CHECK(so.g_ptr[r] <= so.g_ptr[r + 1], "g_ptr monotone at %d", r);
    CHECK(so.s_ptr[r] <= so.s_ptr[r + 1], "s_ptr monotone at %d", r);
    for (int g = so.s_ptr[r] + 1; g < so.s_ptr[r + 1]; ++g) CHECK(so.s_grp[g - 1].x < so.s_grp[g].x, "group order");
  }
  CHECK((int)so.slot_ptr.size() == ns + 1 && so.slot_ptr[ns] == so.nslots, "slot_ptr");
  std::vector<int> seen(so.nslots, 0);
  std::vector<double> wsum(ns, 0.0);
  std::vector<int> slot_sensor(so.nslots, -1);
  for (int s = 0; s < ns; ++s)
    for (int k = so.slot_ptr[s]; k < so.slot_ptr[s + 1]; ++k) slot_sensor[k] = s;
  for (int r = 0; r < nrows; ++r)
    for (int e = so.g_ptr[r]; e < so.g_ptr[r + 1]; ++e) {
      const GTap t = so.g_tap[e];
      CHECK(t.slot >= 0 && t.slot < so.nslots, "slot range");
      CHECK(t.x0 >= 0 && t.x0 + 1 < nx, "x0 range %d", t.x0);
      if (t.slot < 0 || t.slot >= so.nslots) continue;
      seen[t.slot]++;
      wsum[slot_sensor[t.slot]] += (double)t.w0 + (double)t.w1;
    }
  for (int k = 0; k < so.nslots; ++k) CHECK(seen[k] == 1, "slot %d seen %d times", k, seen[k]);
  for (int s = 0; s < ns; ++s) CHECK(std::fabs(wsum[s] - 1.0) < 1e-6, "weights of sensor %d sum %g", s, wsum[s]);
  // transpose identity
  std::normal_distribution<double> nrm;
  const long N = (long)nx * nrows;
  std::vector<double> p(N), h(ns), Wp(ns, 0.0), Wth(N, 0.0);
  for (auto& v : p) v = nrm(rng);
  for (auto& v : h) v = nrm(rng);
  for (int r = 0; r < nrows; ++r)
    for (int e = so.g_ptr[r]; e < so.g_ptr[r + 1]; ++e) {
      const GTap t = so.g_tap[e];
      Wp[slot_sensor[t.slot]] += t.w0 * p[(long)r * nx + t.x0] + t.w1 * p[(long)r * nx + t.x0 + 1];
    }
  for (int r = 0; r < nrows; ++r)
    for (int g = so.s_ptr[r]; g < so.s_ptr[r + 1]; ++g) {
      const SGroup grp = so.s_grp[g];
      CHECK(grp.x >= 0 && grp.x < nx && grp.beg <= grp.end && grp.end <= (int)so.s_tap.size(), "group range");
      for (int e = grp.beg; e < grp.end; ++e) {
        const STap t = so.s_tap[e];
        CHECK(t.s >= 0 && t.s < ns, "scatter sensor range");
        if (t.s >= 0 && t.s < ns) Wth[(long)r * nx + grp.x] += t.w * h[t.s];
      }
    }
  double a = 0, b = 0, na = 0;
  for (int s = 0; s < ns; ++s) a += Wp[s] * h[s], na += std::fabs(Wp[s] * h[s]);
  for (long q = 0; q < N; ++q) b += p[q] * Wth[q];
  CHECK(std::fabs(a - b) <= 1e-6 * (na + 1e-30), "transpose identity %g vs %g", a, b);
}

int main() {
  std::mt19937_64 rng(12345);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const int sizes2[][2] = {{16, 16}, {32, 16}, {16, 64}, {128, 32}};
  const int sizes3[][3] = {{16, 16, 16}, {32, 16, 16}, {16, 32, 64}};
  for (int pass = 0; pass < 2; ++pass) {
    const int count = pass == 0 ? 4 : 3;
    for (int c = 0; c < count; ++c) {
      const int nd = pass == 0 ? 2 : 3;
      const int* n = pass == 0 ? sizes2[c] : sizes3[c];
      pat_desc d = base_desc(nd, n);
      CHECK(validate_desc(&d, true) == PAT_OK, "valid desc rejected");
      // broken descriptors
      pat_desc e = d; e.n[0] = 24; CHECK(validate_desc(&e, true) == PAT_EINVAL, "n not pow2");
      e = d; e.n[nd - 1] = 8; CHECK(validate_desc(&e, true) == PAT_EINVAL, "n < 16");
      e = d; e.n[0] = nd == 3 ? 512 : 2048; CHECK(validate_desc(&e, true) == PAT_EINVAL, "n too large");
      e = d; e.dx[nd - 1] = -1; CHECK(validate_desc(&e, true) == PAT_EINVAL, "dx");
      e = d; e.dx[0] = NAN; CHECK(validate_desc(&e, true) == PAT_EINVAL, "dx nan");
      e = d; e.origin[0] = INFINITY; CHECK(validate_desc(&e, true) == PAT_EINVAL, "origin");
      e = d; e.pml_size[0] = n[0] / 2; CHECK(validate_desc(&e, true) == PAT_EINVAL, "pml");
      e = d; e.nt = 0; CHECK(validate_desc(&e, true) == PAT_EINVAL, "nt");
      e = d; e.cfl = 0; CHECK(validate_desc(&e, true) == PAT_EINVAL, "cfl");
      e = d; e.alpha_power = 1.0; CHECK(validate_desc(&e, true) == PAT_EINVAL && validate_desc(&e, false) == PAT_OK, "y");
      e = d; e.n_sensors = 0; CHECK(validate_desc(&e, true) == PAT_EINVAL, "ns");
      e = d; e.flags = 0x20; CHECK(validate_desc(&e, true) == PAT_EINVAL, "flags");
      e = d; e.flags = 0x4; CHECK(validate_desc(&e, true) == PAT_EINVAL, "flags 0x4");
      e = d; e.flags = PAT_EOS_INIT | PAT_SMOOTH_P0; CHECK(validate_desc(&e, true) == PAT_OK, "flags eos");
      e = d; e.ndim = 4; CHECK(validate_desc(&e, true) == PAT_EINVAL, "ndim");
      CHECK(validate_desc(nullptr, true) == PAT_EINVAL, "null");
      // stability
      const double cm = 1550.0, bound = d.dx[0] / (cm * std::sqrt((double)nd));
      e = d; e.dt = 0.999 * bound; CHECK(check_stability(e, cm, plan_dt(e, cm)) == PAT_OK, "stable");
      e = d; e.dt = 1.001 * bound; CHECK(check_stability(e, cm, plan_dt(e, cm)) == PAT_EUNSTABLE, "unstable");
      CHECK(check_stability(d, NAN, 1e-9) == PAT_EINVAL, "nan c");
      // PML factor in (0, 1], 1 outside the layer
      for (int i = 0; i < n[0]; ++i) {
        const double q = pml_factor(n[0], 2, 2.0, cm, 1e-4, 2e-8, i, i & 1);
        CHECK(q > 0 && q <= 1.0, "pml factor %g", q);
      }
      // sensors: random interior, on the edges and corners, on the last node
      for (int trial = 0; trial < 20; ++trial) {
        const int ns = 1 + (int)(U(rng) * 200);
        d.n_sensors = ns;
        std::vector<double> pos((size_t)ns * nd);
        for (int s = 0; s < ns; ++s)
          for (int j = 0; j < nd; ++j) {
            double g = U(rng) * (n[j] - 1);
            const double r = U(rng);
            if (r < 0.1) g = 0.0;
            else if (r < 0.2) g = n[j] - 1;
            else if (r < 0.3) g = std::floor(g);
            pos[(size_t)s * nd + j] = d.origin[j] + g * d.dx[j];
            if (pos[(size_t)s * nd + j] > d.origin[j] + (n[j] - 1) * d.dx[j])
              pos[(size_t)s * nd + j] = d.origin[j] + (n[j] - 1) * d.dx[j];
          }
        check_sensors(d, pos, rng);
        // one sensor pushed outside on a random axis: rejected
        const int s = (int)(U(rng) * ns), j = (int)(U(rng) * nd);
        std::vector<double> bad = pos;
        bad[(size_t)s * nd + j] = U(rng) < 0.5 ? d.origin[j] - 0.5 * d.dx[j] : d.origin[j] + (n[j] - 0.5) * d.dx[j];
        SensorOps so;
        CHECK(build_sensors(d, bad.data(), so) == PAT_EINVAL, "outside sensor accepted");
        bad[(size_t)s * nd + j] = NAN;
        CHECK(build_sensors(d, bad.data(), so) == PAT_EINVAL, "nan sensor accepted");
      }
    }
  }
  if (fails) {
    std::printf("%d failures\n", fails);
    return 1;
  }
  std::printf("host_check: all checks passed\n");
  return 0;
}
