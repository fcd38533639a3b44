// Host runtime of libpat: plan construction, eager executors, C entry points.
//
// Plan construction derives every coefficient of the scheme in float64 and
// rounds each once to float32:
//   B_j     = dt / rho0_sg,j   (rho0 on the staggered points: mean of the two
//                               neighbours, the last index keeps its value)
//   dtr0    = dt rho0,  c2 = c0^2,  inv_dc2 = 1 / (d c0^2)
//   c2tau   = c0^2 tau, c2eta = c0^2 eta with tau = -2 a0 c0^(y-1),
//             eta = 2 a0 c0^y tan(pi y / 2)           (equation Twelve)
//   a0      = alpha0_dB * 100 * (1e-6 / 2pi)^y / (20 log10 e)  [Np/((rad/s)^y m)]
// plus the per-axis PML factors, the per-axis wavenumber tables and the
// sensor interpolation operator with its transpose.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "host_plan.h"
#include "pat_internal.h"

namespace pat {
hipError_t upload_twiddles_rows(const Tw* host);
hipError_t upload_twiddles_cols(const Tw* host);
hipError_t upload_twiddles_fused(const Tw* host);
}

using namespace pat;


namespace {

#define PAT_TRY_HIP(x)                 \
  do {                                 \
    hipError_t e_ = (x);               \
    if (e_ != hipSuccess) return PAT_EHIP; \
  } while (0)

std::mutex g_tw_mu;
std::vector<int> g_tw_ready;  // per device

int ensure_twiddles() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PAT_EHIP;
  std::lock_guard<std::mutex> lk(g_tw_mu);
  if ((int)g_tw_ready.size() <= dev) g_tw_ready.resize(dev + 1, 0);
  if (g_tw_ready[dev]) return PAT_OK;
  std::vector<Tw> tw(TWN);
  for (int q = 0; q < TWN; ++q) {
    const double a = -2.0 * M_PI * (double)q / (double)TWN;
    const double c = std::cos(a), s = std::sin(a);
    const float ch = (float)c, sh = (float)s;
    tw[q] = Tw{ch, sh, (float)(c - (double)ch), (float)(s - (double)sh)};
  }
  if (upload_twiddles_rows(tw.data()) != hipSuccess || upload_twiddles_cols(tw.data()) != hipSuccess ||
      upload_twiddles_fused(tw.data()) != hipSuccess)
    return PAT_EHIP;
  g_tw_ready[dev] = 1;
  return PAT_OK;
}

// Bump allocator over one device arena (256-byte aligned pieces).  Each
// piece starts 129 x 256 B past the end of the previous one: without that
// gap the N-float fields of a plan (1 MB each at 512^2) sit a power of two
// apart, and a pass that streams several of them at the same index drives
// them through the same few memory channels.  Measured on the 48-instance
// 2D forward + adjoint (same box, three alternating rounds): 686-689 ms
// against 696-700 ms with no gap; gaps of 65, 97, 161, 193, 257 and 1025
// x 256 B gave 689-693 ms, 513 x 256 B 704-707 ms; 128^3 unchanged.
constexpr size_t kPieceGap = 129 * 256;
struct Carve {
  size_t off = 0;
  template <class T>
  size_t take(size_t count) {
    off = (off + kPieceGap + 255) & ~size_t(255);
    const size_t at = off;
    off += count * sizeof(T);
    return at;
  }
};

}  // namespace

// ===================================================================== plan
extern "C" int pat_plan_create(pat_plan** out, const pat_desc* desc, const float* c0_d, const float* rho0_d,
                               const float* alpha0_d, const double* sensor_pos, void* stream) {
  if (!out) return PAT_EINVAL;
  *out = nullptr;
  const bool lossy = alpha0_d != nullptr;
  int rc = validate_desc(desc, lossy);
  if (rc) return rc;
  if (!c0_d || !rho0_d || !sensor_pos) return PAT_EINVAL;
  const pat_desc d = *desc;
  hipStream_t st = (hipStream_t)stream;
  const int nd = d.ndim;
  const int nx = d.n[0], ny = d.n[1], nz = nd == 3 ? d.n[2] : 1;
  const int64_t N = (int64_t)nx * ny * nz;
  if ((rc = ensure_twiddles())) return rc;

  // medium to host (float32 inputs, widened to float64)
  std::vector<float> c0(N), rho0(N), a0db(lossy ? N : 0);
  PAT_TRY_HIP(hipMemcpyAsync(c0.data(), c0_d, N * 4, hipMemcpyDeviceToHost, st));
  PAT_TRY_HIP(hipMemcpyAsync(rho0.data(), rho0_d, N * 4, hipMemcpyDeviceToHost, st));
  if (lossy) PAT_TRY_HIP(hipMemcpyAsync(a0db.data(), alpha0_d, N * 4, hipMemcpyDeviceToHost, st));
  PAT_TRY_HIP(hipStreamSynchronize(st));
  for (int64_t i = 0; i < N; ++i) {
    if (!(c0[i] > 0) || !std::isfinite(c0[i]) || !(rho0[i] > 0) || !std::isfinite(rho0[i])) return PAT_EINVAL;
    if (lossy && (!(a0db[i] >= 0) || !std::isfinite(a0db[i]))) return PAT_EINVAL;
  }
  std::vector<double> cd(c0.begin(), c0.end()), rd(rho0.begin(), rho0.end());
  double cmax = 0;
  for (int64_t i = 0; i < N; ++i) {
    if (!(cd[i] > 0) || !(rd[i] > 0)) return PAT_EINVAL;
    cmax = std::max(cmax, cd[i]);
  }
  const double dt = plan_dt(d, cmax);
  if ((rc = check_stability(d, cmax, dt))) return rc;

  SensorOps so;
  if ((rc = build_sensors(d, sensor_pos, so))) return rc;

  auto* p = new (std::nothrow) pat_plan();
  if (!p) return PAT_ENOMEM;
  p->desc = d;
  hipGetDevice(&p->device);
  p->dt = dt;
  p->c_ref = cmax;
  p->lossy = lossy;
  p->npoints = N;
  p->nslots = so.nslots;

  // ---- device arena layout
  const int M = nx / 2;
  Carve cv;
  size_t oB[3] = {0, 0, 0}, oQ[3], oQs[3], oK[3], oA[3], oBb[3], oW[3], oU[3] = {0, 0, 0}, oR[3] = {0, 0, 0};
  for (int j = 0; j < nd; ++j) oB[j] = cv.take<float>(N);
  const size_t o_dtr0 = cv.take<float>(N), o_c2 = cv.take<float>(N), o_inv = cv.take<float>(N);
  const size_t o_c2tau = lossy ? cv.take<float>(N) : 0, o_c2eta = lossy ? cv.take<float>(N) : 0;
  int tlen[3];
  for (int j = 0; j < nd; ++j) {
    tlen[j] = (j == 0) ? M + 1 : d.n[j];
    oQ[j] = cv.take<float>(d.n[j]);
    oQs[j] = cv.take<float>(d.n[j]);
    oK[j] = cv.take<float>(tlen[j]);
    oA[j] = cv.take<float2>(tlen[j]);
    oBb[j] = cv.take<float2>(tlen[j]);
    oW[j] = cv.take<float>(tlen[j]);
  }
  // forward state between two steps: u_j, rho_j and the x-spectrum of p (S0),
  // one range from u_0 (gaps included) so that a snapshot is one copy
  size_t oS[4] = {0, 0, 0, 0};
  for (int j = 0; j < nd; ++j) oU[j] = cv.take<float>(N);
  for (int j = 0; j < nd; ++j) oR[j] = cv.take<float>(N);
  oS[0] = cv.take<float2>((size_t)N / 2);
  const size_t state_begin = oU[0], state_end = cv.off;
  const size_t o_q = cv.take<float>(N);
  for (int j = 1; j <= nd; ++j) oS[j] = cv.take<float2>((size_t)N / 2);
  const size_t o_gptr = cv.take<int32_t>(so.g_ptr.size()), o_gtap = cv.take<GTap>(std::max<size_t>(1, so.g_tap.size()));
  const size_t o_sptr = cv.take<int32_t>(so.s_ptr.size()), o_sgrp = cv.take<SGroup>(std::max<size_t>(1, so.s_grp.size()));
  const size_t o_stap = cv.take<STap>(std::max<size_t>(1, so.s_tap.size()));
  const size_t o_sc = cv.take<float>(std::max<size_t>(1, (size_t)d.nt * so.s_grp.size()));
  const size_t o_slot = cv.take<int32_t>(so.slot_ptr.size());
  const size_t o_part = cv.take<float>((size_t)d.nt * so.nslots);
  const size_t o_bad = cv.take<int32_t>(1);
  const size_t o_rec = cv.take<DevPlan>(1);
  p->arena_bytes = (cv.off + 255) & ~size_t(255);
  p->state_bytes = state_end - state_begin;
  if (hipMalloc(&p->arena, p->arena_bytes) != hipSuccess) {
    delete p;
    return PAT_ENOMEM;
  }
  char* A = (char*)p->arena;

  // ---- host-side coefficient arrays (float64 -> float32 once)
  std::vector<char> hbuf(state_begin, 0);
  auto hf = [&](size_t off) { return reinterpret_cast<float*>(hbuf.data() + off); };
  auto hc = [&](size_t off) { return reinterpret_cast<float2*>(hbuf.data() + off); };
  const int64_t strides[3] = {1, nx, (int64_t)nx * ny};
  const double y = d.alpha_power;
  const double a_conv = 100.0 * std::pow(1e-6 / (2.0 * M_PI), y) / (20.0 * std::log10(std::exp(1.0)));
  const double tan_y = std::tan(M_PI * y / 2.0);
  double max_eta = 0.0;  // max |eta| over the medium (PAT_EOS_INIT's contraction)
  for (int64_t i = 0; i < N; ++i) {
    const double c = cd[i], r = rd[i];
    for (int j = 0; j < nd; ++j) {
      const int64_t ij = (i / strides[j]) % d.n[j];
      const double rn = (ij + 1 < d.n[j]) ? rd[i + strides[j]] : r;
      hf(oB[j])[i] = (float)(dt / (0.5 * (r + rn)));
    }
    hf(o_dtr0)[i] = (float)(dt * r);
    hf(o_c2)[i] = (float)(c * c);
    hf(o_inv)[i] = (float)(1.0 / (nd * c * c));
    if (lossy) {
      const double a0 = (double)a0db[i] * a_conv;
      const double tau = -2.0 * a0 * std::pow(c, y - 1.0);
      const double eta = 2.0 * a0 * std::pow(c, y) * tan_y;
      hf(o_c2tau)[i] = (float)(c * c * tau);
      hf(o_c2eta)[i] = (float)(c * c * eta);
      max_eta = std::max(max_eta, std::fabs(eta));
    }
  }
  // PAT_EOS_INIT: the fixed-point steps x <- b + eta L2 x contract by at most
  // max |eta| max_k |k|^(y-1) (|k| at the grid's corner for y > 1, the
  // lowest nonzero |k| for y < 1)
  if ((d.flags & PAT_EOS_INIT) && lossy && d.nt > 1) {
    double kmax2 = 0.0, kmin = 1e300;
    for (int j = 0; j < nd; ++j) {
      kmax2 += (M_PI / d.dx[j]) * (M_PI / d.dx[j]);
      kmin = std::min(kmin, 2.0 * M_PI / (d.n[j] * d.dx[j]));
    }
    const double kf = std::pow(y > 1.0 ? std::sqrt(kmax2) : kmin, y - 1.0);
    if (!(max_eta * kf <= kEosMaxContraction)) {
      hipFree(p->arena);
      delete p;
      return PAT_EINVAL;
    }
  }
  const bool pml_on = !(d.flags & PAT_NO_PML);
  for (int j = 0; j < nd; ++j) {
    const int n = d.n[j];
    const int L = pml_on ? d.pml_size[j] : 0;
    for (int i = 0; i < n; ++i) {
      hf(oQ[j])[i] = (float)pml_factor(n, L, d.pml_alpha, cmax, d.dx[j], dt, i, false);
      hf(oQs[j])[i] = (float)pml_factor(n, L, d.pml_alpha, cmax, d.dx[j], dt, i, true);
    }
    for (int m = 0; m < tlen[j]; ++m) {
      const int mt = (m < n / 2) ? m : m - n;
      const double k = 2.0 * M_PI * mt / (n * d.dx[j]);
      const double h = k * d.dx[j] / 2.0;
      hf(oK[j])[m] = (float)(k * k);
      // Blackman window centred on k = 0 (1 there, 0 at the Nyquist bin)
      hf(oW[j])[m] = (float)(0.42 + 0.5 * std::cos(2.0 * M_PI * m / n) + 0.08 * std::cos(4.0 * M_PI * m / n));
      if (2 * m == n) {  // Nyquist: i k e^{+-i pi/2} is exactly real
        hc(oA[j])[m] = make_float2((float)k, 0.f);
        hc(oBb[j])[m] = make_float2((float)(-k), 0.f);
      } else {
        hc(oA[j])[m] = make_float2((float)(-k * std::sin(h)), (float)(k * std::cos(h)));
        hc(oBb[j])[m] = make_float2((float)(k * std::sin(h)), (float)(k * std::cos(h)));
      }
    }
  }
  // from here on every error path releases the arena and the plan
  rc = hipMemcpyAsync(A, hbuf.data(), state_begin, hipMemcpyHostToDevice, st) == hipSuccess ? PAT_OK : PAT_EHIP;

  auto up = [&](size_t off, const void* src, size_t bytes) -> int {
    if (bytes == 0) return PAT_OK;
    return hipMemcpyAsync(A + off, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess ? PAT_OK : PAT_EHIP;
  };
  if (!rc) rc = up(o_gptr, so.g_ptr.data(), so.g_ptr.size() * 4);
  if (!rc) rc = up(o_gtap, so.g_tap.data(), so.g_tap.size() * sizeof(GTap));
  if (!rc) rc = up(o_sptr, so.s_ptr.data(), so.s_ptr.size() * 4);
  if (!rc) rc = up(o_sgrp, so.s_grp.data(), so.s_grp.size() * sizeof(SGroup));
  if (!rc) rc = up(o_stap, so.s_tap.data(), so.s_tap.size() * sizeof(STap));
  if (!rc) rc = up(o_slot, so.slot_ptr.data(), so.slot_ptr.size() * 4);
  if (!rc && hipMemsetAsync(A + o_bad, 0, 4, st) != hipSuccess) rc = PAT_EHIP;

  DevPlan& h = p->hp;
  h.ndim = nd;
  h.n[0] = nx;
  h.n[1] = ny;
  h.n[2] = nz;
  h.nrows = ny * nz;
  h.nt = d.nt;
  h.ns = d.n_sensors;
  h.nslots = so.nslots;
  h.lossy = lossy;
  h.flags = d.flags;
  h.dt = (float)dt;
  h.kap2 = (float)((cmax * dt / 2.0) * (cmax * dt / 2.0));
  h.ym2h = (float)((y - 2.0) / 2.0);
  h.ym1h = (float)((y - 1.0) / 2.0);
  h.inv_dt = (float)(1.0 / dt);
  // uniform absorption coefficient: the state passes form c0^2 tau and
  // c0^2 eta from c0^2 instead of reading them
  h.alpha_uniform = 0;
  if (lossy) {
    bool uni = true;
    for (int64_t i = 1; i < N && uni; ++i) uni = (a0db[i] == a0db[0]);
    if (uni) {
      const double a0 = (double)a0db[0] * a_conv;
      h.alpha_uniform = 1;
      h.ktau = (float)(-2.0 * a0);             // c0^2 tau = -2 a0 c0^(y+1)
      h.etau = (float)((y + 1.0) / 2.0);
      h.keta = (float)(2.0 * a0 * tan_y);      // c0^2 eta = 2 a0 tan(pi y/2) c0^(y+2)
      h.eeta = (float)((y + 2.0) / 2.0);
    }
  }
  h.scale = (float)(1.0 / (double)N);
  for (int j = 0; j < nd; ++j) {
    h.B[j] = (const float*)(A + oB[j]);
    h.Q[j] = (const float*)(A + oQ[j]);
    h.Qsg[j] = (const float*)(A + oQs[j]);
    h.ksq[j] = (const float*)(A + oK[j]);
    h.shA[j] = (const float2*)(A + oA[j]);
    h.shB[j] = (const float2*)(A + oBb[j]);
    h.win[j] = (const float*)(A + oW[j]);
    h.u[j] = (float*)(A + oU[j]);
    h.r[j] = (float*)(A + oR[j]);
  }
  h.dtr0 = (const float*)(A + o_dtr0);
  h.c2 = (const float*)(A + o_c2);
  h.inv_dc2 = (const float*)(A + o_inv);
  h.c2tau = lossy ? (const float*)(A + o_c2tau) : nullptr;
  h.c2eta = lossy ? (const float*)(A + o_c2eta) : nullptr;
  h.q = (float*)(A + o_q);
  for (int j = 0; j <= nd; ++j) h.S[j] = (float2*)(A + oS[j]);
  h.g_ptr = (const int32_t*)(A + o_gptr);
  h.g_tap = (const GTap*)(A + o_gtap);
  h.s_ptr = (const int32_t*)(A + o_sptr);
  h.s_grp = (const SGroup*)(A + o_sgrp);
  h.s_tap = (const STap*)(A + o_stap);
  h.sc = (float*)(A + o_sc);
  h.ngroups = (int32_t)so.s_grp.size();
  h.slot_ptr = (const int32_t*)(A + o_slot);
  h.partial = (float*)(A + o_part);
  h.bad = (int32_t*)(A + o_bad);
  p->dp = (DevPlan*)(A + o_rec);
  if (!rc) rc = up(o_rec, &h, sizeof(DevPlan));
  if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = PAT_EHIP;
  if (rc) {
    hipStreamSynchronize(st);  // no copy may still read the host tables or write the arena
    hipFree(p->arena);
    delete p;
    return rc;
  }
  *out = p;
  return PAT_OK;
}

extern "C" void pat_plan_destroy(pat_plan* p) {
  if (!p) return;
  hipDeviceSynchronize();
  batch_cache_forget(p);
  hipFree(p->arena);
  delete p;
}

extern "C" int pat_plan_info(const pat_plan* p, pat_info* info) {
  if (!p || !info) return PAT_EINVAL;
  info->dt = p->dt;
  info->c_ref = p->c_ref;
  info->npoints = p->npoints;
  info->lossy = p->lossy;
  info->n_slots = p->nslots;
  info->device_bytes = p->arena_bytes;
  info->state_bytes = p->state_bytes;
  return PAT_OK;
}

extern "C" int pat_plan_sync(pat_plan* p, void* stream) {
  if (!p) return PAT_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PAT_EHIP;
  int32_t bad = 0;
  if (hipMemcpy(&bad, p->hp.bad, 4, hipMemcpyDeviceToHost) != hipSuccess) return PAT_EHIP;
  if (bad) {
    if (hipMemset(p->hp.bad, 0, 4) != hipSuccess) return PAT_EHIP;
    return PAT_ENONFINITE;
  }
  return PAT_OK;
}

extern "C" const char* pat_strerror(int code) {
  switch (code) {
    case PAT_OK: return "ok";
    case PAT_EINVAL: return "invalid argument";
    case PAT_EUNSTABLE: return "time step above the stability bound";
    case PAT_ENOMEM: return "out of memory";
    case PAT_EHIP: return "HIP runtime error";
    case PAT_ENONFINITE: return "non-finite pressure produced";
    case PAT_ENOSYS: return "not supported by this library";
    case PAT_ETOOBIG: return "larger than the fixed scratch of the no-allocation entry point";
  }
  return "unknown error";
}

