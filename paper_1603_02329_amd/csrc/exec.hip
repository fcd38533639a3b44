// Executors of the time loop: eager (one instance, launches on the caller's
// stream) and batched (many instances, one launch per pass over a work table
// of every instance of a size class, time loop captured into HIP graphs).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "pat_internal.h"

namespace pat {

// ------------------------------------------------------------------ pass sequences
int step_ops(int dir, int ndim, int lossy, PassOp* ops) {
  int n = 0;
  auto row = [&](RowKind k) { ops[n++] = PassOp{0, k, ColSpec{0, 0, {0, 0, 0}, 0}}; };
  auto col = [&](int mode, int nf, int f0, int a, int b, int c) {
    ops[n++] = PassOp{1, R_COUNT, ColSpec{mode, nf, {a, b, c}, f0}};
  };
  // spectral operator on fields [f0, f0+nf) along the remaining axes: 2D one
  // column pass; 3D a y-transform pass, the z pass with the multipliers and
  // the inverse y-transform of the outputs
  auto spec = [&](int mode, int nf, int f0, int a, int b, int c) {
    if (ndim == 2) {
      col(mode, nf, f0, a, b, c);
      return;
    }
    const int in0 = (mode == 0) ? 0 : f0, nin = (mode == 0) ? 1 : nf;
    const int out0 = (mode == 2) ? 0 : (mode == 0 ? 1 : f0), nout = (mode == 2) ? 1 : nf;
    col(3, nin, in0, 0, 0, 0);
    col(mode, nf, f0, a, b, c);
    col(4, nout, out0, 0, 0, 0);
  };
  const int d = ndim;
  if (dir == 0) {
    spec(0, d, 1, M_AX, M_AY, M_AZ);    // gradient of p at the staggered points
    row(R_FWD_1);                        // velocity update
    spec(1, d, 1, M_BX, M_BY, M_BZ);    // divergence components back on the nodes
    if (lossy) {
      row(R_FWD_2);                      // density update
      spec(1, 2, 1, M_L1DT, M_L2, 0);    // fractional Laplacians
      row(R_FWD_3);                      // equation of state + sensors
    } else {
      row(R_FWD_2LL);                    // density update + equation of state + sensors
    }
  } else if (dir == 2) {
    // adjoint-then-discretize: the forward's passes, density and state in
    // the adjoint system's form
    spec(0, d, 1, M_AX, M_AY, M_AZ);
    row(R_FWD_1);
    spec(1, d, 1, M_BX, M_BY, M_BZ);
    if (lossy) {
      row(R_ATD_2);
      spec(1, 2, 1, M_L1DT, M_L2, 0);
      row(R_ATD_3);
    } else {
      row(R_ATD_2LL);
    }
  } else {
    if (lossy) {
      row(R_ADJ_3);
      spec(1, 2, 1, M_L2, M_L1DT, 0);
      row(R_ADJ_2);
    } else {
      row(R_ADJ_32LL);
    }
    spec(1, d, 1, M_AX, M_AY, M_AZ);
    row(R_ADJ_1);
    spec(2, d, 1, M_BX, M_BY, M_BZ);
  }
  return n;
}

double pass_bytes_per_point(const PassOp& op, int ndim, int lossy) {
  (void)lossy;
  const int d = ndim;
  if (op.is_col) {
    const int f = op.col.nfield;
    // packed spectra: 4 bytes per grid point and field
    if (op.col.mode == 0) return 4.0 * (1 + f);  // one input, f outputs
    if (op.col.mode == 2) return 4.0 * (f + 1);
    return 8.0 * f;  // modes 1, 3, 4: each field read and written
  }
  switch (op.row) {
    case R_FWD_INIT: return 4.0 * (d + 3);       // p0, 1/(d c0^2) -> rho_j, S0
    case R_FWD_1: return 20.0 * d;               // S_j, u_j, B_j -> u_j, S_j
    case R_FWD_2: return 4.0 * (3 * d + 3);      // S_j, rho_j, dt rho0 -> rho_j, S1, S2
    case R_FWD_2LL: return 4.0 * (3 * d + 3);    // S_j, rho_j, dt rho0, c0^2 -> rho_j, S0
    case R_FWD_3: return 4.0 * (d + 6);          // S1, S2, rho_j, c0^2, c0^2 tau, c0^2 eta -> S0 (algorithmic)
    case R_ADJ_3: return 28.0;                   // S0, c0^2, c0^2 eta, c0^2 tau -> q, S1, S2
    case R_ADJ_32LL: return 4.0 * (3 * d + 3);   // S0, c0^2, rho_j, dt rho0 -> rho_j, S_j
    case R_ADJ_2: return 4.0 * (3 * d + 4);      // S1, S2, q, rho_j, dt rho0 -> rho_j, S_j
    case R_ADJ_1: return 20.0 * d;               // S_j, u_j, B_j -> u_j, S_j
    case R_ADJ_FINAL: return 4.0 * (d + 3);      // S0, rho_j, 1/(d c0^2) -> image
    case R_ADJ_SCATTER_ONLY: return 4.0;
    case R_ATD_2: return 4.0 * (3 * d + 4);      // S_j, rho_j, dt rho0, c0^2 -> rho_j, S1, S2
    case R_ATD_2LL: return 4.0 * (3 * d + 3);    // S_j, rho_j, dt rho0, c0^2 -> rho_j, S0
    case R_ATD_3: return 4.0 * (d + 5);          // S1, S2, rho_j, c0^2, dt rho0 -> S0
    case R_ATD_FINAL: return 4.0 * (d + 2);      // rho_j, dt rho0 -> image
    case R_FILT_IN: return 8.0;                  // field -> S0
    case R_FWD_INIT_F: return 4.0 * (d + 3);     // S0, 1/(d c0^2) -> rho_j, S0
    case R_FILT_RE: return 8.0;                  // image -> S0
    case R_FILT_OUT: return 8.0;                 // S0 -> image
    default: return 0.0;
  }
}

namespace {

// ------------------------------------------------------------------ event timing
struct Timing {
  int dir = -1, index = -1, nx = 0;
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  double bytes = 0;
  long launches = 0;
};
std::mutex g_tmu;
Timing g_timing;
bool g_timing_on = false;

// Event pair for one launch of the timed pass (or none): the kernel launch
// stamps the events at its own start and end (hipExtLaunchKernelGGL), so the
// elapsed time is the kernel's duration alone.
struct TimeScope {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TimeScope(int dir, int idx, int nx, double bytes) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing_on || g_timing.dir != dir || g_timing.index != idx) return;
    if (g_timing.nx && g_timing.nx != nx) return;
    if (g_timing.used + 2 > g_timing.ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
      g_timing.ev.push_back(a);
      g_timing.ev.push_back(b);
    }
    e0 = g_timing.ev[g_timing.used];
    e1 = g_timing.ev[g_timing.used + 1];
    g_timing.used += 2;
    g_timing.bytes += bytes;
    g_timing.launches += 1;
  }
};

__global__ void k_set_io(DevPlan* p, const float* in, float* out) {
  p->in = in;
  p->out = out;
}

constexpr int kIoMax = 64;
constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, one L2 each
struct IoArgs {
  const float* in[kIoMax];
  float* out[kIoMax];
};
__global__ void k_set_io_many(DevPlan* recs, int nb, IoArgs a) {
  const int i = threadIdx.x;
  if (i < nb) {
    recs[i].in = a.in[i];
    recs[i].out = a.out[i];
  }
}
// W^T h of every sample, one sum per node group of the scatter operator (a
// grid node that sensor taps land on), for the adjoint state passes: their
// step's sums are then two independent loads per lane, issued before the
// step's transform, instead of a chain of four dependent loads after it.
// The sums run over a group's taps in the order the passes used (bitwise
// the same values).  Block row y: plan y of `plans`.
constexpr int kScatterThreads = 256;
__global__ void __launch_bounds__(kScatterThreads) k_scatter_sums(const DevPlan* __restrict__ plans) {
  const DevPlan& P = plans[blockIdx.y];
  const long total = (long)P.nt * P.ngroups;
  for (long i = (long)blockIdx.x * kScatterThreads + threadIdx.x; i < total; i += (long)gridDim.x * kScatterThreads) {
    const int n = (int)(i / P.ngroups), g = (int)(i - (long)n * P.ngroups);
    const SGroup grp = P.s_grp[g];
    const float* h = P.in + (long)n * P.ns;
    float acc = 0.f;
    for (int e = grp.beg; e < grp.end; ++e) {
      const STap tp = P.s_tap[e];
      acc = fmaf(tp.w, h[tp.s], acc);
    }
    P.sc[i] = acc;
  }
}
int scatter_sums(const DevPlan* recs, int nplans, long max_total, hipStream_t st) {
  if (nplans < 1 || max_total < 1) return PAT_OK;
  const int nb = (int)std::min<long>(1024, (max_total + kScatterThreads - 1) / kScatterThreads);
  hipLaunchKernelGGL(k_scatter_sums, dim3(nb, nplans), dim3(kScatterThreads), 0, st, recs);
  return hipGetLastError() == hipSuccess ? PAT_OK : PAT_EHIP;
}

__global__ void k_set_ctr(int32_t* c, int v) { *c = v; }
__global__ void k_add_ctr(int32_t* c, int v) { *c += v; }

// ------------------------------------------------------------------ runner
// Launch geometry of one group of same-shape instances (one, for eager).
constexpr int kColW = 4;  // column tile widths a batch holds work tables for

struct Runner {
  int ndim, nx, ny, nz, nt, lossy;
  int fused = 0;  // fused launches over instances of several sizes (passes_fused.hip)
  int span = 0;   // fused: steps of the longest instance
  const DevPlan* recs;
  const int2 *row_tab, *red_tab;
  int row_n, red_n;
  // column work tables, one per tile width (none for eager: the block index
  // is the tile of instance 0)
  const int2* col_tabs[kColW];
  int col_ns[kColW], col_ws[kColW], col_bpi[kColW], ncolw;
  const ColVariant* vars;  // chosen variant of pass [dir * kMaxOps + idx] (tile 0: default)
  double points;     // grid points covered by one launch (all instances)
  // fused: per instance grid points and nt (host arrays of ninst entries)
  const double* inst_points = nullptr;
  const int* inst_nt = nullptr;
  int ninst = 0;

  // grid points of the instances a launch at step `step` runs (a fused
  // launch inside the time loop skips the instances not due at that step)
  double points_at(const StepArg& sa) const {
    if (!fused || sa.span <= 0 || sa.ctr) return points;
    double p = 0;
    for (int i = 0; i < ninst; ++i) {
      const long S = inst_nt[i] - 1;
      if (((long)sa.k + 1) * S / sa.span > (long)sa.k * S / sa.span) p += inst_points[i];
    }
    return p;
  }
  int op(int dir, int idx, const PassOp& o, StepArg sa, hipStream_t st, bool timed) const {
    if (timed) {
      const TimeScope ts(dir, idx, nx, pass_bytes_per_point(o, ndim, lossy) * points_at(sa));
      return launch1(dir, idx, o, sa, st, ts.e0, ts.e1);
    }
    return launch1(dir, idx, o, sa, st, nullptr, nullptr);
  }
  int launch_col_w(ColSpec s, ColVariant v, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
                   StepArg sa = StepArg{nullptr, 0}) const {
    if (fused) {
      if (v.tile == 0) v = ColVariant{8, 1};
      for (int j = 0; j < ncolw; ++j)
        if (col_ws[j] == v.tile)
          return launch_col_fused(s, v, Launch{recs, col_tabs[j], col_ns[j], st, e0, e1}, sa) == hipSuccess
                     ? PAT_OK
                     : PAT_EHIP;
      return PAT_EHIP;
    }
    s.tile = v.tile;
    s.fpb = v.fpb;
    v = col_variant_of(s, ndim, ny, nz);
    s.tile = v.tile;
    s.fpb = v.fpb;
    const int w = v.tile;
    const int2* tab = nullptr;
    int n = col_blocks(s, ndim, nx, ny, nz);
    for (int j = 0; j < ncolw; ++j)
      if (col_ws[j] == w && col_bpi[j] == n) tab = col_tabs[j], n = col_ns[j];
    if (ncolw && !tab) return PAT_EHIP;
    return launch_col(s, ndim, nx, ny, nz, Launch{recs, tab, n, st, e0, e1}) == hipSuccess ? PAT_OK : PAT_EHIP;
  }
  int launch1(int dir, int idx, const PassOp& o, StepArg sa, hipStream_t st, hipEvent_t e0, hipEvent_t e1) const {
    if (o.is_col) return launch_col_w(o.col, vars ? vars[dir * kMaxOps + idx] : ColVariant{0, 1}, st, e0, e1, sa);
    const Launch L{recs, row_tab, row_n, st, e0, e1};
    const hipError_t e = fused ? launch_row_fused(o.row, L, sa) : launch_row(o.row, ndim, nx, L, sa);
    return e == hipSuccess ? PAT_OK : PAT_EHIP;
  }
  int row(RowKind k, StepArg sa, hipStream_t st) const {
    const Launch L{recs, row_tab, row_n, st};
    const hipError_t e = fused ? launch_row_fused(k, L, sa) : launch_row(k, ndim, nx, L, sa);
    return e == hipSuccess ? PAT_OK : PAT_EHIP;
  }
  // S0 <- w S0: the smoothing window of p0 along y (2D), or along y and z
  // between the y-transform passes (3D); the x factor rides in the same pass
  int window(hipStream_t st) const {
    const ColSpec w{1, 1, {M_WIN, 0, 0}, 0};
    if (ndim == 2) return launch_col_w(w, ColVariant{0, 1}, st, nullptr, nullptr);
    int rc = launch_col_w(ColSpec{3, 1, {0, 0, 0}, 0}, ColVariant{0, 1}, st, nullptr, nullptr);
    if (!rc) rc = launch_col_w(w, ColVariant{0, 1}, st, nullptr, nullptr);
    if (!rc) rc = launch_col_w(ColSpec{4, 1, {0, 0, 0}, 0}, ColVariant{0, 1}, st, nullptr, nullptr);
    return rc;
  }
  // S1 <- L2 S1 (|k|^(y-1) with the transforms' 1/N): one column pass in 2D,
  // a y pass, the z pass and an inverse y pass in 3D
  int lap2(hipStream_t st) const {
    const ColSpec l{1, 1, {M_L2, 0, 0}, 1};
    if (ndim == 2) return launch_col_w(l, ColVariant{0, 1}, st, nullptr, nullptr);
    int rc = launch_col_w(ColSpec{3, 1, {0, 0, 0}, 1}, ColVariant{0, 1}, st, nullptr, nullptr);
    if (!rc) rc = launch_col_w(l, ColVariant{0, 1}, st, nullptr, nullptr);
    if (!rc) rc = launch_col_w(ColSpec{4, 1, {0, 0, 0}, 1}, ColVariant{0, 1}, st, nullptr, nullptr);
    return rc;
  }
  // kEosSteps fixed-point steps of the t = 0 equation of state, forward
  // (dir 0: the initial density) or transposed (dir 1: before the adjoint's
  // final assembly)
  int eos(int dir, hipStream_t st) const {
    int rc = row(dir == 0 ? R_EOS_FWD_IN : R_EOS_ADJ_IN, StepArg{nullptr, 0}, st);
    for (int k = 0; k < kEosSteps && !rc; ++k) {
      rc = lap2(st);
      if (!rc) rc = row(dir == 0 ? R_EOS_FWD : R_EOS_ADJ, StepArg{nullptr, k == kEosSteps - 1 ? 1 : 0}, st);
    }
    return rc;
  }
  // the forward's initial state, from S p0 when the plans smooth p0, the
  // density from the t = 0 equation of state when they ask for it
  int init(bool smooth, bool eos_init, hipStream_t st) const {
    int rc;
    if (!smooth) {
      rc = row(R_FWD_INIT, StepArg{nullptr, 0}, st);
    } else {
      rc = row(R_FILT_IN, StepArg{nullptr, 0}, st);
      if (!rc) rc = window(st);
      if (!rc) rc = row(R_FWD_INIT_F, StepArg{nullptr, 0}, st);
    }
    if (!rc && eos_init) rc = eos(0, st);
    return rc;
  }
  // the adjoint's final assembly (image from the transposed initial state)
  int adj_final(bool eos_init, hipStream_t st) const {
    int rc = eos_init ? eos(1, st) : PAT_OK;
    if (!rc) rc = row(R_ADJ_FINAL, StepArg{nullptr, 0}, st);
    return rc;
  }
  // image <- S image (the adjoint's last operator when the plans smooth p0)
  int smooth_out(bool smooth, hipStream_t st) const {
    if (!smooth) return PAT_OK;
    int rc = row(R_FILT_RE, StepArg{nullptr, 0}, st);
    if (!rc) rc = window(st);
    if (!rc) rc = row(R_FILT_OUT, StepArg{nullptr, 0}, st);
    return rc;
  }
  int reduce(int n0, int n1, hipStream_t st, int blocks) const {
    return launch_reduce(Launch{recs, red_tab, blocks, st}, n0, n1) == hipSuccess ? PAT_OK : PAT_EHIP;
  }
  // steps [s0, s1) of direction dir, eager
  int steps(int dir, int s0, int s1, hipStream_t st) const {
    PassOp ops[kMaxOps];
    const int nops = step_ops(dir, ndim, lossy, ops);
    int rc = PAT_OK;
    for (int s = s0; s < s1 && !rc; ++s)
      for (int i = 0; i < nops && !rc; ++i) rc = op(dir, i, ops[i], StepArg{nullptr, s, span}, st, true);
    return rc;
  }
};

// Column tile widths of the eager (one-instance) path in 2D.  One grid has
// few columns, so tiles narrower than the default put more workgroups on the
// 256 CUs: forward + adjoint of one 512^2 instance 290 -> 257 ms with 8
// columns per workgroup, 256^2 114 -> 107 ms and 128^2 49 -> 48 ms with 4
// (same-box, results bitwise unchanged).  The 3D z passes keep the default
// (narrower tiles ran 7-14 % slower at 128^3).
struct EagerTiles {
  ColVariant t8[3 * kMaxOps], t4[3 * kMaxOps];
  EagerTiles() {
    for (auto& v : t8) v = ColVariant{8, 1};
    for (auto& v : t4) v = ColVariant{4, 1};
  }
};
const EagerTiles g_eager_tiles;

Runner eager_runner(const pat_plan* p) {
  Runner r{};
  r.ndim = p->desc.ndim;
  r.nx = p->hp.n[0];
  r.ny = p->hp.n[1];
  r.nz = p->hp.n[2];
  r.nt = p->desc.nt;
  r.lossy = p->lossy;
  r.recs = p->dp;
  r.row_tab = r.red_tab = nullptr;
  const int R = row_tile_rows(r.nx);
  r.row_n = (p->hp.nrows + R - 1) / R;
  r.red_n = 0;
  r.ncolw = 0;
  const bool tunable = r.ny == 128 || r.ny == 256 || r.ny == 512;
  r.vars = (r.ndim == 2 && tunable) ? (r.ny == 512 ? g_eager_tiles.t8 : g_eager_tiles.t4) : nullptr;
  r.points = (double)p->npoints;
  return r;
}

int set_io(const pat_plan* p, const float* in, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_set_io, dim3(1), dim3(1), 0, st, p->dp, in, out);
  return hipGetLastError() == hipSuccess ? PAT_OK : PAT_EHIP;
}

int reduce_blocks(long nsamples, long ns) { return (int)((nsamples * ns + 255) / 256); }

bool smooths_p0(const pat_plan* p) { return (p->desc.flags & PAT_SMOOTH_P0) != 0; }
// the density starts from the t = 0 equation of state (lossy plans with
// PAT_EOS_INIT and more than one time sample)
bool eos_init(const pat_plan* p) { return (p->desc.flags & PAT_EOS_INIT) && p->lossy && p->desc.nt > 1; }
// the initial and final passes a plan needs (plans that share launches must agree)
int ends_of(const pat_plan* p) { return (smooths_p0(p) ? 1 : 0) | (eos_init(p) ? 2 : 0); }

}  // namespace
}  // namespace pat

using namespace pat;

// ===================================================================== eager entry points
extern "C" int pat_forward(pat_plan* p, const float* p0, float* data, void* stream) {
  if (!p || !p0 || !data) return PAT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const Runner R = eager_runner(p);
  int rc = set_io(p, p0, data, st);
  if (!rc) rc = R.init(smooths_p0(p), eos_init(p), st);
  if (!rc) rc = R.steps(0, 0, p->desc.nt - 1, st);
  if (!rc) rc = R.reduce(0, 0, st, reduce_blocks(p->desc.nt, p->desc.n_sensors));
  return rc;
}

extern "C" int pat_adjoint(pat_plan* p, const float* data, float* img, void* stream) {
  if (!p || !data || !img) return PAT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const Runner R = eager_runner(p);
  int rc = set_io(p, data, img, st);
  if (rc) return rc;
  if (p->desc.nt == 1) {
    rc = R.row(R_ADJ_SCATTER_ONLY, StepArg{nullptr, 0}, st);
  } else {
    rc = scatter_sums(p->dp, 1, (long)p->desc.nt * p->hp.ngroups, st);
    if (!rc) rc = R.steps(1, 0, p->desc.nt - 1, st);
    if (!rc) rc = R.adj_final(eos_init(p), st);
  }
  if (!rc) rc = R.smooth_out(smooths_p0(p), st);
  return rc;
}

extern "C" int pat_adjoint_atd(pat_plan* p, const float* data, float* img, void* stream) {
  if (!p || !data || !img) return PAT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (p->desc.nt == 1)  // no time step: the trapezoid over an empty interval
    return hipMemsetAsync(img, 0, sizeof(float) * p->npoints, st) == hipSuccess ? PAT_OK : PAT_EHIP;
  const Runner R = eager_runner(p);
  int rc = set_io(p, data, img, st);
  if (rc) return rc;
  // p* = 0 at the start: its x-spectrum, read by the first gradient pass
  if (hipMemsetAsync(p->hp.S[0], 0, sizeof(float) * p->npoints, st) != hipSuccess) return PAT_EHIP;
  rc = R.steps(2, 0, p->desc.nt - 1, st);
  if (!rc) rc = R.row(R_ATD_FINAL, StepArg{nullptr, 0}, st);
  if (!rc) rc = R.smooth_out(smooths_p0(p), st);
  return rc;
}

extern "C" int pat_forward_range(pat_plan* p, const float* p0, float* data, int32_t n_begin, int32_t n_end,
                                 void* state_io, void* stream) {
  if (!p || !data || !state_io) return PAT_EINVAL;
  const int nt = p->desc.nt;
  if (n_begin < 0 || n_end <= n_begin || n_end > nt) return PAT_EINVAL;
  if (n_begin == 0 && !p0) return PAT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const Runner R = eager_runner(p);
  void* state = (void*)p->hp.u[0];
  int rc = set_io(p, p0, data, st);
  if (rc) return rc;
  int s0;
  if (n_begin == 0) {
    rc = R.init(smooths_p0(p), eos_init(p), st);
    s0 = 0;
  } else {
    if (hipMemcpyAsync(state, state_io, p->state_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) return PAT_EHIP;
    s0 = n_begin - 1;
  }
  // step n records sample n + 1: samples n_begin..n_end-1 need steps s0..n_end-2
  if (!rc) rc = R.steps(0, s0, n_end - 1, st);
  if (!rc) rc = R.reduce(n_begin, n_end, st, reduce_blocks(n_end - n_begin, p->desc.n_sensors));
  if (!rc && hipMemcpyAsync(state_io, state, p->state_bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
    rc = PAT_EHIP;
  return rc;
}

// ===================================================================== timing diagnostics
extern "C" int pat_timing_begin(int32_t direction, int32_t pass_index, int32_t nx) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (direction < 0 || direction > 1 || pass_index < 0 || pass_index >= kMaxOps || nx < 0) return PAT_EINVAL;
  g_timing.dir = direction;
  g_timing.index = pass_index;
  g_timing.nx = nx;
  g_timing.used = 0;
  g_timing.bytes = 0;
  g_timing.launches = 0;
  g_timing_on = true;
  return PAT_OK;
}

extern "C" int pat_timing_end(double* total_ms, int64_t* launches, double* alg_bytes) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!total_ms || !launches || !alg_bytes) return PAT_EINVAL;
  g_timing_on = false;
  double ms = 0;
  for (size_t i = 0; i + 1 < g_timing.used; i += 2) {
    if (hipEventSynchronize(g_timing.ev[i + 1]) != hipSuccess) return PAT_EHIP;
    float t = 0;
    if (hipEventElapsedTime(&t, g_timing.ev[i], g_timing.ev[i + 1]) != hipSuccess) return PAT_EHIP;
    ms += t;
  }
  *total_ms = ms;
  *launches = g_timing.launches;
  *alg_bytes = g_timing.bytes;
  g_timing.used = 0;
  return PAT_OK;
}

// ===================================================================== batched executor
namespace {

struct BatchClass {
  int ndim, nx, ny, nz, nt, lossy, ns_max;
  bool smooth_p0 = false;  // the instances smooth p0 (all or none of a class)
  bool eos = false;        // ... start the density from the t = 0 equation of state
  // fused group: instances of several 2D sizes in every launch (nx, ny the
  // largest, nt - 1 = span = the most steps of any instance)
  int fused = 0;
  std::vector<std::pair<int, int>> shapes;  // fused: the (nx, ny) it holds
  std::vector<double> inst_points;          // per instance: grid points and nt
  std::vector<int> inst_nt;
  std::vector<pat_plan*> plans;
  std::vector<int> index;  // position of each plan in the caller's list
  DevPlan* recs = nullptr;
  int2* row_tab = nullptr;
  int2* red_tab = nullptr;
  int row_n = 0, red_n = 0;
  int2* col_tabs[kColW] = {};
  int col_ns[kColW] = {}, col_ws[kColW] = {}, col_bpi[kColW] = {}, ncolw = 0;
  ColVariant vars[2 * kMaxOps];
  // autotuner record: candidate variants and their mean durations per pass
  struct Tuned {
    int dir, idx, ncand;
    ColVariant cand[kMaxColVar];
    float us[kMaxColVar];
  };
  BatchClass() {
    for (auto& v : vars) v = ColVariant{0, 1};
  }
  std::vector<Tuned> tuned;
  int32_t* ctr = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  Runner runner() const {
    Runner r{};
    r.ndim = ndim;
    r.nx = nx;
    r.ny = ny;
    r.nz = nz;
    r.nt = nt;
    r.lossy = lossy;
    r.fused = fused;
    r.span = fused ? nt - 1 : 0;
    r.inst_points = inst_points.data();
    r.inst_nt = inst_nt.data();
    r.ninst = (int)inst_nt.size();
    r.recs = recs;
    r.row_tab = row_tab;
    r.red_tab = red_tab;
    r.row_n = row_n;
    r.red_n = red_n;
    r.ncolw = ncolw;
    for (int j = 0; j < kColW; ++j) {
      r.col_tabs[j] = col_tabs[j];
      r.col_ns[j] = col_ns[j];
      r.col_ws[j] = col_ws[j];
      r.col_bpi[j] = col_bpi[j];
    }
    r.vars = vars;
    double pts = 0;
    for (auto* p : plans) pts += (double)p->npoints;
    r.points = pts;
    return r;
  }
};

}  // namespace

// Width policies of the autotuner's second (in-context) phase: how a pass's
// variant is chosen from its isolated timings.  The first is the incumbent:
// 8 columns, one field per block (the fused passes' untuned default).
enum TunePolicy : int { TP_EXACT8_F1 = 0, TP_FASTEST, TP_MAX8, TP_MAX4, TP_EXACT8, TP_COUNT };
const char* const kPolicyName[TP_COUNT] = {"width=8,fpb=1", "fastest", "width<=8", "width<=4", "width=8"};
// a policy replaces the incumbent only when it runs this much faster
constexpr float kPolicyMargin = 0.005f;
constexpr int kPolicyRounds = 3;

struct pat_batch {
  int chunk = 64;
  std::vector<BatchClass> cls;
  int policy = -1;                 // width policy chosen in context (-1: none)
  float policy_us[TP_COUNT] = {};  // its timing of each policy (0: not timed)
  void* arena = nullptr;
  std::vector<hipStream_t> lanes;  // streams the classes run on (the device's pooled lanes)
  hipStream_t cap = nullptr;  // capture-only stream
  hipEvent_t fork = nullptr;
  hipEvent_t lead = nullptr;  // the first group's first pass (staggered start)
  bool stagger = true;
  int nb = 0;
};

namespace {

// Lane streams, shared by every batch on a device and kept until the process
// ends.  HIP maps each new stream onto one of a few hardware queues (four by
// default); once all of them exist it picks the least used one, the newest
// on a tie, so the second of two streams created one after the other can
// share the first one's queue -- and two groups whose streams share a queue
// run one after the other (measured on the 48-instance batch: a second batch
// created after a one-lane batch ran its two groups in 956 instead of
// 735 ms).  The pool creates its first two lanes together, at the first
// batch on the device, and every later batch reuses them instead of creating
// streams of its own.
std::mutex g_lane_mu;
std::map<int, std::vector<hipStream_t>> g_lanes;

int pooled_lanes(int n, std::vector<hipStream_t>& out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PAT_EHIP;
  std::lock_guard<std::mutex> lk(g_lane_mu);
  auto& pool = g_lanes[dev];
  while ((int)pool.size() < std::max(n, 2)) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return PAT_EHIP;
    pool.push_back(s);
  }
  out.assign(pool.begin(), pool.begin() + n);
  return PAT_OK;
}

void destroy_batch(pat_batch* b) {
  if (!b) return;
  hipDeviceSynchronize();
  for (auto& c : b->cls) {
    for (auto& g : c.graph)
      if (g) hipGraphExecDestroy(g);
    if (c.done) hipEventDestroy(c.done);
  }
  if (b->cap) hipStreamDestroy(b->cap);
  if (b->fork) hipEventDestroy(b->fork);
  if (b->lead) hipEventDestroy(b->lead);
  if (b->arena) hipFree(b->arena);
  delete b;
}

// capture `chunk` steps of direction dir (step index = *ctr + k) + counter advance
int capture(pat_batch* b, BatchClass& c, int dir) {
  const Runner R = c.runner();
  PassOp ops[kMaxOps];
  const int nops = step_ops(dir, c.ndim, c.lossy, ops);
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return PAT_EHIP;
  int rc = PAT_OK;
  for (int k = 0; k < b->chunk && !rc; ++k)
    for (int i = 0; i < nops && !rc; ++i) rc = R.op(dir, i, ops[i], StepArg{c.ctr, k, R.span}, b->cap, false);
  if (!rc) {
    hipLaunchKernelGGL(k_add_ctr, dim3(1), dim3(1), 0, b->cap, c.ctr, b->chunk);
    if (hipGetLastError() != hipSuccess) rc = PAT_EHIP;
  }
  if (hipStreamEndCapture(b->cap, &g) != hipSuccess) rc = PAT_EHIP;
  if (!rc && hipGraphInstantiate(&c.graph[dir], g, nullptr, nullptr, 0) != hipSuccess) rc = PAT_EHIP;
  if (g) hipGraphDestroy(g);
  return rc;
}

// steps [0, nsteps) of direction dir on the class stream: `full` graph chunks
// with the nsteps mod chunk remaining steps run eagerly and spread evenly
// between the chunks (the eager launches are the ones diagnostics can time,
// so they sample the whole run); the device counter skips the eager steps.
// With `lead`, step 0 runs first, eagerly, and `lead` is recorded after its
// first pass.
int run_steps(pat_batch* b, BatchClass& c, int dir, int nsteps, hipEvent_t lead = nullptr) {
  const Runner R = c.runner();
  int rc = PAT_OK;
  int s0 = 0;
  if (lead && nsteps > 0) {
    PassOp ops[kMaxOps];
    const int nops = step_ops(dir, c.ndim, c.lossy, ops);
    for (int i = 0; i < nops && !rc; ++i) {
      rc = R.op(dir, i, ops[i], StepArg{nullptr, 0, R.span}, c.st, true);
      if (!rc && i == 0 && hipEventRecord(lead, c.st) != hipSuccess) rc = PAT_EHIP;
    }
    if (rc) return rc;
    s0 = 1;
  }
  const int full = b->chunk > 1 ? (nsteps - s0) / b->chunk : 0;
  const int rem = nsteps - s0 - full * b->chunk;
  if (full == 0) return R.steps(dir, s0, nsteps, c.st);
  if (!c.graph[dir] && (rc = capture(b, c, dir))) return rc;
  hipLaunchKernelGGL(k_set_ctr, dim3(1), dim3(1), 0, c.st, c.ctr, s0);
  if (hipGetLastError() != hipSuccess) return PAT_EHIP;
  int n = s0, done_eager = 0;
  for (int g = 0; g < full && !rc; ++g) {
    const int want = (int)((long)(g + 1) * rem / full);  // eager steps due by chunk g
    for (; done_eager < want && !rc; ++done_eager, ++n) {
      rc = R.steps(dir, n, n + 1, c.st);
      if (!rc) {
        hipLaunchKernelGGL(k_add_ctr, dim3(1), dim3(1), 0, c.st, c.ctr, 1);
        if (hipGetLastError() != hipSuccess) rc = PAT_EHIP;
      }
    }
    if (!rc && hipGraphLaunch(c.graph[dir], c.st) != hipSuccess) rc = PAT_EHIP;
    n += b->chunk;
  }
  return rc;
}

int set_io_class(BatchClass& c, const float* const* in, float* const* out) {
  for (size_t i0 = 0; i0 < c.plans.size(); i0 += kIoMax) {
    IoArgs a{};
    const int n = (int)std::min<size_t>(kIoMax, c.plans.size() - i0);
    for (int i = 0; i < n; ++i) {
      const int k = c.index[i0 + i];
      if (!in[k] || !out[k]) return PAT_EINVAL;
      a.in[i] = in[k];
      a.out[i] = out[k];
    }
    hipLaunchKernelGGL(k_set_io_many, dim3(1), dim3(kIoMax), 0, c.st, c.recs + i0, n, a);
    if (hipGetLastError() != hipSuccess) return PAT_EHIP;
  }
  return PAT_OK;
}

// Staggered start: with several groups, the groups at odd positions begin
// their time loop once the first group has run one pass, so that the
// streams tend to pair one group's column pass (arithmetic-bound) with
// another's row pass (memory-bound) rather than two of a kind.
int batch_run(pat_batch* b, int dir, const float* const* in, float* const* out, hipStream_t st) {
  if (!b || !in || !out) return PAT_EINVAL;
  if (hipEventRecord(b->fork, st) != hipSuccess) return PAT_EHIP;
  const bool stagger = b->stagger && b->cls.size() > 1;
  int rc = PAT_OK;
  for (size_t k = 0; k < b->cls.size(); ++k) {
    BatchClass& c = b->cls[k];
    if (hipStreamWaitEvent(c.st, b->fork, 0) != hipSuccess) return PAT_EHIP;
    rc = set_io_class(c, in, out);
    if (rc) return rc;
    const Runner R = c.runner();
    hipEvent_t lead = (stagger && k == 0) ? b->lead : nullptr;
    const bool follow = stagger && (k & 1);
    if (dir == 0) {
      rc = R.init(c.smooth_p0, c.eos, c.st);
      if (!rc && follow && hipStreamWaitEvent(c.st, b->lead, 0) != hipSuccess) rc = PAT_EHIP;
      if (!rc) rc = run_steps(b, c, 0, c.nt - 1, lead);
      if (!rc) rc = R.reduce(0, 0, c.st, c.red_n);
    } else if (c.nt == 1) {
      rc = R.row(R_ADJ_SCATTER_ONLY, StepArg{nullptr, 0}, c.st);
      if (!rc) rc = R.smooth_out(c.smooth_p0, c.st);
    } else {
      long most = 0;
      for (auto* pl : c.plans) most = std::max(most, (long)pl->desc.nt * pl->hp.ngroups);
      rc = scatter_sums(c.recs, (int)c.plans.size(), most, c.st);
      if (!rc && follow && hipStreamWaitEvent(c.st, b->lead, 0) != hipSuccess) rc = PAT_EHIP;
      if (!rc) rc = run_steps(b, c, 1, c.nt - 1, lead);
      if (!rc) rc = R.adj_final(c.eos, c.st);
      if (!rc) rc = R.smooth_out(c.smooth_p0, c.st);
    }
    if (rc) return rc;
    if (hipEventRecord(c.done, c.st) != hipSuccess) return PAT_EHIP;
  }
  for (auto& c : b->cls)
    if (hipStreamWaitEvent(st, c.done, 0) != hipSuccess) return PAT_EHIP;
  return PAT_OK;
}

}  // namespace

extern "C" int pat_batch_create(pat_batch** out, pat_plan* const* plans, int32_t nb, int32_t chunk) {
  return pat_batch_create_ex(out, plans, nb, chunk, 0, 0, 0);
}

extern "C" int pat_batch_create_ex(pat_batch** out, pat_plan* const* plans, int32_t nb, int32_t chunk, int32_t parts,
                                   int32_t lanes, uint32_t flags) {
  if (!out) return PAT_EINVAL;
  *out = nullptr;
  if (!plans || nb < 1 || chunk < 0 || parts < 0 || lanes < 0 ||
      (flags & ~(uint32_t)(PAT_BATCH_NO_FUSE | PAT_BATCH_NO_STAGGER)))
    return PAT_EINVAL;
  for (int i = 0; i < nb; ++i)
    if (!plans[i] || plans[i]->desc.ndim != plans[0]->desc.ndim) return PAT_EINVAL;
  auto* b = new (std::nothrow) pat_batch();
  if (!b) return PAT_ENOMEM;
  b->chunk = chunk == 0 ? 64 : chunk;
  b->nb = nb;
  b->stagger = !(flags & PAT_BATCH_NO_STAGGER);
  // group by (shape, nt, lossy), then split every group into `parts` equal
  // parts (default 2).  Each part runs on its own stream, so that the passes
  // of different parts -- memory-bound rows of one, arithmetic-bound columns
  // of another -- overlap on the GPU (measured on the 48-instance 2D batch:
  // two parts per size class beat one by about 8%; finer splits lose, their
  // launches no longer fill the GPU).
  const int split = parts ? parts : 2;
  std::vector<std::vector<int>> groups;
  std::vector<int> group_fused;
  {
    std::map<std::tuple<int, int, int, int, int, int>, int> key2grp;
    std::vector<std::vector<int>> shape_groups;
    for (int i = 0; i < nb; ++i) {
      const pat_plan* p = plans[i];
      const auto key = std::make_tuple(p->hp.n[0], p->hp.n[1], p->hp.n[2], p->desc.nt, p->lossy, ends_of(p));
      auto it = key2grp.find(key);
      if (it == key2grp.end()) {
        it = key2grp.emplace(key, (int)shape_groups.size()).first;
        shape_groups.emplace_back();
      }
      shape_groups[it->second].push_back(i);
    }
    // Fusion: 2D size classes whose axes are 128, 256 or 512 points (and
    // the same physics) share their launches.  Part k of every such class
    // forms fused group k, its instances ordered largest grid first.
    auto fusable = [&](const std::vector<int>& g) {
      const pat_plan* p = plans[g[0]];
      return !(flags & PAT_BATCH_NO_FUSE) && p->desc.ndim == 2 && fused_size(p->hp.n[0]) &&
             fused_size(p->hp.n[1]) && p->desc.nt >= 2;
    };
    auto area = [&](const std::vector<int>& g) { return (long)plans[g[0]]->hp.n[0] * plans[g[0]]->hp.n[1]; };
    // the classes of one fused group share the pass sequence: the same
    // physics (lossy or not) and the same initial and final passes
    for (int phys = 0; phys < 8; ++phys) {
      const int lossy = phys & 1;
      const int ends = phys >> 1;
      std::vector<int> fs;
      for (size_t k = 0; k < shape_groups.size(); ++k) {
        const pat_plan* p = plans[shape_groups[k][0]];
        if (p->lossy == lossy && ends_of(p) == ends && fusable(shape_groups[k])) fs.push_back((int)k);
      }
      if (fs.size() < 2) continue;
      std::stable_sort(fs.begin(), fs.end(), [&](int x, int y) {
        const long ax = area(shape_groups[x]), ay = area(shape_groups[y]);
        return ax != ay ? ax > ay : plans[shape_groups[x][0]]->hp.n[0] > plans[shape_groups[y][0]]->hp.n[0];
      });
      for (int k = 0; k < split; ++k) {
        std::vector<int> g;
        for (int s : fs) {
          const std::vector<int>& sg = shape_groups[s];
          const size_t np = std::min(sg.size(), (size_t)split);
          if ((size_t)k < np) g.insert(g.end(), sg.begin() + sg.size() * k / np, sg.begin() + sg.size() * (k + 1) / np);
        }
        if (!g.empty()) {
          groups.push_back(g);
          group_fused.push_back(1);
        }
      }
      for (int s : fs) shape_groups[s].clear();
    }
    for (auto& g : shape_groups) {
      if (g.empty()) continue;
      const size_t parts = std::min(g.size(), (size_t)split);
      for (size_t k = 0; k < parts; ++k) {
        groups.emplace_back(g.begin() + g.size() * k / parts, g.begin() + g.size() * (k + 1) / parts);
        group_fused.push_back(0);
      }
    }
  }
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const auto& g = groups[gi];
    const pat_plan* p0 = plans[g[0]];
    BatchClass c{};
    c.ndim = p0->desc.ndim;
    c.nx = p0->hp.n[0];
    c.ny = p0->hp.n[1];
    c.nz = p0->hp.n[2];
    c.nt = p0->desc.nt;
    c.lossy = p0->lossy;
    c.smooth_p0 = smooths_p0(p0);
    c.eos = eos_init(p0);
    c.fused = group_fused[gi];
    c.ns_max = 0;
    for (int i : g) {
      c.plans.push_back(plans[i]);
      c.index.push_back(i);
      c.ns_max = std::max(c.ns_max, plans[i]->desc.n_sensors);
      c.nt = std::max(c.nt, plans[i]->desc.nt);
      c.inst_points.push_back((double)plans[i]->npoints);
      c.inst_nt.push_back(plans[i]->desc.nt);
      const std::pair<int, int> sh(plans[i]->hp.n[0], plans[i]->hp.n[1]);
      if (c.fused && std::find(c.shapes.begin(), c.shapes.end(), sh) == c.shapes.end()) c.shapes.push_back(sh);
    }
    b->cls.push_back(std::move(c));
  }
  // device layout: per class records, tables, counter
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    const size_t at = off;
    off += bytes;
    return at;
  };
  struct Lay {
    size_t rec, row, col[kColW], red, ctr;
  };
  std::vector<Lay> lay;
  std::vector<std::vector<int2>> rt(b->cls.size()), dt(b->cls.size());
  std::vector<std::vector<std::vector<int2>>> ct(b->cls.size(), std::vector<std::vector<int2>>(kColW));
  for (size_t k = 0; k < b->cls.size(); ++k) {
    BatchClass& c = b->cls[k];
    const int R = row_tile_rows(c.nx);
    const int rows_per = (c.ny * c.nz + R - 1) / R;
    // every tile width some column pass of the class can run with; a y-axis
    // and a z-axis pass of one width tile the same number of columns only
    // when ny == nz, so the table is per (width, axis)
    std::vector<std::pair<int, int>> widths;  // (width, blocks per instance)
    for (int dir = 0; dir < 2 && !c.fused; ++dir) {
      PassOp ops[kMaxOps];
      const int nops = step_ops(dir, c.ndim, c.lossy, ops);
      for (int i = 0; i < nops; ++i) {
        if (!ops[i].is_col) continue;
        ColVariant cand[kMaxColVar];
        const int nc = col_variants(ops[i].col, c.ndim, c.ny, c.nz, cand);
        for (int j = 0; j < nc; ++j) {
          ColSpec s = ops[i].col;
          s.tile = cand[j].tile;
          s.fpb = cand[j].fpb;
          const std::pair<int, int> wb(cand[j].tile, col_blocks(s, c.ndim, c.nx, c.ny, c.nz));
          if (std::find(widths.begin(), widths.end(), wb) == widths.end()) widths.push_back(wb);
        }
      }
    }
    if ((int)widths.size() > kColW) {
      destroy_batch(b);
      return PAT_EINVAL;
    }
    // XCD-aware order: workgroups are dispatched round-robin over the eight
    // XCDs (each with its own L2), so entry e runs on XCD e mod 8.  Entries
    // interleave the instances of each group of eight, so that every pass of
    // an instance runs on the same XCD and re-reads what the previous pass
    // of that instance left in that XCD's L2.
    const int ninst = (int)c.plans.size();
    // runs of up to eight instances of one grid shape (a fused group lists
    // its instances by shape, largest grid first); tiles_of(instance) work
    // items each.  The runs enter the table in reverse, smallest grid first:
    // blocks are dispatched in table order, so the small instances' blocks
    // start first and finish under the large grid's blocks instead of
    // forming the tail of the launch.
    auto interleave = [&](std::vector<int2>& tab, auto tiles_of) {
      std::vector<std::pair<int, int>> runs;  // (first instance, count)
      for (int g0 = 0; g0 < ninst;) {
        int gn = 1;
        while (g0 + gn < ninst && gn < kXcds && c.plans[g0 + gn]->hp.n[0] == c.plans[g0]->hp.n[0] &&
               c.plans[g0 + gn]->hp.n[1] == c.plans[g0]->hp.n[1])
          ++gn;
        runs.emplace_back(g0, gn);
        g0 += gn;
      }
      for (auto r = runs.rbegin(); r != runs.rend(); ++r) {
        const int g0 = r->first, gn = r->second;
        const int tiles = tiles_of(c.plans[g0]);
        for (int t = 0; t < tiles; ++t)
          for (int l = 0; l < gn; ++l) tab.push_back(make_int2(g0 + l, t));
      }
    };
    if (c.fused) {
      interleave(rt[k], [](const pat_plan* p) {
        const int R2 = fused_row_rows(p->hp.n[0]);
        return (p->hp.n[1] + R2 - 1) / R2;
      });
      const int fw[2] = {8, 4};
      c.ncolw = 2;
      for (int j = 0; j < 2; ++j) {
        interleave(ct[k][j], [&](const pat_plan* p) {
          const int w = fused_col_tile(p->hp.n[1], fw[j]);
          return (p->hp.n[0] / 2 + w - 1) / w;
        });
        c.col_ws[j] = fw[j];
        c.col_bpi[j] = 0;
        c.col_ns[j] = (int)ct[k][j].size();
      }
    } else {
      interleave(rt[k], [&](const pat_plan*) { return rows_per; });
      c.ncolw = (int)widths.size();
      for (int j = 0; j < c.ncolw; ++j) {
        const int bpi = widths[j].second;
        interleave(ct[k][j], [&](const pat_plan*) { return bpi; });
        c.col_ws[j] = widths[j].first;
        c.col_bpi[j] = widths[j].second;
        c.col_ns[j] = (int)ct[k][j].size();
      }
    }
    for (int i = 0; i < ninst; ++i) {
      const int rb = reduce_blocks(c.plans[i]->desc.nt, c.plans[i]->desc.n_sensors);
      for (int t = 0; t < rb; ++t) dt[k].push_back(make_int2(i, t));
    }
    c.row_n = (int)rt[k].size();
    c.red_n = (int)dt[k].size();
    Lay l;
    l.rec = take(sizeof(DevPlan) * c.plans.size());
    l.row = take(sizeof(int2) * rt[k].size());
    for (int j = 0; j < c.ncolw; ++j) l.col[j] = take(sizeof(int2) * ct[k][j].size());
    l.red = take(sizeof(int2) * dt[k].size());
    l.ctr = take(sizeof(int32_t));
    lay.push_back(l);
  }
  int rc = PAT_OK;
  if (hipMalloc(&b->arena, off) != hipSuccess) {
    delete b;
    return PAT_ENOMEM;
  }
  char* A = (char*)b->arena;
  for (size_t k = 0; k < b->cls.size() && !rc; ++k) {
    BatchClass& c = b->cls[k];
    c.recs = (DevPlan*)(A + lay[k].rec);
    c.row_tab = (int2*)(A + lay[k].row);
    c.red_tab = (int2*)(A + lay[k].red);
    c.ctr = (int32_t*)(A + lay[k].ctr);
    std::vector<DevPlan> recs;
    for (auto* p : c.plans) recs.push_back(p->hp);
    if (hipMemcpy(c.recs, recs.data(), sizeof(DevPlan) * recs.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.row_tab, rt[k].data(), sizeof(int2) * rt[k].size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.red_tab, dt[k].data(), sizeof(int2) * dt[k].size(), hipMemcpyHostToDevice) != hipSuccess)
      rc = PAT_EHIP;
    for (int j = 0; j < c.ncolw && !rc; ++j) {
      c.col_tabs[j] = (int2*)(A + lay[k].col[j]);
      if (hipMemcpy(c.col_tabs[j], ct[k][j].data(), sizeof(int2) * ct[k][j].size(), hipMemcpyHostToDevice) !=
          hipSuccess)
        rc = PAT_EHIP;
    }
    if (!rc && hipEventCreateWithFlags(&c.done, hipEventDisableTiming) != hipSuccess) rc = PAT_EHIP;
  }
  // Streams: by default one per group.  With fewer streams than groups, the
  // groups go heaviest first (grid points x steps) to the least-loaded
  // stream, so that small classes share streams with each other rather than
  // queue behind the largest.
  const int nlanes = lanes ? std::min((int)b->cls.size(), (int)lanes) : (int)b->cls.size();
  if (!rc) rc = pooled_lanes(nlanes, b->lanes);
  if (!rc) {
    std::vector<double> work(b->cls.size());
    std::vector<int> order(b->cls.size());
    for (size_t k = 0; k < b->cls.size(); ++k) {
      double pts = 0;
      for (auto* p : b->cls[k].plans) pts += (double)p->npoints;
      work[k] = pts * std::max(1, b->cls[k].nt - 1);
      order[k] = (int)k;
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    std::vector<double> load(b->lanes.size(), 0.0);
    for (int k : order) {
      const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      b->cls[k].st = b->lanes[j];
      load[j] += work[k];
    }
  }
  if (!rc && (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
              hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&b->lead, hipEventDisableTiming) != hipSuccess))
    rc = PAT_EHIP;
  if (rc) {
    destroy_batch(b);
    return rc;
  }
  *out = b;
  return PAT_OK;
}

extern "C" void pat_batch_destroy(pat_batch* b) { destroy_batch(b); }

extern "C" int pat_batch_forward(pat_batch* b, const float* const* p0, float* const* data, void* stream) {
  return batch_run(b, 0, p0, data, (hipStream_t)stream);
}

extern "C" int pat_batch_adjoint(pat_batch* b, const float* const* data, float* const* img, void* stream) {
  return batch_run(b, 1, data, img, (hipStream_t)stream);
}

// ===================================================================== one-call batched entry points
// One batch (default settings) per distinct list of plans, made on the first
// call and kept until one of its plans is destroyed.  The map lives on the
// heap and is never torn down: at process exit the HIP runtime may already
// be gone, so nothing is freed from a static destructor.
namespace {
std::mutex g_bmu;
std::map<std::vector<pat_plan*>, pat_batch*>& batch_cache() {
  static auto* m = new std::map<std::vector<pat_plan*>, pat_batch*>();
  return *m;
}

int cached_batch(pat_plan* const* plans, int nb, pat_batch** out) {
  if (!plans || nb < 1 || !out) return PAT_EINVAL;
  std::vector<pat_plan*> key(plans, plans + nb);
  for (pat_plan* p : key)
    if (!p) return PAT_EINVAL;
  std::lock_guard<std::mutex> lk(g_bmu);
  auto& m = batch_cache();
  auto it = m.find(key);
  if (it == m.end()) {
    pat_batch* b = nullptr;
    const int rc = pat_batch_create_ex(&b, plans, nb, 0, 0, 0, 0);
    if (rc) return rc;
    it = m.emplace(std::move(key), b).first;
  }
  *out = it->second;
  return PAT_OK;
}
}  // namespace

namespace pat {
void batch_cache_forget(const pat_plan* p) {
  std::lock_guard<std::mutex> lk(g_bmu);
  auto& m = batch_cache();
  for (auto it = m.begin(); it != m.end();) {
    if (std::find(it->first.begin(), it->first.end(), p) != it->first.end()) {
      destroy_batch(it->second);
      it = m.erase(it);
    } else {
      ++it;
    }
  }
}
}  // namespace pat

extern "C" int pat_forward_batched(pat_plan* const* plans, int32_t nb, const float* const* p0, float* const* data,
                                   void* stream) {
  if (!p0 || !data) return PAT_EINVAL;
  pat_batch* b = nullptr;
  const int rc = cached_batch(plans, nb, &b);
  return rc ? rc : batch_run(b, 0, p0, data, (hipStream_t)stream);
}

extern "C" int pat_adjoint_batched(pat_plan* const* plans, int32_t nb, const float* const* data, float* const* img,
                                   void* stream) {
  if (!data || !img) return PAT_EINVAL;
  pat_batch* b = nullptr;
  const int rc = cached_batch(plans, nb, &b);
  return rc ? rc : batch_run(b, 1, data, img, (hipStream_t)stream);
}

// ===================================================================== column tile autotuner
// For every column pass of every class that has more than one instantiated
// tile width, each candidate is launched `reps` times over the class's own
// buffers (after one untimed launch) and timed with a pair of events; the
// fastest mean is kept.  The passes run on whatever the state buffers hold:
// their duration does not depend on the values, and every forward and
// adjoint run rewrites the state from its input before reading it.  Captured
// graphs are dropped so that the next run captures the chosen widths.
namespace {

// the candidate a width policy takes for one tuned pass
int pick_variant(const BatchClass::Tuned& t, int policy) {
  int best = -1, fastest = 0;
  for (int j = 0; j < t.ncand; ++j) {
    if (t.us[j] < t.us[fastest]) fastest = j;
    const int w = t.cand[j].tile;
    const bool ok = policy == TP_FASTEST || (policy == TP_MAX8 && w <= 8) || (policy == TP_MAX4 && w <= 4) ||
                    (policy == TP_EXACT8 && w == 8) || (policy == TP_EXACT8_F1 && w == 8 && t.cand[j].fpb == 1);
    if (ok && (best < 0 || t.us[j] < t.us[best])) best = j;
  }
  return best < 0 ? fastest : best;
}

// set the variants of every tuned pass (in class and record order) and drop
// the captured graphs
void apply_choice(pat_batch* b, const std::vector<ColVariant>& v) {
  size_t k = 0;
  for (auto& c : b->cls) {
    for (const auto& t : c.tuned) c.vars[t.dir * kMaxOps + t.idx] = v[k++];
    for (auto& g : c.graph)
      if (g) {
        hipGraphExecDestroy(g);
        g = nullptr;
      }
  }
}

// Forward steps of every group at once, the longest time axis running
// `steps` steps and every other group a proportional number, from one fork
// on `st` to the join of all groups.  The steps only touch plan-owned state
// (the input and output arrays are read and written outside the steps).
int time_concurrent(pat_batch* b, int steps, hipStream_t st, hipEvent_t e0, hipEvent_t e1, float* ms) {
  long ntmax = 1;
  for (const auto& c : b->cls) ntmax = std::max(ntmax, (long)c.nt - 1);
  if (hipEventRecord(e0, st) != hipSuccess) return PAT_EHIP;
  for (auto& c : b->cls) {
    if (hipStreamWaitEvent(c.st, e0, 0) != hipSuccess) return PAT_EHIP;
    const long n = std::min<long>(c.nt - 1, ((long)steps * (c.nt - 1) + ntmax - 1) / ntmax);
    if (n > 0) {
      const int rc = run_steps(b, c, 0, (int)n);
      if (rc) return rc;
    }
    if (hipEventRecord(c.done, c.st) != hipSuccess) return PAT_EHIP;
  }
  for (auto& c : b->cls)
    if (hipStreamWaitEvent(st, c.done, 0) != hipSuccess) return PAT_EHIP;
  if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(ms, e0, e1) != hipSuccess)
    return PAT_EHIP;
  return PAT_OK;
}

}  // namespace

extern "C" int pat_batch_autotune(pat_batch* b, int32_t reps, void* stream) {
  if (!b || reps < 1) return PAT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (hipStreamSynchronize(st) != hipSuccess) return PAT_EHIP;
  for (auto& c : b->cls)
    if (hipStreamSynchronize(c.st) != hipSuccess) return PAT_EHIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return PAT_EHIP;
  }
  int rc = PAT_OK;
  for (auto& c : b->cls) {
    c.tuned.clear();
    for (int dir = 0; dir < 2 && !rc; ++dir) {
      PassOp ops[kMaxOps];
      const int nops = step_ops(dir, c.ndim, c.lossy, ops);
      for (int i = 0; i < nops && !rc; ++i) {
        if (!ops[i].is_col) continue;
        BatchClass::Tuned t{};
        t.dir = dir;
        t.idx = i;
        t.ncand = c.fused ? col_variants_fused(ops[i].col, t.cand) : col_variants(ops[i].col, c.ndim, c.ny, c.nz, t.cand);
        if (t.ncand < 2) continue;
        const Runner R = c.runner();
        int best = 0;
        for (int j = 0; j < t.ncand && !rc; ++j) {
          rc = R.launch_col_w(ops[i].col, t.cand[j], st, nullptr, nullptr);
          if (!rc && hipEventRecord(e0, st) != hipSuccess) rc = PAT_EHIP;
          for (int r = 0; r < reps && !rc; ++r) rc = R.launch_col_w(ops[i].col, t.cand[j], st, nullptr, nullptr);
          if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = PAT_EHIP;
          float ms = 0;
          if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = PAT_EHIP;
          t.us[j] = 1e3f * ms / (float)reps;
          if (t.us[j] < t.us[best]) best = j;
        }
        if (rc) break;
        c.vars[dir * kMaxOps + i] = t.cand[best];
        c.tuned.push_back(t);
      }
    }
    for (auto& g : c.graph)
      if (g) {
        hipGraphExecDestroy(g);
        g = nullptr;
      }
    if (rc) break;
  }
  // Second phase, for batches of several groups: the groups run at the same
  // time, and a variant that wins alone can lose when other groups' blocks
  // hold part of a CU (a wide tile with most of a CU's LDS; both fields of a
  // pass in one block).  Each width policy is applied to every tuned pass and
  // timed on a short concurrent run of forward steps of every group, the
  // policies taking turns over several rounds (the best run of each counts).
  // The incumbent, 8 columns with one field per block, is kept unless
  // another policy beats it by the margin: the run-to-run spread of these
  // timings is a few tenths of a percent, the isolated timings favour
  // variants that lose in context (measured on the 48-instance batch, forward
  // + adjoint: the untuned default 689-693 ms; both fields per block for
  // every two-field pass 721-730 ms; the isolated winners mixed, 736 ms).
  b->policy = -1;
  for (auto& u : b->policy_us) u = 0.f;
  if (!rc && b->cls.size() > 1) {
    std::vector<std::vector<ColVariant>> choice(TP_COUNT);
    std::vector<int> pols;
    for (int pol = 0; pol < TP_COUNT; ++pol) {
      for (auto& c : b->cls)
        for (const auto& t : c.tuned) choice[pol].push_back(t.cand[pick_variant(t, pol)]);
      bool same = false;
      for (int q : pols)
        same = same || std::equal(choice[q].begin(), choice[q].end(), choice[pol].begin(),
                                  [](const ColVariant& x, const ColVariant& y) {
                                    return x.tile == y.tile && x.fpb == y.fpb;
                                  });
      if (!same) pols.push_back(pol);
    }
    for (int r = 0; r < kPolicyRounds && !rc; ++r)
      for (int pol : pols) {
        apply_choice(b, choice[pol]);
        float ms = 0.f;
        rc = time_concurrent(b, 4 * b->chunk, st, e0, e1, &ms);  // captures the graphs
        if (!rc) rc = time_concurrent(b, 4 * b->chunk, st, e0, e1, &ms);
        if (rc) break;
        if (b->policy_us[pol] <= 0.f || 1e3f * ms < b->policy_us[pol]) b->policy_us[pol] = 1e3f * ms;
      }
    if (!rc) {
      int best = pols[0];
      for (int pol : pols)
        if (b->policy_us[pol] < b->policy_us[best]) best = pol;
      if (b->policy_us[best] > (1.f - kPolicyMargin) * b->policy_us[pols[0]]) best = pols[0];
      apply_choice(b, choice[best]);
      b->policy = best;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}

// JSON list of the chosen widths: one object per tuned pass with the class
// shape, direction, pass index, mode, field count, axis length, candidates
// with their mean microseconds and the choice.  Writes at most cap bytes
// (NUL-terminated) and the full length (without the NUL) to *needed.
extern "C" int pat_tuning_report(const pat_batch* b, char* buf, size_t cap, size_t* needed) {
  if (!b || !needed || (cap && !buf)) return PAT_EINVAL;
  std::string s = "[";
  char tmp[256];
  bool firsto = true;
  for (const auto& c : b->cls) {
    for (const auto& t : c.tuned) {
      PassOp ops[kMaxOps];
      step_ops(t.dir, c.ndim, c.lossy, ops);
      const ColSpec& cs = ops[t.idx].col;
      std::snprintf(tmp, sizeof tmp,
                    "%s{\"n\":[%d,%d,%d],\"nt\":%d,\"lossy\":%d,\"instances\":%d,\"dir\":%d,\"pass\":%d,"
                    "\"mode\":%d,\"nfield\":%d,\"axis_len\":%d,",
                    firsto ? "" : ",", c.nx, c.ny, c.nz, c.nt, c.lossy, (int)c.plans.size(), t.dir, t.idx, cs.mode,
                    cs.nfield, col_axis_len(cs, c.ndim, c.ny, c.nz));
      s += tmp;
      if (c.fused) {
        s += "\"fused\":[";
        for (size_t q = 0; q < c.shapes.size(); ++q) {
          std::snprintf(tmp, sizeof tmp, "%s[%d,%d]", q ? "," : "", c.shapes[q].first, c.shapes[q].second);
          s += tmp;
        }
        s += "],";
      }
      s += "\"candidates\":[";
      firsto = false;
      for (int j = 0; j < t.ncand; ++j) {
        std::snprintf(tmp, sizeof tmp, "%s{\"tile\":%d,\"fpb\":%d,\"us\":%.3f}", j ? "," : "", t.cand[j].tile,
                      t.cand[j].fpb, (double)t.us[j]);
        s += tmp;
      }
      const ColVariant& ch = c.vars[t.dir * kMaxOps + t.idx];
      std::snprintf(tmp, sizeof tmp, "],\"tile\":%d,\"fpb\":%d", ch.tile, ch.fpb);
      s += tmp;
      if (b->policy >= 0) {
        std::snprintf(tmp, sizeof tmp, ",\"policy\":\"%s\",\"policy_us\":{", kPolicyName[b->policy]);
        s += tmp;
        bool firstp = true;
        for (int q = 0; q < TP_COUNT; ++q) {
          if (b->policy_us[q] <= 0.f) continue;
          std::snprintf(tmp, sizeof tmp, "%s\"%s\":%.1f", firstp ? "" : ",", kPolicyName[q], (double)b->policy_us[q]);
          s += tmp;
          firstp = false;
        }
        s += "}";
      }
      s += "}";
    }
  }
  s += "]";
  *needed = s.size();
  if (cap) {
    const size_t n = std::min(cap - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return PAT_OK;
}

extern "C" int pat_batch_set_tile(pat_batch* b, const int32_t n[3], int32_t nt, int32_t lossy, int32_t dir,
                                  int32_t pass, int32_t tile, int32_t fields_per_block) {
  if (!b || !n || dir < 0 || dir > 1 || pass < 0 || pass >= kMaxOps || tile < 0 || fields_per_block < 1)
    return PAT_EINVAL;
  bool found = false;
  for (auto& c : b->cls) {
    if (c.nx != n[0] || c.ny != n[1] || c.nz != n[2] || c.nt != nt || c.lossy != (lossy != 0)) continue;
    PassOp ops[kMaxOps];
    const int nops = step_ops(dir, c.ndim, c.lossy, ops);
    if (pass >= nops || !ops[pass].is_col) return PAT_EINVAL;
    ColVariant v{tile, fields_per_block};
    if (tile) {
      ColVariant cand[kMaxColVar];
      const int nc = c.fused ? col_variants_fused(ops[pass].col, cand) : col_variants(ops[pass].col, c.ndim, c.ny, c.nz, cand);
      bool ok = false;
      for (int j = 0; j < nc; ++j) ok |= (cand[j].tile == tile && cand[j].fpb == fields_per_block);
      if (!ok) return PAT_EINVAL;
    } else if (fields_per_block != 1) {
      return PAT_EINVAL;
    }
    if (hipStreamSynchronize(c.st) != hipSuccess) return PAT_EHIP;
    c.vars[dir * kMaxOps + pass] = v;
    for (auto& g : c.graph)
      if (g) {
        hipGraphExecDestroy(g);
        g = nullptr;
      }
    found = true;
  }
  return found ? PAT_OK : PAT_EINVAL;
}

// ===================================================================== pass timing
// Back-to-back launches of one pass over the work tables of every class of
// grid width nx (0: all classes), one class at a time, timed with a pair of
// events around each class's burst.  The launches run a generic step (index
// 1, or 0 for a time axis of two samples) on whatever the state holds.
extern "C" int pat_batch_time_pass(pat_batch* b, int32_t dir, int32_t pass, int32_t nx, int32_t reps, void* stream,
                                   double* us_per_launch, double* bytes_per_launch) {
  if (!b || dir < 0 || dir > 1 || pass < 0 || pass >= kMaxOps || nx < 0 || reps < 1 || !us_per_launch ||
      !bytes_per_launch)
    return PAT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (hipStreamSynchronize(st) != hipSuccess) return PAT_EHIP;
  for (auto& c : b->cls)
    if (hipStreamSynchronize(c.st) != hipSuccess) return PAT_EHIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return PAT_EHIP;
  }
  int rc = PAT_OK;
  double ms_total = 0, bytes = 0;
  long launches = 0;
  for (auto& c : b->cls) {
    if (nx && c.nx != nx) continue;
    PassOp ops[kMaxOps];
    const int nops = step_ops(dir, c.ndim, c.lossy, ops);
    // passes that read the caller's arrays (the adjoint's data scatter) are
    // not timed here: those arrays may be gone
    if (pass >= nops || c.nt < 2 || (!ops[pass].is_col && (ops[pass].row == R_ADJ_3 || ops[pass].row == R_ADJ_32LL))) {
      rc = PAT_EINVAL;
      break;
    }
    const Runner R = c.runner();
    const StepArg sa{nullptr, c.nt > 2 ? 1 : 0};
    rc = R.launch1(dir, pass, ops[pass], sa, st, nullptr, nullptr);
    if (!rc && hipEventRecord(e0, st) != hipSuccess) rc = PAT_EHIP;
    for (int r = 0; r < reps && !rc; ++r) rc = R.launch1(dir, pass, ops[pass], sa, st, nullptr, nullptr);
    if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = PAT_EHIP;
    float ms = 0;
    if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) rc = PAT_EHIP;
    if (rc) break;
    ms_total += ms;
    launches += reps;
    bytes += reps * pass_bytes_per_point(ops[pass], c.ndim, c.lossy) * R.points;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (!rc && launches == 0) rc = PAT_EINVAL;
  if (rc) return rc;
  *us_per_launch = 1e3 * ms_total / (double)launches;
  *bytes_per_launch = bytes / (double)launches;
  return PAT_OK;
}
