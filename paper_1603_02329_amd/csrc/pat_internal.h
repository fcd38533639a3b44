// Internal declarations shared by the host runtime and the gfx950 kernels.
//
// A solver instance ("plan") lives in device memory as a DevPlan record: the
// kernels read every size, pointer and scalar they need from it, so a single
// launch can serve many instances through a work table of (instance, tile)
// pairs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pat.h"
#include "host_plan.h"

namespace pat {

constexpr int kMaxDim = 3;
// fixed-point steps of the t = 0 equation of state (PAT_EOS_INIT); plans
// whose contraction max |eta| |k|^(y-1) exceeds kEosMaxContraction are
// rejected: 0.05^7 < 1e-9, below float rounding
constexpr int kEosSteps = 6;
constexpr double kEosMaxContraction = 0.05;
constexpr int TWN = 1024;  // twiddle table length: exp(-2 pi i q / TWN), q < TWN

// Twiddle stored as an unevaluated float sum hi + lo (per component), so
// that the systematic float32 rounding of the table does not enter the FFT.
struct alignas(16) Tw {
  float hr, hi, lr, li;
};

// Everything one instance needs on the device.  Arrays are float32,
// row-major with x fastest; "packed spectra" hold per row nx/2 complex
// values of the x-transform, with bin 0 carrying (X[0], X[nx/2]) -- both real.
struct DevPlan {
  int32_t ndim;
  int32_t n[3];      // nx, ny, nz (nz = 1 in 2D)
  int32_t nrows;     // ny * nz
  int32_t nt;
  int32_t ns;
  int32_t nslots;
  int32_t lossy;
  uint32_t flags;
  float dt;
  float kap2;        // (c_ref * dt / 2)^2: kappa = sinc(sqrt(kap2 * |k|^2))
  float ym2h, ym1h;  // (y - 2)/2 and (y - 1)/2: |k|^(y-2) = (|k|^2)^ym2h
  float inv_dt;
  float scale;       // 1 / (nx ny nz): normalisation of a forward+inverse pair
  // spatially uniform alpha0: c0^2 tau = ktau (c0^2)^etau, c0^2 eta = keta (c0^2)^eeta
  int32_t alpha_uniform;
  float ktau, etau, keta, eeta;

  // medium coefficients (N each)
  const float* B[3];     // dt / rho0 at the staggered points of each axis
  const float* dtr0;     // dt * rho0
  const float* c2;       // c0^2
  const float* c2tau;    // c0^2 tau
  const float* c2eta;    // c0^2 eta
  const float* inv_dc2;  // 1 / (d c0^2)

  // per-axis 1-D tables
  const float* Q[3];       // PML factor exp(-sigma dt/2) on nodes, length n[j]
  const float* Qsg[3];     // ... on staggered points
  const float* ksq[3];     // k_j^2; x: packed bins 0..nx/2, y/z: 0..n-1
  const float2* shA[3];    // i k_j exp(+i k_j dx_j/2)
  const float2* shB[3];    // i k_j exp(-i k_j dx_j/2)
  const float* win[3];     // smoothing window of p0 (PAT_SMOOTH_P0), bins as ksq

  // state (N floats each) and packed spectra (N/2 complex each)
  float* u[3];
  float* r[3];
  float* q;
  float2* S[4];

  // sensors
  const int32_t* g_ptr;   // [nrows + 1]
  const GTap* g_tap;
  const int32_t* s_ptr;   // [nrows + 1]
  const SGroup* s_grp;
  const STap* s_tap;
  float* sc;                // [nt][ngroups]: W^T h of every sample per node group (adjoint, formed per call)
  int32_t ngroups;          // node groups of the scatter operator
  const int32_t* slot_ptr;  // [ns + 1]
  float* partial;           // [nt][nslots]
  int32_t* bad;             // non-finite flag (PAT_CHECK_FINITE)

  // per-call I/O pointers (set by the executor before launching)
  const float* in;   // p0 (forward) or data (adjoint)
  float* out;        // data (forward) or image (adjoint)
};

// Step index of a launch: n = (ctr ? *ctr : 0) + k.  Graph-captured chunks
// pass a device counter advanced once per chunk; eager launches pass k only.
// span: steps of the longest instance of a fused launch (0: not fused).
struct StepArg {
  const int32_t* ctr;
  int32_t k;
  int32_t span = 0;
};

__device__ __forceinline__ int step_of(const StepArg& s) { return (s.ctr ? *s.ctr : 0) + s.k; }

// Step of one instance inside a fused launch.  The launch's step n (of
// `span`) runs the instance's step floor(n S / span), S = nt - 1 of the
// instance, at the n where that value advances: each of the instance's S
// steps runs exactly once, in order, spread evenly over the span.  With
// span = 0 every instance runs step n.  Returns whether the instance runs.
__device__ __forceinline__ bool fused_step(const DevPlan& P, const StepArg& s, int& it) {
  const int n = step_of(s);
  if (s.span <= 0) {
    it = n;
    return true;
  }
  const long S = P.nt - 1;
  const long a = (long)n * S / s.span, b = ((long)n + 1) * S / s.span;
  it = (int)a;
  return b > a;
}

// multiplier kinds of the column passes
enum Mult : int32_t {
  M_AX = 0, M_AY = 1, M_AZ = 2,   // a_j = i k_j kappa e^{+i k_j dx_j/2}
  M_BX = 3, M_BY = 4, M_BZ = 5,   // b_j = i k_j kappa e^{-i k_j dx_j/2}
  M_L1DT = 6,                      // |k|^(y-2) / dt
  M_L2 = 7,                        // |k|^(y-1)
  M_WIN = 8,                       // separable smoothing window of p0, real
};

// ---------------------------------------------------------------- launchers
// (defined in passes.hip; all return hipError_t of the launch)
struct Launch {
  const DevPlan* plans;  // device array
  const int2* table;     // device work table (instance, tile) or nullptr
  int32_t nblocks;
  hipStream_t stream;
  hipEvent_t ev0 = nullptr;  // optional: stamped at the kernel's start and end
  hipEvent_t ev1 = nullptr;
};

enum RowKind : int32_t {
  R_FWD_INIT = 0,
  R_FWD_1 = 1,
  R_FWD_2 = 2,       // lossy: density update, feeds the absorption pass
  R_FWD_2LL = 3,     // lossless: density update + equation of state + gather
  R_FWD_3 = 4,       // lossy equation of state + gather
  R_ADJ_3 = 5,       // lossy: scatter, transposed equation of state (first half)
  R_ADJ_32LL = 6,    // lossless: scatter + transposed state + density
  R_ADJ_2 = 7,       // lossy: transposed absorption + density
  R_ADJ_1 = 8,       // transposed velocity update
  R_ADJ_FINAL = 9,   // transposed initial condition -> image
  R_ADJ_SCATTER_ONLY = 10,  // nt == 1: image = W^T h[0]
  // adjoint-then-discretize (the paper's adjoint system, eq. moma, massa,
  // statea): the forward's passes with the time-reversed data as a mass
  // source and the state equation in statea's order
  R_ATD_2 = 11,      // lossy: density + data source, feeds the absorption pass
  R_ATD_2LL = 12,    // lossless: density + data source + equation of state
  R_ATD_3 = 13,      // lossy equation of state (statea)
  R_ATD_FINAL = 14,  // image = sum_j rho*_j / rho0 (eq. adjj)
  // smoothing of the initial pressure (PAT_SMOOTH_P0): S = F^-1 w F, the
  // window w applied by a column pass (M_WIN) between two row passes
  R_FILT_IN = 15,    // S0 <- F_x in         (forward: p0)
  R_FWD_INIT_F = 16, // R_FWD_INIT from the filtered p0 = F_x^-1 S0
  R_FILT_RE = 17,    // S0 <- F_x out        (adjoint: the image)
  R_FILT_OUT = 18,   // out <- F_x^-1 S0
  // initial density from the equation of state at t = 0 (PAT_EOS_INIT),
  // c0^2 (1 - eta L2) rho(0) = p0, by fixed-point steps x <- b + eta L2 x
  // (forward) and y <- b + L2 (eta y) (adjoint), L2 applied by a column pass
  // on S1 between two row passes; step_of() = 1 marks the last step
  R_EOS_FWD_IN = 19,  // S1 <- F_x r_0 (r_j = p0 / (d c0^2) after R_FWD_INIT)
  R_EOS_FWD = 20,     // r_0 <- r_1 + eta F_x^-1 S1; then S1 <- F_x r_0, or (last) every r_j <- r_0
  R_EOS_ADJ_IN = 21,  // q <- sum_j r_j / d; r_0 <- q; S1 <- F_x (eta r_0)
  R_EOS_ADJ = 22,     // r_0 <- q + F_x^-1 S1; then S1 <- F_x (eta r_0), or (last) r_0 <- d r_0, r_j <- 0 (j > 0)
  R_COUNT = 23
};

hipError_t launch_row(RowKind kind, int ndim, int nx, const Launch& L, StepArg s);
// rows per work item of the row passes for row length nx
int row_tile_rows(int nx);

// Column passes.  Modes 0-2 run along the last axis (y in 2D, z in 3D):
// transform, k-space multiplier(s), inverse transform.  Modes 3-4 are the
// forward / inverse transform along y alone (3D).
// mode 0: S[1+i] = mult[i] S[0]                    (i < nfield)
// mode 1: S[f]   = mult[i] S[f],  f = f0 + i       (fields split over
//         blockIdx.y, `fpb` fields per block)
// mode 2: S[0]   = sum_i mult[i] S[f0 + i]
// mode 3/4: S[f0 + i] <- F_y / F_y^-1 S[f0 + i]    (blockIdx.y = i)
struct ColSpec {
  int32_t mode;
  int32_t nfield;
  int32_t mult[3];
  int32_t f0;
  int32_t tile = 0;  // columns per block (0: the default)
  int32_t fpb = 1;   // mode 1: fields per block, 1 or nfield
};
// a compiled launch shape of a column pass: columns per block and (mode 1)
// fields per block
struct ColVariant {
  int32_t tile, fpb;
};
constexpr int kMaxColVar = 8;
hipError_t launch_col(const ColSpec& spec, int ndim, int nx, int ny, int nz, const Launch& L);
int col_blocks(const ColSpec& spec, int ndim, int nx, int ny, int nz);
// the compiled variants of a pass (the default first); returns their count
int col_variants(const ColSpec& spec, int ndim, int ny, int nz, ColVariant* out);
// the variant spec.tile / spec.fpb name, or the default when not compiled
ColVariant col_variant_of(const ColSpec& spec, int ndim, int ny, int nz);
int col_axis_len(const ColSpec& spec, int ndim, int ny, int nz);

hipError_t launch_reduce(const Launch& L, int n0, int n1);

// Fused launches (2D, both axis lengths 128, 256 or 512): one launch covers
// instances of several sizes, each block running the pass of its own
// instance's size.  Row passes: 256 threads, 4096 / nx rows per block.
// Column passes: variant tile t (8 or 4) means NTH = 64 t threads per block,
// NTH * 8 / ny columns per block for a column of ny points.
bool fused_size(int n);
int fused_row_rows(int nx);
int fused_col_tile(int ny, int tile);
int col_variants_fused(const ColSpec& spec, ColVariant* out);
hipError_t launch_row_fused(RowKind kind, const Launch& L, StepArg s);
hipError_t launch_col_fused(const ColSpec& spec, ColVariant v, const Launch& L, StepArg s);

// Forward / adjoint pass sequences shared by the eager and batched executors.
// Each entry is one launch: a row pass (kind) or a column pass (spec).
struct PassOp {
  int32_t is_col;
  RowKind row;
  ColSpec col;
};
// fills ops[] with the passes of one time step; returns their count
constexpr int kMaxOps = 16;
int step_ops(int direction /*0 fwd, 1 adj*/, int ndim, int lossy, PassOp* ops);

// algorithmic HBM bytes per grid point of one launch of a pass (float32,
// 2D): reads + writes of full-grid arrays the pass must touch
double pass_bytes_per_point(const PassOp& op, int ndim, int lossy);

// drop the batches pat_forward_batched / pat_adjoint_batched keep for plan
// lists that hold p (called when p is destroyed)
void batch_cache_forget(const pat_plan* p);


}  // namespace pat

struct pat_plan {
  pat_desc desc{};
  int device = 0;
  double dt = 0, c_ref = 0;
  int lossy = 0;
  int64_t npoints = 0;
  int nslots = 0;
  pat::DevPlan hp{};            // host image of the device record
  pat::DevPlan* dp = nullptr;   // device record
  void* arena = nullptr;        // all device buffers of the plan
  size_t arena_bytes = 0;
  size_t state_bytes = 0;
};
