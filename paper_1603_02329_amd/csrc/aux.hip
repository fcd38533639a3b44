// Auxiliary operators of the multi-grid ISTA/FISTA iteration on gfx950:
// the TV proximal map (dual FGP), the level-transfer operators and the
// float64 reductions.  All are O(N) per call (the prox: O(N) per iteration).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "pat_internal.h"

namespace {

#define PAT_TRY_HIP(x)                     \
  do {                                     \
    hipError_t e_ = (x);                   \
    if (e_ != hipSuccess) return PAT_EHIP; \
  } while (0)

struct Grid3 {
  int n[3];
  long N;
  long stride[3];
};

int make_grid(int ndim, const int32_t* n, Grid3& g) {
  if ((ndim != 2 && ndim != 3) || !n) return PAT_EINVAL;
  g.N = 1;
  for (int j = 0; j < 3; ++j) {
    g.n[j] = (j < ndim) ? n[j] : 1;
    if (g.n[j] < 1) return PAT_EINVAL;
  }
  g.stride[0] = 1;
  g.stride[1] = g.n[0];
  g.stride[2] = (long)g.n[0] * g.n[1];
  g.N = (long)g.n[0] * g.n[1] * g.n[2];
  return PAT_OK;
}

inline int blocks_for(long n, int per = 256) { return (int)((n + per - 1) / per); }

// ------------------------------------------------------------------ FGP prox
// x = max(z - lam * L r, lower), with (L r)_i = sum_a r_a[i] - r_a[i - e_a]
// (r_a is zero on axis a's last index and outside the grid).
__device__ __forceinline__ void prox_primal_at(const Grid3& g, int ndim, long i, const float* __restrict__ z,
                                               const float* __restrict__ lower, const float* __restrict__ r,
                                               float lam, float* __restrict__ x) {
  long rem = i;
  int idx[3];
  for (int j = 0; j < 3; ++j) {
    idx[j] = (int)(rem % g.n[j]);
    rem /= g.n[j];
  }
  float div = 0.f;
  for (int a = 0; a < ndim; ++a) {
    const float* ra = r + (long)a * g.N;
    if (idx[a] < g.n[a] - 1) div += ra[i];
    if (idx[a] > 0) div -= ra[i - g.stride[a]];
  }
  const float lo = lower ? lower[i] : 0.f;
  x[i] = fmaxf(z[i] - lam * div, lo);
}
__global__ void k_prox_primal(Grid3 g, int ndim, const float* __restrict__ z, const float* __restrict__ lower,
                              const float* __restrict__ r, float lam, float* __restrict__ x) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g.N) prox_primal_at(g, ndim, i, z, lower, r, lam, x);
}

// p = P_P(r + step * Lt x) with Lt x = x[i] - x[i + e_a] (0 on the last index);
// r <- p + theta (p - p_prev); p_prev <- p.
__device__ __forceinline__ void prox_dual_at(const Grid3& g, int ndim, long i, const float* __restrict__ x,
                                             float step, float theta, float* __restrict__ r,
                                             float* __restrict__ pprev) {
  long rem = i;
  int idx[3];
  for (int j = 0; j < 3; ++j) {
    idx[j] = (int)(rem % g.n[j]);
    rem /= g.n[j];
  }
  float v[3] = {0.f, 0.f, 0.f};
  float nrm2 = 0.f;
  for (int a = 0; a < ndim; ++a) {
    const float d = (idx[a] < g.n[a] - 1) ? x[i] - x[i + g.stride[a]] : 0.f;
    v[a] = r[(long)a * g.N + i] + step * d;
    nrm2 += v[a] * v[a];
  }
  const float s = fmaxf(1.f, sqrtf(nrm2));
  for (int a = 0; a < ndim; ++a) {
    const float pa = v[a] / s;
    const long k = (long)a * g.N + i;
    const float pp = pprev[k];
    r[k] = pa + theta * (pa - pp);
    pprev[k] = pa;
  }
}
__global__ void k_prox_dual(Grid3 g, int ndim, const float* __restrict__ x, float step, float theta,
                            float* __restrict__ r, float* __restrict__ pprev) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < g.N) prox_dual_at(g, ndim, i, x, step, theta, r, pprev);
}

// Several images in one launch: image k owns blocks [begin[k], begin[k+1]).
// The argument block stays under the 4 KB of kernel arguments.
constexpr int kProxBatch = 24;
struct ProxBatch {
  int count, ndim;
  int begin[kProxBatch + 1];
  Grid3 g[kProxBatch];
  const float* z[kProxBatch];
  const float* lower[kProxBatch];
  float* x[kProxBatch];
  float* r[kProxBatch];      // dual iterate (ndim * N), then p_prev (ndim * N), then x_t (N)
  float lam[kProxBatch], step[kProxBatch];
};
__device__ __forceinline__ int prox_image(const ProxBatch& b) {
  int k = 0;
  while (k + 1 < b.count && (int)blockIdx.x >= b.begin[k + 1]) ++k;
  return k;
}
// final = 0: x_t <- P_C(z - lam L r); final = 1: x <- P_C(z - lam L p_prev)
__global__ void k_prox_primal_b(ProxBatch b, int final) {
  const int k = prox_image(b);
  const long i = (long)(blockIdx.x - b.begin[k]) * blockDim.x + threadIdx.x;
  const Grid3& g = b.g[k];
  if (i >= g.N) return;
  const float* r = b.r[k] + (final ? (long)b.ndim * g.N : 0);
  float* out = final ? b.x[k] : b.r[k] + 2L * b.ndim * g.N;
  prox_primal_at(g, b.ndim, i, b.z[k], b.lower[k], r, b.lam[k], out);
}
__global__ void k_prox_dual_b(ProxBatch b, float theta) {
  const int k = prox_image(b);
  const long i = (long)(blockIdx.x - b.begin[k]) * blockDim.x + threadIdx.x;
  const Grid3& g = b.g[k];
  if (i >= g.N) return;
  float* r = b.r[k];
  prox_dual_at(g, b.ndim, i, r + 2L * b.ndim * g.N, b.step[k], theta, r, r + (long)b.ndim * g.N);
}
__global__ void k_prox_zero_b(ProxBatch b) {  // r and p_prev of every image
  const int k = prox_image(b);
  const long i = (long)(blockIdx.x - b.begin[k]) * blockDim.x + threadIdx.x;
  const Grid3& g = b.g[k];
  if (i >= g.N) return;
  for (int a = 0; a < 2 * b.ndim; ++a) b.r[k][(long)a * g.N + i] = 0.f;
}

__global__ void k_proj(long n, const float* __restrict__ z, const float* __restrict__ lower, float* __restrict__ x) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = fmaxf(z[i], lower ? lower[i] : 0.f);
}

__global__ void k_zero(long n, float* __restrict__ a) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.f;
}

// ------------------------------------------------------------------ transfers
__global__ void k_restrict(Grid3 c, int ndim, const float* __restrict__ fine, float* __restrict__ coarse) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.N) return;
  const int cx = (int)(i % c.n[0]);
  const int cy = (int)((i / c.n[0]) % c.n[1]);
  const int cz = (int)(i / ((long)c.n[0] * c.n[1]));
  const long fx = 2L * c.n[0], fy = 2L * c.n[1];
  float acc = 0.f;
  const int nzc = ndim == 3 ? 2 : 1;
  for (int dz = 0; dz < nzc; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const long f = (2L * cx + dx) + fx * ((2L * cy + dy) + fy * (ndim == 3 ? (2L * cz + dz) : 0));
        acc += fine[f];
      }
  coarse[i] = acc * (ndim == 3 ? 0.125f : 0.25f);
}

__global__ void k_prolong(Grid3 f, int ndim, const float* __restrict__ coarse, float* __restrict__ fine) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= f.N) return;
  const int fx = (int)(i % f.n[0]);
  const int fy = (int)((i / f.n[0]) % f.n[1]);
  const int fz = (int)(i / ((long)f.n[0] * f.n[1]));
  const long cxn = f.n[0] / 2, cyn = f.n[1] / 2;
  const long c = (fx / 2) + cxn * ((fy / 2) + cyn * (ndim == 3 ? (fz / 2) : 0));
  fine[i] = coarse[c];
}

// ------------------------------------------------------------------ smoothed TV
// The smoothed TV of equation Thirty-two, J_rho(x) = sum_j sqrt(|Lt x|_j^2 +
// rho^2) - rho, with Lt x the forward differences of the prox (zero across
// each axis' last face), and its gradient L w, w = Lt x / sqrt(|Lt x|^2 +
// rho^2) (for rho = 0, w = 0 where Lt x = 0).
struct TvPoint {
  float d[3];
  float s;  // sqrt(|Lt x|^2 + rho^2)
};
__device__ __forceinline__ TvPoint tv_point(const Grid3& g, int ndim, const float* __restrict__ x, long j,
                                            const int* idx, float rho2) {
  TvPoint p{{0.f, 0.f, 0.f}, 0.f};
  float q = rho2;
  for (int a = 0; a < ndim; ++a) {
    p.d[a] = (idx[a] < g.n[a] - 1) ? x[j] - x[j + g.stride[a]] : 0.f;
    q += p.d[a] * p.d[a];
  }
  p.s = sqrtf(q);
  return p;
}
__device__ __forceinline__ float tv_w(const TvPoint& p, int a) { return p.s > 0.f ? p.d[a] / p.s : 0.f; }

// grad += scale * (L w)_i, (L w)_i = sum_a w_a[i] - w_a[i - e_a]
__global__ void k_tv_grad(Grid3 g, int ndim, const float* __restrict__ x, float rho2, float scale,
                          float* __restrict__ grad) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  long rem = i;
  int idx[3];
  for (int j = 0; j < 3; ++j) {
    idx[j] = (int)(rem % g.n[j]);
    rem /= g.n[j];
  }
  const TvPoint pi = tv_point(g, ndim, x, i, idx, rho2);
  float acc = 0.f;
  for (int a = 0; a < ndim; ++a) {
    acc += tv_w(pi, a);
    if (idx[a] > 0) {
      int jdx[3] = {idx[0], idx[1], idx[2]};
      jdx[a] -= 1;
      const TvPoint pj = tv_point(g, ndim, x, i - g.stride[a], jdx, rho2);
      acc -= tv_w(pj, a);
    }
  }
  grad[i] += scale * acc;
}

// ------------------------------------------------------------------ bound restriction
// lower_c[I] = (R y)[I] - min over the block {2I + delta} of (y - l): for
// every coarse x_c >= lower_c, y + P(x_c - R y) >= l on the block (l = 0
// when fl is null).
__global__ void k_restrict_lower(Grid3 c, int ndim, const float* __restrict__ fine, const float* __restrict__ fl,
                                 float* __restrict__ lower) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.N) return;
  const int cx = (int)(i % c.n[0]);
  const int cy = (int)((i / c.n[0]) % c.n[1]);
  const int cz = (int)(i / ((long)c.n[0] * c.n[1]));
  const long fx = 2L * c.n[0], fy = 2L * c.n[1];
  float acc = 0.f, mn = INFINITY;
  const int nzc = ndim == 3 ? 2 : 1;
  for (int dz = 0; dz < nzc; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const long f = (2L * cx + dx) + fx * ((2L * cy + dy) + fy * (ndim == 3 ? (2L * cz + dz) : 0));
        acc += fine[f];
        mn = fminf(mn, fl ? fine[f] - fl[f] : fine[f]);
      }
  lower[i] = acc * (ndim == 3 ? 0.125f : 0.25f) - mn;
}

// ------------------------------------------------------------------ vector updates
__global__ void k_axpby(long n, float a, const float* x, float b, const float* y, float* out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * x[i] + b * y[i];
}

// ------------------------------------------------------------------ float64 reductions
constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;

// Fixed partition: block b sums the contiguous chunk b of the input, each
// thread a strided subsequence in order, then a fixed tree -> deterministic.
template <int OP>  // 0: a*b   1: (a-b)^2/2 and r = a-b
__global__ void __launch_bounds__(kRedThreads) k_red1(const float* __restrict__ a, const float* __restrict__ b,
                                                      float* __restrict__ r, long n, double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  const long chunk = (n + kRedBlocks - 1) / kRedBlocks;
  const long beg = (long)blockIdx.x * chunk;
  const long end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  for (long i = beg + threadIdx.x; i < end; i += kRedThreads) {
    if (OP == 0) {
      acc += (double)a[i] * (double)b[i];
    } else {
      const float d = a[i] - b[i];
      r[i] = d;
      acc += 0.5 * (double)d * (double)d;
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__device__ __forceinline__ void k_red2_body(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}
__global__ void __launch_bounds__(kRedThreads) k_red2(const double* __restrict__ part, double* __restrict__ out) {
  k_red2_body(part, out);
}

// Batched residuals: block (b, i) runs k_red1<1>'s block b on pair i, so
// that every pair's value equals the unbatched call's bitwise.
constexpr int kResMax = 64;  // pairs per launch (kernel arguments)
struct ResPairs {
  const float* a[kResMax];
  const float* b[kResMax];
  float* r[kResMax];
  long n[kResMax];
};
__global__ void __launch_bounds__(kRedThreads) k_res1_b(ResPairs P, double* __restrict__ part) {
  const int i = blockIdx.y;
  __shared__ double sh[kRedThreads];
  const long n = P.n[i];
  const float* __restrict__ a = P.a[i];
  const float* __restrict__ b = P.b[i];
  float* __restrict__ r = P.r[i];
  const long chunk = (n + kRedBlocks - 1) / kRedBlocks;
  const long beg = (long)blockIdx.x * chunk;
  const long end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  for (long k = beg + threadIdx.x; k < end; k += kRedThreads) {
    const float d = a[k] - b[k];
    r[k] = d;
    acc += 0.5 * (double)d * (double)d;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long)i * kRedBlocks + blockIdx.x] = sh[0];
}
// out[i] = k_red2 over pair i's partials; block i
__global__ void __launch_bounds__(kRedThreads) k_res2_b(const double* __restrict__ part, double* __restrict__ out) {
  k_red2_body(part + (long)blockIdx.x * kRedBlocks, out + blockIdx.x);
}
// out[count] = sum of out[0 .. count) in index order
__global__ void k_res_sum(double* __restrict__ out, int count) {
  double s = 0.0;
  for (int i = 0; i < count; ++i) s += out[i];
  out[count] = s;
}

// sum_j sqrt(|Lt x|_j^2 + rho^2) - rho, same fixed partition as k_red1
__global__ void __launch_bounds__(kRedThreads) k_red_tv(Grid3 g, int ndim, const float* __restrict__ x, double rho,
                                                        double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  const long chunk = (g.N + kRedBlocks - 1) / kRedBlocks;
  const long beg = (long)blockIdx.x * chunk;
  const long end = beg + chunk < g.N ? beg + chunk : g.N;
  double acc = 0.0;
  for (long i = beg + threadIdx.x; i < end; i += kRedThreads) {
    long rem = i;
    int idx[3];
    for (int j = 0; j < 3; ++j) {
      idx[j] = (int)(rem % g.n[j]);
      rem /= g.n[j];
    }
    double q = rho * rho;
    for (int a = 0; a < ndim; ++a) {
      const double d = (idx[a] < g.n[a] - 1) ? (double)x[i] - (double)x[i + g.stride[a]] : 0.0;
      q += d * d;
    }
    acc += sqrt(q) - rho;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Scratch of the float64 reductions (kRedBlocks partials + 1 result), one
// buffer per (device, stream): calls on one stream run in stream order and
// share it; calls on different streams, or from different threads on
// different streams, never do.  Allocated on a stream's first reduction and
// kept until the process ends (4 KB each).
std::mutex g_red_mu;
std::map<std::pair<int, hipStream_t>, double*> g_red_buf;

int red_buffer(hipStream_t st, double** out) {
  int dev = 0;
  PAT_TRY_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_red_mu);
  double*& b = g_red_buf[std::make_pair(dev, st)];
  if (!b && hipMalloc(&b, sizeof(double) * (kRedBlocks + 1)) != hipSuccess) {
    b = nullptr;
    return PAT_ENOMEM;
  }
  *out = b;
  return PAT_OK;
}

}  // namespace

// ===================================================================== C entry points
extern "C" size_t pat_tv_prox_work_bytes(int32_t ndim, const int32_t n[3]) {
  Grid3 g;
  if (make_grid(ndim, n, g)) return 0;
  return (size_t)(2 * ndim + 1) * (size_t)g.N * sizeof(float);
}

extern "C" int pat_tv_prox_batched(int32_t count, int32_t ndim, const int32_t* n, const float* const* z,
                                   float* const* x, const double* lambda_eff, int32_t n_iter,
                                   const float* const* lower, void* const* work, const size_t* work_bytes,
                                   void* stream) {
  if (count < 0 || (count > 0 && (!n || !z || !x || !lambda_eff || !work || !work_bytes)) || n_iter < 0)
    return PAT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  // validate everything before launching anything
  for (int k = 0; k < count; ++k) {
    Grid3 g;
    if (make_grid(ndim, n + 3 * k, g)) return PAT_EINVAL;
    if (!z[k] || !x[k] || z[k] == x[k] || !(lambda_eff[k] >= 0) || !std::isfinite(lambda_eff[k])) return PAT_EINVAL;
    if (lambda_eff[k] > 0 && n_iter > 0 &&
        (!work[k] || work_bytes[k] < pat_tv_prox_work_bytes(ndim, n + 3 * k)))
      return PAT_EINVAL;
  }
  std::vector<int> iter;  // images that run FGP iterations; the others are projections
  for (int k = 0; k < count; ++k) {
    if (lambda_eff[k] > 0 && n_iter > 0) {
      iter.push_back(k);
    } else {
      const int rc = pat_tv_prox(ndim, n + 3 * k, z[k], x[k], lambda_eff[k], n_iter, lower ? lower[k] : nullptr,
                                 work[k], work_bytes[k], stream);
      if (rc) return rc;
    }
  }
  for (size_t k0 = 0; k0 < iter.size(); k0 += kProxBatch) {
    ProxBatch b{};
    b.count = (int)std::min<size_t>(kProxBatch, iter.size() - k0);
    b.ndim = ndim;
    b.begin[0] = 0;
    for (int j = 0; j < b.count; ++j) {
      const int k = iter[k0 + j];
      make_grid(ndim, n + 3 * k, b.g[j]);
      b.z[j] = z[k];
      b.lower[j] = lower ? lower[k] : nullptr;
      b.x[j] = x[k];
      b.r[j] = (float*)work[k];
      b.lam[j] = (float)lambda_eff[k];
      b.step[j] = (float)(1.0 / (4.0 * ndim * lambda_eff[k]));
      b.begin[j + 1] = b.begin[j] + blocks_for(b.g[j].N);
    }
    const int nb = b.begin[b.count];
    hipLaunchKernelGGL(k_prox_zero_b, dim3(nb), dim3(256), 0, st, b);
    double t = 1.0;
    for (int it = 0; it < n_iter; ++it) {
      const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      const float theta = (float)((t - 1.0) / tn);
      hipLaunchKernelGGL(k_prox_primal_b, dim3(nb), dim3(256), 0, st, b, 0);
      hipLaunchKernelGGL(k_prox_dual_b, dim3(nb), dim3(256), 0, st, b, theta);
      t = tn;
    }
    hipLaunchKernelGGL(k_prox_primal_b, dim3(nb), dim3(256), 0, st, b, 1);
    if (hipGetLastError() != hipSuccess) return PAT_EHIP;
  }
  return PAT_OK;
}

namespace {

// The FGP iterations of pat_tv_prox on a workspace of (2 ndim + 1) N floats
// (dual r, previous dual, primal iterate), which it clears itself.
int tv_prox_run(const Grid3& g, int ndim, const float* z, float* x, double lambda_eff, int n_iter,
                const float* lower, float* work, hipStream_t st) {
  const int nb = blocks_for(g.N);
  if (lambda_eff == 0.0 || n_iter == 0) {  // P_C(z - lam L 0) = P_C(z)
    hipLaunchKernelGGL(k_proj, dim3(nb), dim3(256), 0, st, g.N, z, lower, x);
    return hipGetLastError() == hipSuccess ? PAT_OK : PAT_EHIP;
  }
  float* r = work;
  float* pprev = r + (long)ndim * g.N;
  float* xt = pprev + (long)ndim * g.N;
  hipLaunchKernelGGL(k_zero, dim3(blocks_for(2L * ndim * g.N)), dim3(256), 0, st, 2L * ndim * g.N, r);
  const float lam = (float)lambda_eff;
  const float step = (float)(1.0 / (4.0 * ndim * lambda_eff));
  double t = 1.0;
  for (int k = 0; k < n_iter; ++k) {
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    const float theta = (float)((t - 1.0) / tn);
    hipLaunchKernelGGL(k_prox_primal, dim3(nb), dim3(256), 0, st, g, ndim, z, lower, r, lam, xt);
    hipLaunchKernelGGL(k_prox_dual, dim3(nb), dim3(256), 0, st, g, ndim, xt, step, theta, r, pprev);
    t = tn;
  }
  hipLaunchKernelGGL(k_prox_primal, dim3(nb), dim3(256), 0, st, g, ndim, z, lower, pprev, lam, x);
  return hipGetLastError() == hipSuccess ? PAT_OK : PAT_EHIP;
}

// Workspace of pat_tv_prox_noalloc: one copy per device, held until the
// process ends.  Host code never passes the array's name to a kernel; it
// uses the device address hipGetSymbolAddress returns for the current
// device (noalloc_scratch()).
constexpr long kNoallocFloats = PAT_TV_PROX_NOALLOC_FLOATS;
static __device__ __align__(256) float scratch[kNoallocFloats];

std::mutex g_scratch_mu;
std::vector<float*> g_scratch_ptr;  // per device: address of `scratch`

int noalloc_scratch(float** out) {
  int dev = 0;
  PAT_TRY_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PAT_EHIP;
    g_scratch_ptr[dev] = (float*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return PAT_OK;
}

}  // namespace

extern "C" int pat_tv_prox(int32_t ndim, const int32_t n[3], const float* z, float* x, double lambda_eff,
                           int32_t n_iter, const float* lower, void* work, size_t work_bytes, void* stream) {
  Grid3 g;
  if (make_grid(ndim, n, g)) return PAT_EINVAL;
  if (!z || !x || z == x || !(lambda_eff >= 0) || !std::isfinite(lambda_eff) || n_iter < 0) return PAT_EINVAL;
  if (lambda_eff != 0.0 && n_iter != 0 && (!work || work_bytes < pat_tv_prox_work_bytes(ndim, n))) return PAT_EINVAL;
  return tv_prox_run(g, ndim, z, x, lambda_eff, n_iter, lower, (float*)work, (hipStream_t)stream);
}

extern "C" int pat_tv_prox_noalloc(int32_t ndim, const int32_t n[3], const float* z, float* x, double lambda_eff,
                                   int32_t n_iter, const float* lower, void* stream) {
  Grid3 g;
  if (make_grid(ndim, n, g)) return PAT_EINVAL;
  if (!z || !x || z == x || !(lambda_eff >= 0) || !std::isfinite(lambda_eff) || n_iter < 0) return PAT_EINVAL;
  if ((long)(2 * ndim + 1) * g.N > kNoallocFloats) return PAT_ETOOBIG;
  float* work = nullptr;
  const int rc = noalloc_scratch(&work);
  if (rc) return rc;
  return tv_prox_run(g, ndim, z, x, lambda_eff, n_iter, lower, work, (hipStream_t)stream);
}

extern "C" int pat_restrict(int32_t ndim, const int32_t n_fine[3], const float* fine, float* coarse, void* stream) {
  Grid3 f;
  if (make_grid(ndim, n_fine, f) || !fine || !coarse) return PAT_EINVAL;
  int32_t nc[3];
  for (int j = 0; j < 3; ++j) {
    if (j < ndim && (f.n[j] % 2)) return PAT_EINVAL;
    nc[j] = j < ndim ? f.n[j] / 2 : 1;
  }
  Grid3 c;
  make_grid(ndim, nc, c);
  hipLaunchKernelGGL(k_restrict, dim3(blocks_for(c.N)), dim3(256), 0, (hipStream_t)stream, c, ndim, fine, coarse);
  return hipGetLastError() == hipSuccess ? PAT_OK : PAT_EHIP;
}

extern "C" int pat_prolong(int32_t ndim, const int32_t n_coarse[3], const float* coarse, float* fine, void* stream) {
  Grid3 c;
  if (make_grid(ndim, n_coarse, c) || !fine || !coarse) return PAT_EINVAL;
  int32_t nf[3];
  for (int j = 0; j < 3; ++j) nf[j] = j < ndim ? 2 * c.n[j] : 1;
  Grid3 f;
  make_grid(ndim, nf, f);
  hipLaunchKernelGGL(k_prolong, dim3(blocks_for(f.N)), dim3(256), 0, (hipStream_t)stream, f, ndim, coarse, fine);
  return hipGetLastError() == hipSuccess ? PAT_OK : PAT_EHIP;
}

static int reduce_common(int op, const float* a, const float* b, float* r, int64_t n, double* out_host,
                         hipStream_t st) {
  if (!out_host || n < 0 || ((!a || !b) && n > 0) || (op == 1 && !r && n > 0)) return PAT_EINVAL;
  if (n == 0) {
    *out_host = 0.0;
    return PAT_OK;
  }
  double* buf = nullptr;
  int rc = red_buffer(st, &buf);
  if (rc) return rc;
  if (op == 0)
    hipLaunchKernelGGL(k_red1<0>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, a, b, r, (long)n, buf);
  else
    hipLaunchKernelGGL(k_red1<1>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, a, b, r, (long)n, buf);
  hipLaunchKernelGGL(k_red2, dim3(1), dim3(kRedThreads), 0, st, buf, buf + kRedBlocks);
  PAT_TRY_HIP(hipGetLastError());
  PAT_TRY_HIP(hipMemcpyAsync(out_host, buf + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, st));
  PAT_TRY_HIP(hipStreamSynchronize(st));
  return PAT_OK;
}

extern "C" int pat_dot_f64(const float* a, const float* b, int64_t n, double* out_host, void* stream) {
  return reduce_common(0, a, b, nullptr, n, out_host, (hipStream_t)stream);
}

extern "C" int pat_residual_f64(const float* a, const float* b, float* r, int64_t n, double* half_sq_host,
                                void* stream) {
  return reduce_common(1, a, b, r, n, half_sq_host, (hipStream_t)stream);
}

extern "C" size_t pat_residual_batched_work_bytes(int32_t count) {
  return count < 1 ? 0 : (size_t)count * kRedBlocks * sizeof(double);
}

extern "C" int pat_residual_f64_batched(int32_t count, const float* const* a, const float* const* b, float* const* r,
                                        const int64_t* n, double* work_dev, double* out_dev, void* stream) {
  if (count < 1 || count > 4096 || !a || !b || !r || !n || !work_dev || !out_dev) return PAT_EINVAL;
  for (int i = 0; i < count; ++i)
    if (n[i] < 0 || (n[i] > 0 && (!a[i] || !b[i] || !r[i]))) return PAT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  for (int i0 = 0; i0 < count; i0 += kResMax) {
    const int m = count - i0 < kResMax ? count - i0 : kResMax;
    ResPairs P{};
    for (int i = 0; i < m; ++i) {
      P.a[i] = a[i0 + i];
      P.b[i] = b[i0 + i];
      P.r[i] = r[i0 + i];
      P.n[i] = (long)n[i0 + i];
    }
    double* part = work_dev + (long)i0 * kRedBlocks;
    hipLaunchKernelGGL(k_res1_b, dim3(kRedBlocks, m), dim3(kRedThreads), 0, st, P, part);
    hipLaunchKernelGGL(k_res2_b, dim3(m), dim3(kRedThreads), 0, st, part, out_dev + i0);
  }
  hipLaunchKernelGGL(k_res_sum, dim3(1), dim3(1), 0, st, out_dev, count);
  PAT_TRY_HIP(hipGetLastError());
  return PAT_OK;
}

extern "C" int pat_tv_smooth(int32_t ndim, const int32_t n[3], const float* x, double rho, double scale, float* grad,
                             double* value_host, void* stream) {
  Grid3 g;
  if (make_grid(ndim, n, g) || !x || !(rho >= 0) || !std::isfinite(rho) || !std::isfinite(scale) ||
      (!grad && !value_host) || (const float*)grad == x)
    return PAT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (grad) {
    hipLaunchKernelGGL(k_tv_grad, dim3(blocks_for(g.N)), dim3(256), 0, st, g, ndim, x, (float)(rho * rho),
                       (float)scale, grad);
    PAT_TRY_HIP(hipGetLastError());
  }
  if (value_host) {
    double* buf = nullptr;
    int rc = red_buffer(st, &buf);
    if (rc) return rc;
    hipLaunchKernelGGL(k_red_tv, dim3(kRedBlocks), dim3(kRedThreads), 0, st, g, ndim, x, rho, buf);
    hipLaunchKernelGGL(k_red2, dim3(1), dim3(kRedThreads), 0, st, buf, buf + kRedBlocks);
    PAT_TRY_HIP(hipGetLastError());
    PAT_TRY_HIP(hipMemcpyAsync(value_host, buf + kRedBlocks, sizeof(double), hipMemcpyDeviceToHost, st));
    PAT_TRY_HIP(hipStreamSynchronize(st));
  }
  return PAT_OK;
}

extern "C" int pat_restrict_lower(int32_t ndim, const int32_t n_fine[3], const float* fine,
                                  const float* fine_lower, float* lower, void* stream) {
  Grid3 f;
  if (make_grid(ndim, n_fine, f) || !fine || !lower) return PAT_EINVAL;
  int32_t nc[3];
  for (int j = 0; j < 3; ++j) {
    if (j < ndim && (f.n[j] % 2)) return PAT_EINVAL;
    nc[j] = j < ndim ? f.n[j] / 2 : 1;
  }
  Grid3 c;
  make_grid(ndim, nc, c);
  hipLaunchKernelGGL(k_restrict_lower, dim3(blocks_for(c.N)), dim3(256), 0, (hipStream_t)stream, c, ndim, fine,
                     fine_lower, lower);
  return hipGetLastError() == hipSuccess ? PAT_OK : PAT_EHIP;
}

extern "C" int pat_axpby(int64_t n, double a, const float* x, double b, const float* y, float* out, void* stream) {
  if (n < 0 || (n > 0 && (!x || !y || !out))) return PAT_EINVAL;
  if (n == 0) return PAT_OK;
  hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, (long)n, (float)a, x, (float)b,
                     y, out);
  return hipGetLastError() == hipSuccess ? PAT_OK : PAT_EHIP;
}

extern "C" int pat_project(int64_t n, const float* x, const float* lower, float* out, void* stream) {
  if (n < 0 || (n > 0 && (!x || !out))) return PAT_EINVAL;
  if (n == 0) return PAT_OK;
  hipLaunchKernelGGL(k_proj, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, (long)n, x, lower, out);
  return hipGetLastError() == hipSuccess ? PAT_OK : PAT_EHIP;
}
