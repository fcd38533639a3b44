// Diagnostics of the launch structure: the cost of a grid-wide barrier in a
// cooperative (persistent) launch against a kernel boundary between
// back-to-back launches, in a stream and replayed from a graph.  The
// batched executor's per-pass launches rest on this comparison.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "pat_internal.h"

namespace {
namespace cg = cooperative_groups;

// per_block floats of streaming work per block, then a grid barrier
__global__ void __launch_bounds__(256) k_diag_coop(float* a, int per_block, int iters) {
  cg::grid_group g = cg::this_grid();
  for (int it = 0; it < iters; ++it) {
    float* p = a + (size_t)blockIdx.x * per_block;
    for (int i = threadIdx.x; i < per_block; i += 256) p[i] = p[i] * 0.999f + 1.0f;
    g.sync();
  }
}
// The same loop with a hand-written barrier: one device-scope atomic add per
// block on an arrival counter, the last block to arrive resets it and bumps
// a generation word that the others wait on.  Every wait is bounded: after
// kSpinLimit polls a block gives up, records it in *bad and carries on, so
// the kernel always exits (the timing is then marked invalid).
constexpr unsigned kSpinLimit = 1u << 24;
__device__ __forceinline__ void atomic_grid_barrier(unsigned* count, unsigned* gen, unsigned nblocks, int* bad) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();  // this block's writes before the arrival
    const unsigned g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived = atomicAdd(count, 1u) + 1u;
    if (arrived == nblocks) {
      __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (++spins == kSpinLimit) {
          atomicOr(bad, 1);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
  }
  __syncthreads();
}
__global__ void __launch_bounds__(256) k_diag_atomic(float* a, int per_block, int iters, unsigned* sync, int* bad) {
  for (int it = 0; it < iters; ++it) {
    float* p = a + (size_t)blockIdx.x * per_block;
    for (int i = threadIdx.x; i < per_block; i += 256) p[i] = p[i] * 0.999f + 1.0f;
    atomic_grid_barrier(sync, sync + 1, gridDim.x, bad);
  }
}
__global__ void k_diag_clear(unsigned* sync, int* bad) {
  sync[0] = 0u;
  sync[1] = 0u;
  *bad = 0;
}
__global__ void __launch_bounds__(256) k_diag_step(float* a, int per_block) {
  float* p = a + (size_t)blockIdx.x * per_block;
  for (int i = threadIdx.x; i < per_block; i += 256) p[i] = p[i] * 0.999f + 1.0f;
}

#define PAT_DTRY(x)                          \
  do {                                       \
    if ((x) != hipSuccess) {                 \
      rc = PAT_EHIP;                         \
      goto done;                             \
    }                                        \
  } while (0)

}  // namespace

extern "C" int pat_diag_sync_costs(int32_t blocks_per_cu, int32_t floats_per_block, int32_t iters,
                                   double* us_grid_barrier, double* us_atomic_barrier, double* us_stream_launch,
                                   double* us_graph_launch) {
  if (blocks_per_cu < 1 || floats_per_block < 0 || iters < 1 || iters > 100000 || !us_grid_barrier ||
      !us_atomic_barrier || !us_stream_launch || !us_graph_launch)
    return PAT_EINVAL;
  int dev = 0, ncu = 0, coop = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_diag_coop, 256, 0) != hipSuccess)
    return PAT_EHIP;
  if (!coop) return PAT_ENOSYS;
  if (blocks_per_cu > per_cu) return PAT_EINVAL;  // the grid must be co-resident
  const int nb = ncu * blocks_per_cu;
  const size_t n = (size_t)nb * (floats_per_block > 0 ? floats_per_block : 1);
  int rc = PAT_OK;
  float* a = nullptr;
  unsigned* sync = nullptr;
  int* bad = nullptr;
  int bad_h = 0;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipGraph_t gr = nullptr;
  hipGraphExec_t ge = nullptr;
  float ms = 0;
  const int reps = iters < 100 ? iters : 100;  // launches per captured graph
  int it_arg = iters, pb = floats_per_block;
  void* args[] = {&a, &pb, &it_arg};
  void* args2[] = {&a, &pb, &it_arg, &sync, &bad};
  PAT_DTRY(hipMalloc(&a, n * sizeof(float)));
  PAT_DTRY(hipMalloc(&sync, 2 * sizeof(unsigned)));
  PAT_DTRY(hipMalloc(&bad, sizeof(int)));
  PAT_DTRY(hipStreamCreate(&s));
  PAT_DTRY(hipEventCreate(&e0));
  PAT_DTRY(hipEventCreate(&e1));
  hipLaunchKernelGGL(k_diag_step, dim3(nb), dim3(256), 0, s, a, 0);
  // cooperative: iters barriers in one launch (warmed once)
  PAT_DTRY(hipLaunchCooperativeKernel((void*)k_diag_coop, dim3(nb), dim3(256), args, 0, s));
  PAT_DTRY(hipEventRecord(e0, s));
  PAT_DTRY(hipLaunchCooperativeKernel((void*)k_diag_coop, dim3(nb), dim3(256), args, 0, s));
  PAT_DTRY(hipEventRecord(e1, s));
  PAT_DTRY(hipEventSynchronize(e1));
  PAT_DTRY(hipEventElapsedTime(&ms, e0, e1));
  *us_grid_barrier = ms * 1e3 / iters;
  // the hand-written barrier, also in a cooperative launch (co-residency)
  hipLaunchKernelGGL(k_diag_clear, dim3(1), dim3(1), 0, s, sync, bad);
  PAT_DTRY(hipLaunchCooperativeKernel((void*)k_diag_atomic, dim3(nb), dim3(256), args2, 0, s));
  PAT_DTRY(hipEventRecord(e0, s));
  PAT_DTRY(hipLaunchCooperativeKernel((void*)k_diag_atomic, dim3(nb), dim3(256), args2, 0, s));
  PAT_DTRY(hipEventRecord(e1, s));
  PAT_DTRY(hipEventSynchronize(e1));
  PAT_DTRY(hipEventElapsedTime(&ms, e0, e1));
  PAT_DTRY(hipMemcpy(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost));
  *us_atomic_barrier = bad_h ? -1.0 : ms * 1e3 / iters;
  // back-to-back launches of the same work
  for (int i = 0; i < reps; ++i) hipLaunchKernelGGL(k_diag_step, dim3(nb), dim3(256), 0, s, a, floats_per_block);
  PAT_DTRY(hipEventRecord(e0, s));
  for (int i = 0; i < iters; ++i) hipLaunchKernelGGL(k_diag_step, dim3(nb), dim3(256), 0, s, a, floats_per_block);
  PAT_DTRY(hipEventRecord(e1, s));
  PAT_DTRY(hipEventSynchronize(e1));
  PAT_DTRY(hipEventElapsedTime(&ms, e0, e1));
  *us_stream_launch = ms * 1e3 / iters;
  // the same launches replayed from a graph of `reps` launches
  PAT_DTRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < reps; ++i) hipLaunchKernelGGL(k_diag_step, dim3(nb), dim3(256), 0, s, a, floats_per_block);
  PAT_DTRY(hipStreamEndCapture(s, &gr));
  PAT_DTRY(hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0));
  PAT_DTRY(hipGraphLaunch(ge, s));
  PAT_DTRY(hipEventRecord(e0, s));
  for (int i = 0; i < iters / reps; ++i) PAT_DTRY(hipGraphLaunch(ge, s));
  PAT_DTRY(hipEventRecord(e1, s));
  PAT_DTRY(hipEventSynchronize(e1));
  PAT_DTRY(hipEventElapsedTime(&ms, e0, e1));
  *us_graph_launch = ms * 1e3 / ((iters / reps) * reps);
done:
  if (s) hipStreamSynchronize(s);
  if (ge) hipGraphExecDestroy(ge);
  if (gr) hipGraphDestroy(gr);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (s) hipStreamDestroy(s);
  if (a) hipFree(a);
  if (sync) hipFree(sync);
  if (bad) hipFree(bad);
  return rc;
}
