// Device helpers shared by the row and column passes of the k-space scheme.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fft.h"
#include "pat_internal.h"

namespace pat {

// twiddle table exp(-2 pi i q / TWN) as hi/lo pairs; one copy per
// translation unit, uploaded by that unit's upload function
static __device__ Tw g_tw[TWN];

// ------------------------------------------------------------------ helpers
// Accesses to device memory through the global address space.  The arrays
// reach the kernels as generic pointers inside the plan records; addressed
// generically, a load or store becomes a flat instruction, which the wait
// counters track together with the LDS operations, so every LDS wait of a
// transform would also wait for all loads and stores still in flight.
// (The host pass of the compiler only parses these bodies.)
template <class T>
__device__ __forceinline__ T gld(const T* p, long i) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(1))) T*)p)[i];
#else
  return p[i];
#endif
}
template <class T>
__device__ __forceinline__ void gst(T* p, long i, T v) {
#if defined(__HIP_DEVICE_COMPILE__)
  ((__attribute__((address_space(1))) T*)p)[i] = v;
#else
  p[i] = v;
#endif
}
__device__ __forceinline__ float2 ld2(const float* a, long i) { return gld(reinterpret_cast<const float2*>(a), i); }
__device__ __forceinline__ void st2(float* a, long i, float2 v) { gst(reinterpret_cast<float2*>(a), i, v); }
__device__ __forceinline__ float2 f2(float a, float b) { return make_float2(a, b); }
__device__ __forceinline__ float2 mul2(float2 a, float2 b) { return make_float2(a.x * b.x, a.y * b.y); }
__device__ __forceinline__ float2 scl2(float s, float2 a) { return make_float2(s * a.x, s * a.y); }

}  // namespace pat
