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
__device__ __forceinline__ float2 ld2(const float* a, long i) { return reinterpret_cast<const float2*>(a)[i]; }
__device__ __forceinline__ void st2(float* a, long i, float2 v) { reinterpret_cast<float2*>(a)[i] = v; }
__device__ __forceinline__ float2 f2(float a, float b) { return make_float2(a, b); }
__device__ __forceinline__ float2 mul2(float2 a, float2 b) { return make_float2(a.x * b.x, a.y * b.y); }
__device__ __forceinline__ float2 scl2(float s, float2 a) { return make_float2(s * a.x, s * a.y); }

}  // namespace pat
