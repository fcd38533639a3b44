// Register/LDS Stockham FFT for gfx950.
//
// One transform of length M is carried by T = M / E threads, each holding E
// complex values in registers.  Thread t owns the elements at indices
// t + T*m (m = 0..E-1) both on entry (time/space order) and on exit
// (natural frequency order): consecutive lanes touch consecutive elements,
// so loads and stores to global memory coalesce.  Each stage is a radix-R
// butterfly (R = E, or smaller for the last stage) in registers; between
// stages the values pass through the transform's LDS region in Stockham
// (self-sorting) order.
//
// Twiddles come from a table of exp(-2 pi i q / TWN) held as hi + lo float
// pairs, and the radix-8 constant sqrt(1/2) likewise: the product x*w is
// formed as x*w_hi + x*w_lo, so the table's float32 rounding -- a fixed,
// systematic perturbation of the DFT that would otherwise accumulate over
// thousands of time steps -- is removed.  Only the arithmetic rounding of
// the butterflies remains.
#pragma once

#include <hip/hip_runtime.h>

#include "pat_internal.h"

namespace pat {

__device__ __forceinline__ float2 operator+(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 operator-(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 operator*(float s, float2 a) { return make_float2(s * a.x, s * a.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// x * (w_hi + w_lo) for the table twiddle w (SIGN < 0) or its conjugate (SIGN > 0)
template <int SIGN>
__device__ __forceinline__ float2 twmul(float2 x, const Tw w) {
  const float wr = w.hr, wi = (SIGN < 0) ? w.hi : -w.hi;
  const float lr = w.lr, li = (SIGN < 0) ? w.li : -w.li;
  const float tr = x.x * lr - x.y * li;
  const float ti = x.x * li + x.y * lr;
  return make_float2(fmaf(x.x, wr, fmaf(-x.y, wi, tr)), fmaf(x.x, wi, fmaf(x.y, wr, ti)));
}

// x * (SIGN i)
template <int SIGN>
__device__ __forceinline__ float2 mul_si(float2 x) {
  return (SIGN < 0) ? make_float2(x.y, -x.x) : make_float2(-x.y, x.x);
}

// sqrt(1/2) = S8H + S8L
constexpr float S8H = 0.70710676908493042f;
constexpr float S8L = 1.2101617485882343e-08f;
__device__ __forceinline__ float mul_s8(float v) { return fmaf(v, S8H, v * S8L); }

// x * exp(SIGN i pi/4) and x * exp(SIGN 3 i pi/4)
template <int SIGN>
__device__ __forceinline__ float2 mul_w8(float2 x) {
  return (SIGN < 0) ? make_float2(mul_s8(x.x + x.y), mul_s8(x.y - x.x))
                    : make_float2(mul_s8(x.x - x.y), mul_s8(x.y + x.x));
}
template <int SIGN>
__device__ __forceinline__ float2 mul_w83(float2 x) {
  return (SIGN < 0) ? make_float2(mul_s8(x.y - x.x), mul_s8(-x.x - x.y))
                    : make_float2(mul_s8(-x.x - x.y), mul_s8(x.x - x.y));
}

template <int R, int SIGN>
struct Dft;

template <int SIGN>
struct Dft<1, SIGN> {
  __device__ __forceinline__ static void run(float2*) {}
};

template <int SIGN>
struct Dft<2, SIGN> {
  __device__ __forceinline__ static void run(float2* x) {
    const float2 a = x[0];
    x[0] = a + x[1];
    x[1] = a - x[1];
  }
};

template <int SIGN>
struct Dft<4, SIGN> {
  __device__ __forceinline__ static void run(float2* x) {
    const float2 c0 = x[0] + x[2], c1 = x[0] - x[2];
    const float2 c2 = x[1] + x[3], c3 = mul_si<SIGN>(x[1] - x[3]);
    x[0] = c0 + c2;
    x[2] = c0 - c2;
    x[1] = c1 + c3;
    x[3] = c1 - c3;
  }
};

template <int SIGN>
struct Dft<8, SIGN> {
  __device__ __forceinline__ static void run(float2* x) {
    float2 a[4], b[4];
    a[0] = x[0] + x[4];
    b[0] = x[0] - x[4];
    a[1] = x[1] + x[5];
    b[1] = mul_w8<SIGN>(x[1] - x[5]);
    a[2] = x[2] + x[6];
    b[2] = mul_si<SIGN>(x[2] - x[6]);
    a[3] = x[3] + x[7];
    b[3] = mul_w83<SIGN>(x[3] - x[7]);
    Dft<4, SIGN>::run(a);
    Dft<4, SIGN>::run(b);
    x[0] = a[0];
    x[2] = a[1];
    x[4] = a[2];
    x[6] = a[3];
    x[1] = b[0];
    x[3] = b[1];
    x[5] = b[2];
    x[7] = b[3];
  }
};

// Barrier flavours between Stockham stages: the whole block, or only the
// wavefront (when every thread of a transform lives in the same wavefront,
// the LDS exchange needs no block-wide barrier, only ordering of this
// wavefront's LDS accesses).
struct BlockSync {
  __device__ __forceinline__ static void sync() { __syncthreads(); }
};
struct WaveSync {
  __device__ __forceinline__ static void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

// Twiddle layouts of a transform:
//   TwStrided   one table tw[q] = exp(-2 pi i q / TL), TL = TWS * M; stage
//               (L, R) reads tw[(i j) TL / (L R)].  Suited to the column
//               passes, where the lanes of a wavefront share j (broadcast).
//   TwStaged    per stage (L, R) a table of (R - 1) L entries, entry
//               [(i - 1) L + j] = exp(-2 pi i (i j) / (L R)), the stages one
//               after another: lanes with consecutive j read consecutive
//               entries (no LDS bank conflicts in the row passes, where
//               consecutive lanes carry consecutive j).
// Exchange layouts: plain (element a at a) or padded (at a + a / 8): the
// padded layout spreads the radix-8 write patterns (stride 8 and blocks of 8
// at stride 64) over all LDS banks; the region then needs M + M / 8 slots.
enum TwLayout : int { TwStrided = 0, TwStaged = 1 };

__host__ __device__ constexpr int fft_radix(int M, int E, int L) { return (M / L) < E ? (M / L) : E; }
// offset of stage L's entries in a TwStaged table, and the table's length
__host__ __device__ constexpr int staged_off(int M, int E, int L) {
  int off = 0;
  for (int l = 1; l < L; l *= fft_radix(M, E, l)) off += (fft_radix(M, E, l) - 1) * l;
  return off;
}
__host__ __device__ constexpr int staged_len(int M, int E) { return staged_off(M, E, M); }
__device__ __forceinline__ constexpr int pad8(int a) { return a + (a >> 3); }

// One Stockham stage of span L (product of the radices already applied).
// TWS: TwStrided table length TWS * M (1 or 2); PAD: padded exchange layout;
// STOP: the span at which to stop -- the stage that reaches it writes its
// values to the exchange region and returns before any barrier (M: run to
// the end, the last stage leaving its values in registers).
template <int M, int E, int SIGN, int L, class Sync, int TWS, int LAY = TwStrided, bool PAD = false, int STOP = M>
struct FftStage {
  static constexpr int T = M / E;
  static constexpr int R = fft_radix(M, E, L);
  static constexpr int NB = E / R;
  static constexpr bool LAST = (L * R == M);

  __device__ __forceinline__ static int at(int a) { return PAD ? pad8(a) : a; }

  __device__ __forceinline__ static void run(float2 (&v)[E], float2* lds, int t, const Tw* tw) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int k = t + T * b;
      const int j = k & (L - 1);
      float2 x[R];
#pragma unroll
      for (int i = 0; i < R; ++i) x[i] = v[b + i * NB];
      if constexpr (L > 1) {
#pragma unroll
        for (int i = 1; i < R; ++i) {
          if constexpr (LAY == TwStaged)
            x[i] = twmul<SIGN>(x[i], tw[staged_off(M, E, L) + (i - 1) * L + j]);
          else
            x[i] = twmul<SIGN>(x[i], tw[(i * j) * (TWS * M / (L * R))]);
        }
      }
      Dft<R, SIGN>::run(x);
      if constexpr (LAST) {
#pragma unroll
        for (int i = 0; i < R; ++i) v[b + i * NB] = x[i];
      } else {
        const int base = (k - j) * R + j;
#pragma unroll
        for (int i = 0; i < R; ++i) lds[at(base + i * L)] = x[i];
      }
    }
    if constexpr (!LAST && L * R != STOP) {
      Sync::sync();
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = lds[at(t + T * m)];
      Sync::sync();
      FftStage<M, E, SIGN, L * R, Sync, TWS, LAY, PAD, STOP>::run(v, lds, t, tw);
    }
  }
};

// Unnormalised DFT of length M (SIGN = -1 forward, +1 inverse) of the values
// v[m] = x[t + T m] held by the T threads of one transform; `lds` is that
// transform's region of M complex values (M + M / 8 when PAD) and `tw` its
// twiddle table in layout LAY.  With BlockSync every thread of the block
// must call it.
template <int M, int E, int SIGN, class Sync = BlockSync, int TWS = 1, int LAY = TwStrided, bool PAD = false>
__device__ __forceinline__ void fft(float2 (&v)[E], float2* lds, int t, const Tw* tw) {
  static_assert((M & (M - 1)) == 0 && M >= E && M <= TWN, "unsupported FFT length");
  FftStage<M, E, SIGN, 1, Sync, TWS, LAY, PAD>::run(v, lds, t, tw);
}

// The same transform in pieces, for callers that hold a transform's values
// in different threads at its two ends (the column passes load and store
// with the column fastest across lanes, but transform with a column's lanes
// consecutive): each piece ends with its values written to, or starts with
// them read from, the exchange region at t + T m, and the caller places the
// barrier between the two thread mappings.
__host__ __device__ constexpr int fft_last_span(int M, int E) {
  int L = 1;
  while (L * fft_radix(M, E, L) < M) L *= fft_radix(M, E, L);
  return L;
}
// first stage: butterflies of the thread's values, written to the region
template <int M, int E, int SIGN, int LAY, bool PAD>
__device__ __forceinline__ void fft_head(float2 (&v)[E], float2* lds, int t) {
  static_assert(fft_radix(M, E, 1) < M, "the transform has a single stage");
  FftStage<M, E, SIGN, 1, WaveSync, 1, LAY, PAD, fft_radix(M, E, 1)>::run(v, lds, t, nullptr);
}
// the stages after the first, on values read at t + T m of its output
template <int M, int E, int SIGN, class Sync, int LAY, bool PAD>
__device__ __forceinline__ void fft_tail(float2 (&v)[E], float2* lds, int t, const Tw* tw) {
  FftStage<M, E, SIGN, fft_radix(M, E, 1), Sync, 1, LAY, PAD>::run(v, lds, t, tw);
}
// every stage but the last: the last exchange's values are left in the region
template <int M, int E, int SIGN, class Sync, int LAY, bool PAD>
__device__ __forceinline__ void fft_body(float2 (&v)[E], float2* lds, int t, const Tw* tw) {
  static_assert(fft_radix(M, E, 1) < M, "the transform has a single stage");
  FftStage<M, E, SIGN, 1, Sync, 1, LAY, PAD, fft_last_span(M, E)>::run(v, lds, t, tw);
}
// the last stage, on values read at t + T m of the region (no LDS access)
template <int M, int E, int SIGN, int LAY, bool PAD>
__device__ __forceinline__ void fft_last(float2 (&v)[E], int t, const Tw* tw) {
  FftStage<M, E, SIGN, fft_last_span(M, E), WaveSync, 1, LAY, PAD>::run(v, nullptr, t, tw);
}

// K transforms of length M carried by the same threads, stage by stage
// (column passes with several fields): the K butterflies of a stage share
// its twiddles, the K exchanges share its barriers, and the K independent
// instruction streams hide each other's LDS and arithmetic latency.
// Transform q exchanges through the region at lds + q * QS; otherwise as
// FftStage (staged or strided twiddles with TWS = 1).
template <int K, int QS, int M, int E, int SIGN, int L, class Sync, int LAY, bool PAD, int STOP = M>
struct FftStageK {
  static constexpr int T = M / E;
  static constexpr int R = fft_radix(M, E, L);
  static constexpr int NB = E / R;
  static constexpr bool LAST = (L * R == M);

  __device__ __forceinline__ static int at(int a) { return PAD ? pad8(a) : a; }

  __device__ __forceinline__ static void run(float2 (&v)[K][E], float2* lds, int t, const Tw* tw) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int k = t + T * b;
      const int j = k & (L - 1);
      float2 x[K][R];
#pragma unroll
      for (int q = 0; q < K; ++q)
#pragma unroll
        for (int i = 0; i < R; ++i) x[q][i] = v[q][b + i * NB];
      if constexpr (L > 1) {
#pragma unroll
        for (int i = 1; i < R; ++i) {
          const Tw w = (LAY == TwStaged) ? tw[staged_off(M, E, L) + (i - 1) * L + j] : tw[(i * j) * (M / (L * R))];
#pragma unroll
          for (int q = 0; q < K; ++q) x[q][i] = twmul<SIGN>(x[q][i], w);
        }
      }
#pragma unroll
      for (int q = 0; q < K; ++q) Dft<R, SIGN>::run(x[q]);
      if constexpr (LAST) {
#pragma unroll
        for (int q = 0; q < K; ++q)
#pragma unroll
          for (int i = 0; i < R; ++i) v[q][b + i * NB] = x[q][i];
      } else {
        const int base = (k - j) * R + j;
#pragma unroll
        for (int q = 0; q < K; ++q)
#pragma unroll
          for (int i = 0; i < R; ++i) lds[q * QS + at(base + i * L)] = x[q][i];
      }
    }
    if constexpr (!LAST && L * R != STOP) {
      Sync::sync();
#pragma unroll
      for (int q = 0; q < K; ++q)
#pragma unroll
        for (int m = 0; m < E; ++m) v[q][m] = lds[q * QS + at(t + T * m)];
      Sync::sync();
      FftStageK<K, QS, M, E, SIGN, L * R, Sync, LAY, PAD, STOP>::run(v, lds, t, tw);
    }
  }
};
// the pieces of fft_head / fft_tail / fft_body / fft_last for K transforms
template <int K, int QS, int M, int E, int SIGN, int LAY, bool PAD>
__device__ __forceinline__ void fft_head_k(float2 (&v)[K][E], float2* lds, int t) {
  static_assert(fft_radix(M, E, 1) < M, "the transform has a single stage");
  FftStageK<K, QS, M, E, SIGN, 1, WaveSync, LAY, PAD, fft_radix(M, E, 1)>::run(v, lds, t, nullptr);
}
template <int K, int QS, int M, int E, int SIGN, class Sync, int LAY, bool PAD>
__device__ __forceinline__ void fft_tail_k(float2 (&v)[K][E], float2* lds, int t, const Tw* tw) {
  FftStageK<K, QS, M, E, SIGN, fft_radix(M, E, 1), Sync, LAY, PAD>::run(v, lds, t, tw);
}
template <int K, int QS, int M, int E, int SIGN, class Sync, int LAY, bool PAD>
__device__ __forceinline__ void fft_body_k(float2 (&v)[K][E], float2* lds, int t, const Tw* tw) {
  static_assert(fft_radix(M, E, 1) < M, "the transform has a single stage");
  FftStageK<K, QS, M, E, SIGN, 1, Sync, LAY, PAD, fft_last_span(M, E)>::run(v, lds, t, tw);
}
template <int K, int QS, int M, int E, int SIGN, int LAY, bool PAD>
__device__ __forceinline__ void fft_last_k(float2 (&v)[K][E], int t, const Tw* tw) {
  FftStageK<K, QS, M, E, SIGN, fft_last_span(M, E), WaveSync, LAY, PAD>::run(v, nullptr, t, tw);
}

// Source in the global length-TWN table of entry q of a TwStaged table for
// transforms of length M (E values per thread), q counted from stage L's
// first entry.  The entries of the first stage (L = 1) are exp(0) = 1.
template <int M, int E, int L = 1>
__device__ __forceinline__ int staged_src(int q) {
  constexpr int R = fft_radix(M, E, L);
  if constexpr (L * R < M) {
    if (q >= (R - 1) * L) return staged_src<M, E, L * R>(q - (R - 1) * L);
  }
  static_assert(TWN % (L * R) == 0, "stage longer than the global table");
  return ((q / L + 1) * (q % L)) * (TWN / (L * R));
}

// Copy NTOT entries from the global table into an LDS table, entry q from
// g[src(q)], NTH threads taking part.  Each thread issues all its global
// loads before its first LDS write, so the table costs one memory round
// trip.  Called after a pass has issued its own loads, it overlaps them.
template <int NTOT, int NTH, class Src>
__device__ __forceinline__ void load_table(Tw* dst, const Tw* __restrict__ g, Src src) {
  constexpr int PER = (NTOT + NTH - 1) / NTH;
  Tw v[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int q = (int)threadIdx.x + NTH * r;
    v[r] = g[src(q < NTOT ? q : NTOT - 1)];
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int q = (int)threadIdx.x + NTH * r;
    if (q < NTOT) dst[q] = v[r];
  }
}

// Copy the length-TL twiddle table (from the global length-TWN one) into LDS.
template <int TL, int NTH>
__device__ __forceinline__ void load_twiddles(Tw* dst, const Tw* __restrict__ g) {
  static_assert(TWN % TL == 0, "table length must divide TWN");
  for (int q = threadIdx.x; q < TL; q += NTH) dst[q] = g[q * (TWN / TL)];
}

}  // namespace pat
