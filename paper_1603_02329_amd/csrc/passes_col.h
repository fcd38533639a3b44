// Column passes of the k-space scheme on gfx950: per tile of packed
// x-frequency columns, the FFT along y (and z), the k-space multipliers
// (staggered derivatives with the k-space correction, fractional
// Laplacians), and the inverse FFT.  See passes_row.hip for the step.
//
// Kernel templates and per-length launchers; the instances are compiled in
// two translation units (short and long axes) that build in parallel.
#pragma once

#include "passes_common.h"

namespace pat {

// TW: columns per block (0 = the default, 16 or as many as 1024 threads allow)
template <int NY, int TW = 0>
struct ColGeo {
  static constexpr int E = 8;
  static constexpr int TC = NY / E;                          // threads per column
  static constexpr int TDEF = (1024 / TC) < 16 ? (1024 / TC) : 16;
  static constexpr int TILE = TW ? TW : TDEF;
  static constexpr int NTH = TILE * TC;
  static constexpr int LD = NY + 1;                          // padded LDS column stride
  static_assert(NTH <= 1024, "column tile too wide");
};

// axis lengths with several compiled tile widths (16, 8 and 4 columns)
__host__ __device__ constexpr bool col_tunable(int na) { return na == 128 || na == 256 || na == 512; }

// ------------------------------------------------------------------ column passes
// sinc(sqrt(s)) = sum_n (-s)^n / (2n+1)!, nine terms: exact to float32
// rounding for s <= (pi/2)^2, i.e. for every time step the stability bound
// admits (c_ref dt |k|_max / 2 <= pi/2).
__device__ __forceinline__ float sinc_sqrt(float s) {
  float p = 2.8114572543455208e-15f;        // 1/17!
  p = fmaf(p, s, -7.6471637318198164e-13f);  // -1/15!
  p = fmaf(p, s, 1.6059043836821613e-10f);   // 1/13!
  p = fmaf(p, s, -2.5052108385441720e-08f);  // -1/11!
  p = fmaf(p, s, 2.7557319223985893e-06f);   // 1/9!
  p = fmaf(p, s, -1.9841269841269841e-04f);  // -1/7!
  p = fmaf(p, s, 8.3333333333333333e-03f);   // 1/5!
  p = fmaf(p, s, -1.6666666666666667e-01f);  // -1/3!
  return fmaf(p, s, 1.0f);
}


// the x-bin part of the multipliers, constant per column
struct XBin {
  float k2;
  float2 sa, sb;
};
__device__ __forceinline__ XBin xbin(const DevPlan& P, int kxi) {
  return XBin{gld(P.ksq[0], kxi), gld(P.shA[0], kxi), gld(P.shB[0], kxi)};
}

// Multiplier families of the column passes (compile-time): staggered
// derivatives a_j = i k_j kappa e^{+i k_j dx_j/2}, b_j (e^{-...}), the
// fractional Laplacians |k|^(y-2)/dt, |k|^(y-1), or the separable smoothing
// window of the initial pressure, w_x(kx) w_y(ky) [w_z(kz)].
enum ColFam : int { F_A = 0, F_B = 1, F_ABS = 2, F_WIN = 3 };

// Column pass over a tile of TILE consecutive packed x-bins and all NA points
// of one axis.
//
// Packed column 0 holds the x-bins 0 and nx/2 as C = A + iB, A and B being
// transforms of real lines.  In 2D the pass separates them with the mirror
// bin C(-ky) of the same column.  In 3D the y-transform pass (mode 3), which
// holds whole y-columns, stores column 0 unpacked -- A(ky) at 0 < ky < ny/2
// and B(ky) at ny - ky -- and the inverse y pass (mode 4) packs it again, so
// the z pass of a y-bin never needs another y-bin's column (y-bins 0 and
// ny/2 stay packed and are separated along z within their own column).
//
// Modes 0-2 transform along the last axis (y in 2D, z in 3D), apply k-space
// multipliers and transform back; modes 3/4 are the forward / inverse
// transform along y alone (3D).  Thread (t, c) with the column c fastest: a
// wavefront's loads and stores at one axis position cover TILE consecutive
// complex values (coalesced) and arrive directly in the FFT's register order
// (a = t + TC m).

// Position of one block's tile: the instance's grid, the column of this
// thread and the packed-column-0 flags.
struct ColPos {
  int M, ny, nz, stride, obase, o, kxi;
  bool along_y, ok, cvalid, tile0, selfpair, col0;
};
template <int TILE>
__device__ __forceinline__ ColPos col_pos(const DevPlan& P, int tile_index, int c, bool ypass) {
  ColPos q;
  q.M = P.n[0] / 2;
  q.ny = P.n[1];
  q.nz = P.n[2];
  q.along_y = ypass || (P.ndim == 2);
  q.stride = q.along_y ? q.M : q.ny * q.M;
  const int other_n = q.along_y ? q.nz : q.ny;
  const int tiles = (q.M + TILE - 1) / TILE;
  q.o = tile_index / tiles;
  const int kt = tile_index - q.o * tiles;
  q.ok = q.o < other_n;
  q.obase = q.along_y ? q.o * q.ny * q.M : q.o * q.M;
  const int width = q.M < TILE ? q.M : TILE;
  const int c0 = kt * TILE;
  q.cvalid = c < width;
  q.kxi = c0 + (q.cvalid ? c : 0);
  q.tile0 = (c0 == 0);                                     // tile holds packed column 0
  q.selfpair = q.along_y || q.o == 0 || 2 * q.o == q.ny;   // column 0 still packed here
  q.col0 = q.tile0 && c == 0;
  return q;
}

// loads are issued for every lane (kxi is a valid column for all) and
// zeroed for lanes past the tile's width: no branch between them
template <int NA, int TC, int E>
__device__ __forceinline__ void col_load(const float2* __restrict__ src, const ColPos& q, int t, float2 (&v)[E]) {
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const float2 x = gld(src, q.obase + (t + TC * m) * q.stride + q.kxi);
    v[m] = q.cvalid ? x : f2(0.f, 0.f);
  }
}
template <int NA, int TC, int E>
__device__ __forceinline__ void col_store(float2* __restrict__ dst, const ColPos& q, int t, const float2 (&v)[E]) {
  if (!q.cvalid) return;
#pragma unroll
  for (int m = 0; m < E; ++m) gst(dst, q.obase + (t + TC * m) * q.stride + q.kxi, v[m]);
}

// ---- modes 3 / 4: transform along y alone (3D), column 0 unpacked / packed
template <int NA, int MODE>
__global__ void __launch_bounds__((ColGeo<NA>::NTH)) k_coly(const DevPlan* __restrict__ plans,
                                                           const int2* __restrict__ table, ColSpec spec) {
  using G = ColGeo<NA>;
  constexpr int E = G::E, TC = G::TC, LD = G::LD, TILE = G::TILE;
  __shared__ float2 lds[TILE * LD];
  __shared__ Tw tws[NA];
  load_twiddles<NA, G::NTH>(tws, g_tw);
  const int2 job = table ? table[blockIdx.x] : make_int2(0, (int)blockIdx.x);
  const DevPlan& P = plans[job.x];
  const int c = threadIdx.x % TILE, t = threadIdx.x / TILE;
  const ColPos q = col_pos<TILE>(P, job.y, c, true);
  if (!q.ok) return;  // block-uniform
  float2* Lc = lds + c * LD;
  const int f = spec.f0 + (int)blockIdx.y;
  float2 v[E], vm[E];
  col_load<NA, TC>(P.S[f], q, t, v);
  __syncthreads();  // twiddles
  if constexpr (MODE == 3) {
    fft<NA, E, -1>(v, Lc, t, tws);
    if (q.tile0) {  // unpack column 0: A(a) at 0 < a < ny/2, B(ny - a) at ny/2 < a < ny
#pragma unroll
      for (int m = 0; m < E; ++m) Lc[t + TC * m] = v[m];
      __syncthreads();
#pragma unroll
      for (int m = 0; m < E; ++m) vm[m] = conjf2(Lc[(NA - (t + TC * m)) & (NA - 1)]);
      __syncthreads();
      if (c == 0) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int a = t + TC * m;
          if (a == 0 || 2 * a == NA) continue;
          if (2 * a < NA)
            v[m] = 0.5f * (v[m] + vm[m]);
          else  // (conj(Q) - conj(P)) (-i/2), P = C(a), Q = conj(C(-a))
            v[m] = 0.5f * mul_si<-1>(conjf2(vm[m]) - conjf2(v[m]));
        }
      }
    }
  } else {
    if (q.tile0) {  // pack column 0 again: C(a) = A(a) + i B(a), C(-a) = conj(A(a)) + i conj(B(a))
#pragma unroll
      for (int m = 0; m < E; ++m) Lc[t + TC * m] = v[m];
      __syncthreads();
#pragma unroll
      for (int m = 0; m < E; ++m) vm[m] = Lc[(NA - (t + TC * m)) & (NA - 1)];  // U(ny - a)
      __syncthreads();
      if (c == 0) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int a = t + TC * m;
          if (a == 0 || 2 * a == NA) continue;
          if (2 * a < NA)
            v[m] = v[m] + mul_si<+1>(vm[m]);
          else
            v[m] = conjf2(vm[m]) + mul_si<+1>(conjf2(v[m]));
        }
      }
    }
    fft<NA, E, +1>(v, Lc, t, tws);
  }
  col_store<NA, TC>(P.S[f], q, t, v);
}

// ---- modes 0-2: transform along the last axis, multipliers, transform back.
//
// Two thread mappings of one tile: for global memory the column is the
// fastest index (a wavefront's access at one axis position covers TILE
// consecutive complex values); for the transforms the TC threads of one
// column are consecutive lanes, so that (for columns of up to 512 points) a
// column lives in one wavefront and its FFT exchanges need only wavefront
// ordering, not block barriers.  Data pass between the mappings through the
// column's LDS region (padded layout, odd column stride: conflict-free).
// Every input a block needs is loaded before the first transform (up to two
// fields), so that the second field's loads overlap the first's arithmetic.
// FPB (mode 1): fields per block, taken one after another.
template <bool WAVE>
struct SyncOf {
  using type = BlockSync;
};
template <>
struct SyncOf<true> {
  using type = WaveSync;
};

// Fields a column pass transforms side by side (FftStageK): the forward and
// inverse transforms of mode 1 (FPB fields).  Modes 0 and 2 take their
// outputs / inputs one at a time: with one set of LDS regions (45 KB instead
// of 82 KB for a 512-point tile of 8 columns) their blocks fit beside the
// other group's in a batch, which outweighs the pairing (same-box A/B on the
// 48-instance batch: the adjoint 1.7 % faster with mode 2 sequential, then
// the forward 1.5 % faster with mode 0 sequential).  A two-output mode 0
// applies both multipliers before its first inverse transform, so that only
// the second product, not the spectrum and the multiplier operands, waits
// in registers through it (109 VGPRs; 137 when each output was formed just
// before its transform).  Three-field passes (3D) take their fields one at
// a time.
// Tiles whose two sets of regions would take more than 80 KB of LDS (512
// points, 16 columns) transform one field at a time.
template <int NA, int TW>
constexpr bool col_pair_fits() { return ColGeo<NA, TW>::TILE * (NA + NA / 8 - 1) * 16 <= 81920; }
template <int NA, int TW, int MODE, int NF, int FPB>
constexpr int col_kf() {
  return !col_pair_fits<NA, TW>() ? 1 : MODE == 1 ? FPB : 1;
}
template <int NA, int TW, int MODE, int NF, int FPB>
constexpr int col_ki() {
  return !col_pair_fits<NA, TW>() ? 1 : MODE == 1 ? FPB : 1;
}
template <int NA, int TW, int MODE, int NF, int FPB>
constexpr int col_k() {
  return col_kf<NA, TW, MODE, NF, FPB>() > col_ki<NA, TW, MODE, NF, FPB>() ? col_kf<NA, TW, MODE, NF, FPB>()
                                                                            : col_ki<NA, TW, MODE, NF, FPB>();
}

// The spectrum of packed column 0 (the source of its mirror bins) is kept in
// that column's own region of each set, free between the forward and the
// inverse transforms, unless a mode-0 pass needs it across several groups of
// inverse transforms (the three-output 3D gradient, which forms each product
// just before its transform): then in an array of its own.
template <int NA, int TW, int MODE, int NF, int FPB>
constexpr bool col_sep_mirror() { return MODE == 0 && NF > 2 && NF > col_ki<NA, TW, MODE, NF, FPB>(); }

// LDS of one column-pass block: K sets of the tile's column regions (padded
// exchange; the odd stride spreads the columns over the banks), the mirror
// spectrum when kept apart, and the staged twiddles.  Two sets of a 512-point
// tile of 8 columns with their twiddles take 81,776 bytes: two blocks fit
// in a compute unit's 160 KB.
template <int NA, int TW, int K = 1, bool SEPMIR = false>
struct ColLds {
  static constexpr int LDT = NA + NA / 8 - 1;            // pad8(NA - 1) + 1
  static constexpr int QS = ColGeo<NA, TW>::TILE * LDT;  // one set of regions
  static constexpr int TWL = staged_len(NA, ColGeo<NA, TW>::E);
  float2 lds[K * QS];
  float2 lmir[SEPMIR ? NA : 1];
  Tw tws[TWL > 0 ? TWL : 1];
};
template <int NA, int TW, int MODE, int NF, int FPB>
using ColLdsOf = ColLds<NA, TW, col_k<NA, TW, MODE, NF, FPB>(), col_sep_mirror<NA, TW, MODE, NF, FPB>()>;

// One column pass over tile `tile_index` of instance P (ColGeo<NA, TW>::NTH
// threads); the field of a per-field pass is blockIdx.y.
template <int NA, int MODE, int NF, int FAM, int TW, int FPB>
__device__ __forceinline__ void colm_pass(const DevPlan& P, int tile_index, const ColSpec& spec,
                                          ColLdsOf<NA, TW, MODE, NF, FPB>& sh) {
  using G = ColGeo<NA, TW>;
  constexpr int E = G::E, TC = G::TC, TILE = G::TILE;
  using Sh = ColLdsOf<NA, TW, MODE, NF, FPB>;
  constexpr int LDT = Sh::LDT, QS = Sh::QS;
  constexpr bool SEPMIR = col_sep_mirror<NA, TW, MODE, NF, FPB>();
  constexpr int KF = col_kf<NA, TW, MODE, NF, FPB>(), KI = col_ki<NA, TW, MODE, NF, FPB>();
  using Sync = typename SyncOf<(TC <= 64)>::type;
  constexpr int NIN = (MODE == 0) ? 1 : (MODE == 1 ? FPB : NF);  // input fields per block
  constexpr bool UPFRONT = NIN <= 2;
  float2* const lds = sh.lds;
  Tw* const tws = sh.tws;
  // mapping A (memory): column ca, position ta; mapping B (transforms): column cb, lane tb
  const int ca = threadIdx.x % TILE, ta = threadIdx.x / TILE;
  const int cb = threadIdx.x / TC, tb = threadIdx.x % TC;
  const ColPos qa = col_pos<TILE>(P, tile_index, ca, false);
  if (!qa.ok) return;  // block-uniform
  const ColPos q = col_pos<TILE>(P, tile_index, cb, false);
  float2* La = lds + ca * LDT;
  float2* Lb = lds + cb * LDT;
  const bool special = q.tile0 && q.selfpair;  // block holds a packed column 0 (block-uniform)
  const bool fix = q.col0 && q.selfpair;       // this lane's column is it
  // mirror spectrum of transform r: column 0's region of set r (only column
  // 0's lanes touch it between the transforms), or the separate array
  auto mir = [&](int r) -> float2* { return SEPMIR ? sh.lmir : lds + r * QS; };

  // input k of this block, output i
  const int fbase = (MODE == 1) ? spec.f0 + (int)blockIdx.y * FPB : spec.f0;
  auto in_ptr = [&](int k) -> const float2* { return MODE == 0 ? P.S[0] : P.S[fbase + k]; };
  auto out_ptr = [&](int i) -> float2* { return MODE == 0 ? P.S[1 + i] : (MODE == 1 ? P.S[fbase + i] : P.S[0]); };
  // multiplier kind of input / output i: derivative axis (F_A, F_B) or Mult kind
  auto which_of = [&](int i) { return (FAM == F_ABS || FAM == F_WIN) ? spec.mult[i] : i; };

  float2 vin[UPFRONT ? NIN : 1][E];
  if constexpr (UPFRONT) {
#pragma unroll
    for (int k = 0; k < NIN; ++k) col_load<NA, TC>(in_ptr(k), qa, ta, vin[k]);
  }

  // ---- multiplier geometry of this lane's column (mapping B)
  // bin of element m: along y (2D) ky = a; along z (3D) ky = o, kz = a.
  // Column 0 outside the self-paired y-bins holds B of y-bin ny - o at
  // x-bin nx/2 (3D unpacked layout).
  const bool unpackedB = q.col0 && !q.selfpair && 2 * q.o > q.ny;
  const int kyf = q.along_y ? 0 : (unpackedB ? q.ny - q.o : q.o);
  const XBin xb = xbin(P, unpackedB ? q.M : q.kxi);
  const XBin xbN = xbin(P, q.M);
  const float k2y = q.along_y ? 0.f : gld(P.ksq[1], kyf);
  const float k2fix = xb.k2 + k2y, k2fixN = xbN.k2 + k2y;
  const int ax_last = q.along_y ? 1 : 2;
  // Every operand of the multipliers is read, and the per-element factors
  // formed, here, before the transforms: their loads then overlap the input
  // loads.  Read where they are used, after the forward transform, each
  // table load's latency would stall the block (the LDS barriers keep the
  // compiler from hoisting them).
  const float kap2 = P.kap2, scale = P.scale, ym2h = P.ym2h, ym1h = P.ym1h, inv_dt = P.inv_dt;
  constexpr bool DERIV = (FAM == F_A || FAM == F_B), SA = (FAM != F_B);
  auto k2at = [&](int m) { return gld(P.ksq[ax_last], tb + TC * m); };
  // derivatives: kappa/N at this column's elements, the staggered shift along
  // the transform axis, and (3D, along z) the y shift of this column;
  // Laplacians: |k|^2 along the axis
  float gv[(DERIV || FAM == F_ABS) ? E : 1];
  float2 shv[DERIV ? E : 1];
  float2 shyf = f2(0.f, 0.f);
  if constexpr (DERIV) {
    const float2* sht = SA ? P.shA[ax_last] : P.shB[ax_last];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      shv[m] = gld(sht, tb + TC * m);
      gv[m] = sinc_sqrt(kap2 * (k2fix + k2at(m))) * scale;
    }
    if (!q.along_y) shyf = gld(SA ? P.shA[1] : P.shB[1], kyf);
  } else if constexpr (FAM == F_ABS) {
    // log2 |k|^2 (-inf at k = 0, where both Laplacians vanish)
#pragma unroll
    for (int m = 0; m < E; ++m) gv[m] = __builtin_amdgcn_logf(k2fix + k2at(m));
  }
  // window family: the x (and, along z, the y) factor of this column, the
  // x factor at x-bin nx/2 for the packed column 0, and the along-axis one
  float wfix = 1.f, wfixN = 1.f, wv[E];
  if constexpr (FAM == F_WIN) {
    const float wy = q.along_y ? 1.f : gld(P.win[1], kyf);
    wfix = gld(P.win[0], unpackedB ? q.M : q.kxi) * wy * scale;
    wfixN = gld(P.win[0], q.M) * wy * scale;
#pragma unroll
    for (int m = 0; m < E; ++m) wv[m] = gld(P.win[ax_last], tb + TC * m);
  }
  // the staged twiddles, after the block's own loads (first read after the
  // barrier that ends the first transform's first stage)
  load_table<Sh::TWL, G::NTH>(tws, g_tw, [](int i) { return staged_src<NA, E>(i); });
  // Laplacian factor |k|^(2e) = exp2(e log2 |k|^2), e = (y-2)/2 or (y-1)/2,
  // times 1/dt for L1, from lk = log2 |k|^2: the absorption terms are small
  // corrections, so the hardware log2/exp2 suffice
  auto lapl = [&](float lk, int which) -> float {
    const float e = which == M_L1DT ? ym2h : ym1h;
    const float v = lk > -INFINITY ? __builtin_amdgcn_exp2f(e * lk) : 0.f;
    return (which == M_L1DT ? v * inv_dt : v) * scale;
  };
  // staggered shift of derivative axis `axis` at element m, for this
  // column's x-bin (nyq: at x-bin nx/2)
  auto shift = [&](int axis, int m, bool nyq) -> float2 {
    if (axis == 0) return nyq ? (SA ? xbN.sa : xbN.sb) : (SA ? xb.sa : xb.sb);
    if (axis == 1 && !q.along_y) return shyf;
    return shv[DERIV ? m : 0];
  };
  // multiplier of element m (nyq: at x-bin nx/2, for the packed column 0)
  auto mult = [&](int which, int m, bool nyq) -> float2 {
    if constexpr (FAM == F_WIN) {
      return f2((nyq ? wfixN : wfix) * wv[m], 0.f);
    } else if constexpr (FAM == F_ABS) {
      return f2(lapl(nyq ? __builtin_amdgcn_logf(k2fixN + k2at(m)) : gv[m], which), 0.f);
    } else {
      const float g = nyq ? sinc_sqrt(kap2 * (k2fixN + k2at(m))) * scale : gv[m];
      return scl2(g, shift(which, m, nyq));
    }
  };
  // acc += mult * s.  The packed column 0 holds C = A + iB (x-bins 0 and
  // nx/2): there the product is 1/2 (m0 + mN) C + 1/2 (m0 - mN) conj(C(-k)),
  // with the mirror bins read from the spectrum of transform r in LDS.
  auto apply = [&](int which, const float2 (&s)[E], float2 (&acc)[E], int r) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const float2 mv = mult(which, m, false);
      if (fix) {
        const float2 mN = mult(which, m, true);
        const float2 vm = conjf2(mir(r)[(NA - (tb + TC * m)) & (NA - 1)]);
        acc[m] = acc[m] + cmul(0.5f * (mv + mN), s[m]) + cmul(0.5f * (mv - mN), vm);
      } else {
        acc[m] = acc[m] + cmul(mv, s[m]);
      }
    }
  };
  // Forward transforms of K inputs side by side (mapping A in, spectra in
  // mapping B out): the first stage runs in mapping A, where each thread
  // already holds the eight values of its butterfly, and its exchange
  // carries the values over to mapping B; a block holding column 0 keeps
  // that column's spectra in LDS for their mirror bins.  v is overwritten.
  // The block's first transform finds the regions unused and skips the
  // barrier that waits for their earlier readers.
  auto forward = [&](auto& v, auto& s, bool first) {
    constexpr int K = sizeof(v) / sizeof(v[0]);
    if (!first) __syncthreads();  // earlier readers of the regions are done
    fft_head_k<K, QS, NA, E, -1, TwStaged, true>(v, La, ta);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
      for (int m = 0; m < E; ++m) s[r][m] = Lb[r * QS + pad8(tb + TC * m)];
    Sync::sync();  // the transforms reuse the regions
    fft_tail_k<K, QS, NA, E, -1, Sync, TwStaged, true>(s, Lb, tb, tws);
    if (special) {
      if (fix) {
#pragma unroll
        for (int r = 0; r < K; ++r)
#pragma unroll
          for (int m = 0; m < E; ++m) mir(r)[tb + TC * m] = s[r][m];
      }
      Sync::sync();
    }
  };
  // Inverse transforms of K outputs side by side (mapping B in) and their
  // stores (mapping A): every stage but the last in mapping B, whose final
  // exchange carries the values over to mapping A for the last stage.
  // After the block's last transform no barrier releases the regions.
  auto inverse_store = [&](auto& acc, auto dst, bool last) {
    constexpr int K = sizeof(acc) / sizeof(acc[0]);
    if (!SEPMIR && special) Sync::sync();  // the mirror reads precede the region's reuse
    fft_body_k<K, QS, NA, E, +1, Sync, TwStaged, true>(acc, Lb, tb, tws);
    __syncthreads();
    float2 v[K][E];
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
      for (int m = 0; m < E; ++m) v[r][m] = La[r * QS + pad8(ta + TC * m)];
    if (!last) __syncthreads();  // the regions are free for the next transform
    fft_last_k<K, QS, NA, E, +1, TwStaged, true>(v, ta, tws);
#pragma unroll
    for (int r = 0; r < K; ++r) col_store<NA, TC>(dst(r), qa, ta, v[r]);
  };

  // inputs k .. k + KF - 1 of the block, from the up-front loads or loaded now
  auto take = [&](int k, float2 (&v)[KF][E]) {
#pragma unroll
    for (int r = 0; r < KF; ++r) {
      if constexpr (UPFRONT) {
#pragma unroll
        for (int m = 0; m < E; ++m) v[r][m] = vin[k + r][m];
      } else {
        col_load<NA, TC>(in_ptr(k + r), qa, ta, v[r]);
      }
    }
  };

  if constexpr (MODE == 2) {
    // NF inputs, KF at a time, summed into one output
    float2 acc[1][E];
#pragma unroll
    for (int m = 0; m < E; ++m) acc[0][m] = f2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < NF; k += KF) {
      float2 v[KF][E], s[KF][E];
      take(k, v);
      forward(v, s, k == 0);
#pragma unroll
      for (int r = 0; r < KF; ++r) apply(which_of(k + r), s[r], acc[0], r);
    }
    inverse_store(acc, [&](int) { return out_ptr(0); }, true);
  } else if constexpr (MODE == 1) {
    // FPB fields, each to its own output, KF side by side
#pragma unroll
    for (int k = 0; k < FPB; k += KF) {
      float2 v[KF][E], s[KF][E];
      take(k, v);
      forward(v, s, k == 0);
      float2 acc[KF][E];
#pragma unroll
      for (int r = 0; r < KF; ++r) {
#pragma unroll
        for (int m = 0; m < E; ++m) acc[r][m] = f2(0.f, 0.f);
        apply(which_of((int)blockIdx.y * FPB + k + r), s[r], acc[r], r);
      }
      inverse_store(acc, [&](int r) { return out_ptr(k + r); }, k + KF >= FPB);
    }
  } else {
    // mode 0: one input, NF outputs, KI at a time
    float2 v[1][E], s[1][E];
    take(0, v);
    forward(v, s, true);
    if constexpr (NF == 2 && KI == 1) {  // both products first, then the two inverse transforms
      float2 acc[2][1][E];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int m = 0; m < E; ++m) acc[i][0][m] = f2(0.f, 0.f);
        apply(which_of(i), s[0], acc[i][0], 0);
      }
      inverse_store(acc[0], [&](int) { return out_ptr(0); }, false);
      inverse_store(acc[1], [&](int) { return out_ptr(1); }, true);
      return;
    }
#pragma unroll
    for (int i = 0; i < NF; i += KI) {
      float2 acc[KI][E];
#pragma unroll
      for (int r = 0; r < KI; ++r) {
#pragma unroll
        for (int m = 0; m < E; ++m) acc[r][m] = f2(0.f, 0.f);
        apply(which_of(i + r), s[0], acc[r], 0);
      }
      inverse_store(acc, [&](int r) { return out_ptr(i + r); }, i + KI >= NF);
    }
  }
}

template <int NA, int MODE, int NF, int FAM, int TW, int FPB>
__global__ void __launch_bounds__((ColGeo<NA, TW>::NTH)) k_colm(const DevPlan* __restrict__ plans,
                                                               const int2* __restrict__ table, ColSpec spec) {
  __shared__ ColLdsOf<NA, TW, MODE, NF, FPB> sh;
  const int2 job = table ? table[blockIdx.x] : make_int2(0, (int)blockIdx.x);
  colm_pass<NA, MODE, NF, FAM, TW, FPB>(plans[job.x], job.y, spec, sh);
}

// multiplier family from the kinds: derivatives a_j / b_j listed in axis
// order, or the two fractional Laplacians
inline int col_family(const ColSpec& spec) {
  if (spec.mult[0] == M_WIN) return F_WIN;
  if (spec.mult[0] == M_L1DT || spec.mult[0] == M_L2) return F_ABS;
  return (spec.mult[0] >= M_BX) ? F_B : F_A;
}

template <int NA, int TW, int FPB>
hipError_t launch_colm(const ColSpec& spec, const Launch& L) {
  const dim3 block(ColGeo<NA, TW>::NTH);
  const int fam = col_family(spec);
#define PAT_COLM(MODE, NF, FAMV, GY)                                                                         \
  hipExtLaunchKernelGGL((k_colm<NA, MODE, NF, FAMV, TW, FPB>), dim3(L.nblocks, GY), block, 0, L.stream, L.ev0, \
                        L.ev1, 0, L.plans, L.table, spec)
#define PAT_COLM_FAM(MODE, NF, GY)                      \
  do {                                                  \
    if (fam == F_A) PAT_COLM(MODE, NF, F_A, GY);        \
    else if (fam == F_B) PAT_COLM(MODE, NF, F_B, GY);   \
    else PAT_COLM(MODE, NF, F_ABS, GY);                 \
  } while (0)
  if (fam == F_WIN) {  // the smoothing window: one field, mode 1
    if constexpr (FPB == 1) {
      if (spec.mode != 1 || spec.nfield != 1) return hipErrorInvalidValue;
      PAT_COLM(1, 1, F_WIN, 1);
    } else {
      return hipErrorInvalidValue;
    }
  } else if constexpr (FPB != 1) {
    if (spec.mode != 1 || spec.nfield != FPB) return hipErrorInvalidValue;
    PAT_COLM_FAM(1, FPB, 1);
  } else if (spec.mode == 1) {
    PAT_COLM_FAM(1, 1, spec.nfield);
  } else if (spec.mode == 0 || spec.mode == 2) {
    if (spec.nfield == 2) {
      if (spec.mode == 0) PAT_COLM_FAM(0, 2, 1);
      else PAT_COLM_FAM(2, 2, 1);
    } else if (spec.nfield == 3) {
      if constexpr (TW == 0) {
        if (spec.mode == 0) PAT_COLM_FAM(0, 3, 1);
        else PAT_COLM_FAM(2, 3, 1);
      } else {
        return hipErrorInvalidValue;
      }
    } else {
      return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
  }
#undef PAT_COLM_FAM
#undef PAT_COLM
  return hipGetLastError();
}

// one column pass of axis length NA in variant (tile, fpb)
template <int NA>
hipError_t launch_col_na(const ColSpec& spec, ColVariant v, const Launch& L) {
  if (spec.mode == 3 || spec.mode == 4) {
    if (v.tile != ColGeo<NA>::TILE || v.fpb != 1) return hipErrorInvalidValue;
    const dim3 grid(L.nblocks, spec.nfield), block(ColGeo<NA>::NTH);
    if (spec.mode == 3)
      hipExtLaunchKernelGGL((k_coly<NA, 3>), grid, block, 0, L.stream, L.ev0, L.ev1, 0, L.plans, L.table, spec);
    else
      hipExtLaunchKernelGGL((k_coly<NA, 4>), grid, block, 0, L.stream, L.ev0, L.ev1, 0, L.plans, L.table, spec);
    return hipGetLastError();
  }
  if (v.fpb != 1 && v.fpb != 2) return hipErrorInvalidValue;
  if constexpr (col_tunable(NA)) {
    if (v.tile == ColGeo<NA>::TILE) return v.fpb == 1 ? launch_colm<NA, 0, 1>(spec, L) : launch_colm<NA, 0, 2>(spec, L);
    if (v.tile == 8) return v.fpb == 1 ? launch_colm<NA, 8, 1>(spec, L) : launch_colm<NA, 8, 2>(spec, L);
    if (v.tile == 4) return v.fpb == 1 ? launch_colm<NA, 4, 1>(spec, L) : launch_colm<NA, 4, 2>(spec, L);
  } else {
    if (v.tile == ColGeo<NA>::TILE && v.fpb == 1) return launch_colm<NA, 0, 1>(spec, L);
  }
  return hipErrorInvalidValue;
}

}  // namespace pat
