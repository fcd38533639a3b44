// Column passes of the k-space scheme on gfx950: per tile of packed
// x-frequency columns, the FFT along y (and z), the k-space multipliers
// (staggered derivatives with the k-space correction, fractional
// Laplacians), and the inverse FFT.  See passes_row.hip for the step.
#include <algorithm>

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

// |k|^(2e) from |k|^2 (e = (y-2)/2 or (y-1)/2): the absorption terms are
// small corrections, so the hardware log2/exp2 suffice.
__device__ __forceinline__ float kpow(float k2, float e) {
  return k2 > 0.f ? __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(k2)) : 0.f;
}

// the x-bin part of the multipliers, constant per column
struct XBin {
  float k2;
  float2 sa, sb;
};
__device__ __forceinline__ XBin xbin(const DevPlan& P, int kxi) {
  return XBin{P.ksq[0][kxi], P.shA[0][kxi], P.shB[0][kxi]};
}

// Multiplier families of the column passes (compile-time): staggered
// derivatives a_j = i k_j kappa e^{+i k_j dx_j/2}, b_j (e^{-...}), or the
// fractional Laplacians |k|^(y-2)/dt, |k|^(y-1).
enum ColFam : int { F_A = 0, F_B = 1, F_ABS = 2 };

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
template <int NA, int MODE, int NF, int FAM, int TW>
__global__ void __launch_bounds__((ColGeo<NA, TW>::NTH)) k_col(const DevPlan* __restrict__ plans,
                                                             const int2* __restrict__ table, ColSpec spec) {
  using G = ColGeo<NA, TW>;
  constexpr int E = G::E, TC = G::TC, LD = G::LD, TILE = G::TILE;
  __shared__ float2 lds[TILE * LD];
  __shared__ Tw tws[NA];
  load_twiddles<NA, G::NTH>(tws, g_tw);
  const int2 job = table ? table[blockIdx.x] : make_int2(0, (int)blockIdx.x);
  const DevPlan& P = plans[job.x];
  const int M = P.n[0] / 2, ny = P.n[1], nz = P.n[2];
  const bool along_y = (MODE >= 3) || (P.ndim == 2);
  const int stride = along_y ? M : ny * M;
  const int other_n = along_y ? nz : ny;
  const int tiles = (M + TILE - 1) / TILE;
  const int o = job.y / tiles, kt = job.y - o * tiles;
  if (o >= other_n) return;  // block-uniform
  const int obase = along_y ? o * ny * M : o * M;
  const int width = M < TILE ? M : TILE;
  const int c0 = kt * TILE;
  const int c = threadIdx.x % TILE, t = threadIdx.x / TILE;
  float2* Lc = lds + c * LD;
  const bool cvalid = c < width;
  const int kxi = c0 + (cvalid ? c : 0);
  const bool tile0 = (c0 == 0);                            // tile holds packed column 0
  const bool selfpair = along_y || o == 0 || 2 * o == ny;  // column 0 still packed here
  const bool special = tile0 && MODE < 3 && selfpair;      // separation needs the mirror bin
  const bool col0 = tile0 && c == 0;
  __syncthreads();

  auto load = [&](const float2* __restrict__ src, float2 (&v)[E]) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cvalid ? src[obase + (t + TC * m) * stride + kxi] : f2(0.f, 0.f);
  };
  auto store = [&](float2* __restrict__ dst, const float2 (&v)[E]) {
    if (!cvalid) return;
#pragma unroll
    for (int m = 0; m < E; ++m) dst[obase + (t + TC * m) * stride + kxi] = v[m];
  };
  // mirror bin conj(C[-a]) along this column's axis (block-uniform call)
  auto mirror = [&](const float2 (&v)[E], float2 (&vm)[E]) {
#pragma unroll
    for (int m = 0; m < E; ++m) Lc[t + TC * m] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) vm[m] = conjf2(Lc[(NA - (t + TC * m)) & (NA - 1)]);
    __syncthreads();
  };

  if constexpr (MODE >= 3) {
    const int f = spec.f0 + (int)blockIdx.y;
    float2 v[E], vm[E];
    load(P.S[f], v);
    if constexpr (MODE == 3) {
      fft<NA, E, -1>(v, Lc, t, tws);
      if (tile0) {  // unpack column 0: A(a) at 0 < a < ny/2, B(ny - a) at ny/2 < a < ny
        mirror(v, vm);
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
      if (tile0) {  // pack column 0 again: C(a) = A(a) + i B(a), C(-a) = conj(A(a)) + i conj(B(a))
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
    store(P.S[f], v);
    return;
  } else {
    // ---- multiplier geometry, shared by every field and output of the block
    // y/z bin of element m: along y (2D) ky = a; along z (3D) ky = o, kz = a.
    // Column 0 outside the self-paired y-bins holds B of y-bin ny - o at
    // x-bin nx/2 (3D unpacked layout).
    const bool unpackedB = col0 && !selfpair && 2 * o > ny;
    const int kyf = along_y ? 0 : (unpackedB ? ny - o : o);
    const XBin xb = xbin(P, unpackedB ? M : kxi);
    const XBin xbN = xbin(P, M);
    const float k2fix = xb.k2 + (along_y ? 0.f : P.ksq[1][kyf]);
    const float k2fixN = xbN.k2 + (along_y ? 0.f : P.ksq[1][kyf]);
    const int ax_last = along_y ? 1 : 2;
    float k2v[E];
#pragma unroll
    for (int m = 0; m < E; ++m) k2v[m] = P.ksq[ax_last][t + TC * m];
    // per-element factor g (kappa/N, or the Laplacian factor) at the column's
    // x-bin and, for the packed column, at x-bin nx/2
    auto factor = [&](float k2, int which) -> float {
      if constexpr (FAM == F_ABS) {
        return (which == M_L1DT ? kpow(k2, P.ym2h) * P.inv_dt : kpow(k2, P.ym1h)) * P.scale;
      } else {
        return sinc_sqrt(P.kap2 * k2) * P.scale;
      }
    };
    // shift factors of derivative axis `axis` for the E elements of this
    // thread (the x shift is per column, the others per element or per block)
    auto shifts = [&](int axis, float2 (&sh)[E], float2 (&shN)[E]) {
      constexpr int SF = (FAM == F_ABS) ? F_A : FAM;
      if (axis == 0) {
        const float2 s0 = (SF == F_A) ? xb.sa : xb.sb, s1 = (SF == F_A) ? xbN.sa : xbN.sb;
#pragma unroll
        for (int m = 0; m < E; ++m) {
          sh[m] = s0;
          shN[m] = s1;
        }
      } else if (axis == 1 && !along_y) {
        const float2 s0 = (SF == F_A) ? P.shA[1][kyf] : P.shB[1][kyf];
#pragma unroll
        for (int m = 0; m < E; ++m) sh[m] = shN[m] = s0;
      } else {
        const float2* tab = (SF == F_A) ? P.shA[axis] : P.shB[axis];
#pragma unroll
        for (int m = 0; m < E; ++m) sh[m] = shN[m] = tab[t + TC * m];
      }
    };
    // acc += mult(kind/axis) * spectrum for one field
    auto apply = [&](int which, const float2 (&v)[E], const float2 (&vm)[E], float2 (&acc)[E]) {
      float2 sh[E], shN[E];
      if constexpr (FAM != F_ABS) shifts(which, sh, shN);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        float2 mv, mN;
        const float g = factor(k2fix + k2v[m], which);
        if constexpr (FAM == F_ABS) {
          mv = f2(g, 0.f);
        } else {
          mv = scl2(g, sh[m]);
        }
        if (col0 && selfpair) {
          const float gN = factor(k2fixN + k2v[m], which);
          if constexpr (FAM == F_ABS) {
            mN = f2(gN, 0.f);
          } else {
            mN = scl2(gN, shN[m]);
          }
          acc[m] = acc[m] + cmul(0.5f * (mv + mN), v[m]) + cmul(0.5f * (mv - mN), vm[m]);
        } else {
          acc[m] = acc[m] + cmul(mv, v[m]);
        }
      }
    };
    // which: derivative axis (0, 1, 2) for F_A / F_B, else the Mult kind
    auto which_of = [&](int i) { return FAM == F_ABS ? spec.mult[i] : i; };

    float2 v[E], vm[E], acc[E];
#pragma unroll
    for (int m = 0; m < E; ++m) vm[m] = f2(0.f, 0.f);
    if constexpr (MODE == 0) {
      load(P.S[0], v);
      fft<NA, E, -1>(v, Lc, t, tws);
      if (special) mirror(v, vm);
#pragma unroll
      for (int i = 0; i < NF; ++i) {
#pragma unroll
        for (int m = 0; m < E; ++m) acc[m] = f2(0.f, 0.f);
        apply(which_of(i), v, vm, acc);
        fft<NA, E, +1>(acc, Lc, t, tws);
        store(P.S[1 + i], acc);
      }
    } else if constexpr (MODE == 1) {
      const int i = (int)blockIdx.y;
      const int f = spec.f0 + i;
      load(P.S[spec.src >= 0 ? spec.src : f], v);
      fft<NA, E, -1>(v, Lc, t, tws);
      if (special) mirror(v, vm);
#pragma unroll
      for (int m = 0; m < E; ++m) acc[m] = f2(0.f, 0.f);
      apply(which_of(i), v, vm, acc);
      fft<NA, E, +1>(acc, Lc, t, tws);
      store(P.S[f], acc);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) acc[m] = f2(0.f, 0.f);
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        load(P.S[spec.f0 + i], v);
        fft<NA, E, -1>(v, Lc, t, tws);
        if (special) mirror(v, vm);
        apply(which_of(i), v, vm, acc);
      }
      fft<NA, E, +1>(acc, Lc, t, tws);
      store(P.S[0], acc);
    }
  }
}

// ------------------------------------------------------------------ launchers
static int default_tile(int na) {
  switch (na) {
    case 16: return ColGeo<16>::TILE;
    case 32: return ColGeo<32>::TILE;
    case 64: return ColGeo<64>::TILE;
    case 128: return ColGeo<128>::TILE;
    case 256: return ColGeo<256>::TILE;
    case 512: return ColGeo<512>::TILE;
    case 1024: return ColGeo<1024>::TILE;
  }
  return 0;
}

// tile widths with instantiated kernels for a column pass of axis length na
// (the autotuner's candidates): the default and, for the multiplier passes
// on one or two fields per launch and axes of 128 to 512 points, 8 and 4
int col_tile_candidates(int na, int mode, int nfield, int* out) {
  int n = 0;
  const int d = default_tile(na);
  if (!d) return 0;
  out[n++] = d;
  if ((mode == 1 || (mode != 3 && mode != 4 && nfield == 2)) && (na == 128 || na == 256 || na == 512)) {
    if (d != 8) out[n++] = 8;
    out[n++] = 4;
  }
  return n;
}

int col_axis_len(const ColSpec& spec, int ndim, int ny, int nz) {
  return (ndim == 2 || spec.mode >= 3) ? ny : nz;
}

int col_tile_of(const ColSpec& spec, int ndim, int ny, int nz) {
  const int na = col_axis_len(spec, ndim, ny, nz);
  int cand[4];
  const int n = col_tile_candidates(na, spec.mode, spec.nfield, cand);
  for (int i = 0; i < n; ++i)
    if (cand[i] == spec.tile) return spec.tile;
  return n ? cand[0] : 0;
}

// blocks of one column-pass launch for one instance: y-axis passes use nz
// groups of tiles, z-axis passes ny groups
int col_blocks(const ColSpec& spec, int ndim, int nx, int ny, int nz) {
  const int M = nx / 2;
  const int w = col_tile_of(spec, ndim, ny, nz);
  if (!w) return 0;
  const bool along_y = (ndim == 2 || spec.mode >= 3);
  const int other = (ndim == 2) ? 1 : (along_y ? nz : ny);
  return other * ((M + w - 1) / w);
}

template <int NA, int TW>
static hipError_t launch_col_nt(const ColSpec& spec, const Launch& L, int fam) {
  const dim3 block(ColGeo<NA, TW>::NTH);
  const dim3 grid1(L.nblocks), gridf(L.nblocks, spec.nfield);
#define PAT_COL(MODE, NF, FAMV, GRID)                                                                              \
  hipExtLaunchKernelGGL((k_col<NA, MODE, NF, FAMV, TW>), GRID, block, 0, L.stream, L.ev0, L.ev1, 0, L.plans, L.table, \
                        spec)
#define PAT_COL_FAM(MODE, NF, GRID)                       \
  do {                                                    \
    if (fam == F_A) PAT_COL(MODE, NF, F_A, GRID);         \
    else if (fam == F_B) PAT_COL(MODE, NF, F_B, GRID);    \
    else PAT_COL(MODE, NF, F_ABS, GRID);                  \
  } while (0)
  switch (spec.mode) {
    case 0:
      if (spec.nfield == 2) PAT_COL_FAM(0, 2, grid1);
      else if (TW == 0 && spec.nfield == 3) PAT_COL_FAM(0, 3, grid1);
      else return hipErrorInvalidValue;
      break;
    case 1: PAT_COL_FAM(1, 1, gridf); break;
    case 2:
      if (spec.nfield == 2) PAT_COL_FAM(2, 2, grid1);
      else if (TW == 0 && spec.nfield == 3) PAT_COL_FAM(2, 3, grid1);
      else return hipErrorInvalidValue;
      break;
    case 3:
      if (TW == 0) PAT_COL(3, 1, F_A, gridf);
      else return hipErrorInvalidValue;
      break;
    case 4:
      if (TW == 0) PAT_COL(4, 1, F_A, gridf);
      else return hipErrorInvalidValue;
      break;
    default: return hipErrorInvalidValue;
  }
#undef PAT_COL_FAM
#undef PAT_COL
  return hipGetLastError();
}

template <int NA>
static hipError_t launch_col_n(const ColSpec& spec, const Launch& L, int w) {
  // multiplier family from the kinds: derivatives a_j / b_j listed in axis
  // order, or the two fractional Laplacians
  int fam;
  if (spec.mode >= 3)
    fam = F_A;
  else if (spec.mult[0] == M_L1DT || spec.mult[0] == M_L2)
    fam = F_ABS;
  else
    fam = (spec.mult[0] >= M_BX) ? F_B : F_A;
  if (w == ColGeo<NA>::TILE) return launch_col_nt<NA, 0>(spec, L, fam);
  if constexpr (NA == 128 || NA == 256 || NA == 512) {
    if (w == 8) return launch_col_nt<NA, 8>(spec, L, fam);
    if (w == 4) return launch_col_nt<NA, 4>(spec, L, fam);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_col(const ColSpec& spec, int ndim, int nx, int ny, int nz, const Launch& L) {
  (void)nx;
  const int na = col_axis_len(spec, ndim, ny, nz);
  const int w = col_tile_of(spec, ndim, ny, nz);
  switch (na) {
    case 16: return launch_col_n<16>(spec, L, w);
    case 32: return launch_col_n<32>(spec, L, w);
    case 64: return launch_col_n<64>(spec, L, w);
    case 128: return launch_col_n<128>(spec, L, w);
    case 256: return launch_col_n<256>(spec, L, w);
    case 512: return launch_col_n<512>(spec, L, w);
    case 1024: return launch_col_n<1024>(spec, L, w);
  }
  return hipErrorInvalidValue;
}

hipError_t upload_twiddles_cols(const Tw* host) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tw), host, sizeof(Tw) * TWN, 0, hipMemcpyHostToDevice);
}

}  // namespace pat
