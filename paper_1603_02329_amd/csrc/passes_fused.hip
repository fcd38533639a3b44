// Fused passes of the batched executor: one launch per pass covers 2D
// instances of several grid sizes (both axis lengths 128, 256 or 512), each
// block dispatching on the size of its own instance to the pass body of the
// per-length kernels, and each instance advancing at its own rate through
// the launch's common step counter (fused_step).  Instances whose time axes
// differ -- a size class of N_t = 600 beside one of 2400 -- thus ride in the
// launches of the longest one instead of queueing their own short launches.
#include "passes_col.h"
#include "passes_row.h"

namespace pat {

namespace {
constexpr int kRowThreads = 256;

// rows per block of a fused row pass over rows of n points: 256 threads
template <int N>
constexpr int frows() {
  return kRowThreads / RowGeo<N>::T;
}
template <int N>
constexpr int row_lds() {
  return frows<N>() * RowGeo<N>::LDR;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
}  // namespace

template <int D, int K>
__global__ void __launch_bounds__(kRowThreads) k_rowf(const DevPlan* __restrict__ plans,
                                                      const int2* __restrict__ table, StepArg sa) {
  constexpr int LDSN = cmax(row_lds<512>(), cmax(row_lds<256>(), row_lds<128>()));
  constexpr int TWB = cmax(sizeof(RowTw<512>), cmax(sizeof(RowTw<256>), sizeof(RowTw<128>)));
  __shared__ float2 lds[LDSN];
  __shared__ __align__(16) unsigned char twraw[TWB];
  const int2 job = table[blockIdx.x];
  const DevPlan& P = plans[job.x];
  int it;
  if (!fused_step(P, sa, it)) return;  // block-uniform
  switch (P.n[0]) {
    case 512: row_pass<512, D, K, frows<512>()>(P, job.y, it, lds, *reinterpret_cast<RowTw<512>*>(twraw)); break;
    case 256: row_pass<256, D, K, frows<256>()>(P, job.y, it, lds, *reinterpret_cast<RowTw<256>*>(twraw)); break;
    case 128: row_pass<128, D, K, frows<128>()>(P, job.y, it, lds, *reinterpret_cast<RowTw<128>*>(twraw)); break;
    default: break;
  }
}

template <int NTH, int MODE, int NF, int FAM, int FPB>
__global__ void __launch_bounds__(NTH) k_colf(const DevPlan* __restrict__ plans, const int2* __restrict__ table,
                                              ColSpec spec, StepArg sa) {
  constexpr int T512 = NTH / 64, T256 = NTH / 32, T128 = NTH / 16;
  using L5 = ColLdsOf<512, T512, MODE, NF, FPB>;
  using L2 = ColLdsOf<256, T256, MODE, NF, FPB>;
  using L1 = ColLdsOf<128, T128, MODE, NF, FPB>;
  constexpr int B = cmax(sizeof(L5), cmax(sizeof(L2), sizeof(L1)));
  __shared__ __align__(16) unsigned char raw[B];
  const int2 job = table[blockIdx.x];
  const DevPlan& P = plans[job.x];
  int it;
  if (!fused_step(P, sa, it)) return;  // block-uniform
  switch (P.n[1]) {
    case 512:
      colm_pass<512, MODE, NF, FAM, T512, FPB>(P, job.y, spec, *reinterpret_cast<L5*>(raw));
      break;
    case 256:
      colm_pass<256, MODE, NF, FAM, T256, FPB>(P, job.y, spec, *reinterpret_cast<L2*>(raw));
      break;
    case 128:
      colm_pass<128, MODE, NF, FAM, T128, FPB>(P, job.y, spec, *reinterpret_cast<L1*>(raw));
      break;
    default: break;
  }
}

bool fused_size(int n) { return n == 128 || n == 256 || n == 512; }
int fused_row_rows(int nx) { return nx == 512 ? frows<512>() : nx == 256 ? frows<256>() : nx == 128 ? frows<128>() : 0; }
int fused_col_tile(int ny, int tile) { return fused_size(ny) && (tile == 8 || tile == 4) ? tile * 512 / ny : 0; }

int col_variants_fused(const ColSpec& spec, ColVariant* out) {
  if (spec.mode > 2) return 0;
  const bool two = spec.mode == 1 && spec.nfield == 2;
  int n = 0;
  for (int t : {8, 4}) {
    out[n++] = ColVariant{t, 1};
    if (two) out[n++] = ColVariant{t, 2};
  }
  return n;
}

hipError_t launch_row_fused(RowKind kind, const Launch& L, StepArg s) {
  const bool per_axis = (kind == R_FWD_1 || kind == R_ADJ_1);
  const dim3 grid(L.nblocks, per_axis ? 2 : 1), block(kRowThreads);
#define PAT_ROWF_CASE(KK)                                                                                     \
  case KK:                                                                                                    \
    hipExtLaunchKernelGGL((k_rowf<2, KK>), grid, block, 0, L.stream, L.ev0, L.ev1, 0, L.plans, L.table, s); \
    break;
  switch (kind) {
    PAT_ROWF_CASE(R_FWD_INIT)
    PAT_ROWF_CASE(R_FWD_1)
    PAT_ROWF_CASE(R_FWD_2)
    PAT_ROWF_CASE(R_FWD_2LL)
    PAT_ROWF_CASE(R_FWD_3)
    PAT_ROWF_CASE(R_ADJ_3)
    PAT_ROWF_CASE(R_ADJ_32LL)
    PAT_ROWF_CASE(R_ADJ_2)
    PAT_ROWF_CASE(R_ADJ_1)
    PAT_ROWF_CASE(R_ADJ_FINAL)
    PAT_ROWF_CASE(R_ADJ_SCATTER_ONLY)
    PAT_ROWF_CASE(R_FILT_IN)
    PAT_ROWF_CASE(R_FWD_INIT_F)
    PAT_ROWF_CASE(R_FILT_RE)
    PAT_ROWF_CASE(R_FILT_OUT)
    PAT_ROWF_CASE(R_EOS_FWD_IN)
    PAT_ROWF_CASE(R_EOS_FWD)
    PAT_ROWF_CASE(R_EOS_ADJ_IN)
    PAT_ROWF_CASE(R_EOS_ADJ)
    default: return hipErrorInvalidValue;
  }
#undef PAT_ROWF_CASE
  return hipGetLastError();
}

namespace {
template <int NTH>
hipError_t launch_colf(const ColSpec& spec, int fpb, const Launch& L, StepArg s) {
  const int fam = col_family(spec);
  const dim3 block(NTH);
#define PAT_COLF(MODE, NF, FAMV, FPBV, GY)                                                                        \
  hipExtLaunchKernelGGL((k_colf<NTH, MODE, NF, FAMV, FPBV>), dim3(L.nblocks, GY), block, 0, L.stream, L.ev0, L.ev1, \
                        0, L.plans, L.table, spec, s)
  if (spec.mode == 0 && spec.nfield == 2 && fam == F_A && fpb == 1) {
    PAT_COLF(0, 2, F_A, 1, 1);
  } else if (spec.mode == 1 && spec.nfield == 2 && fpb == 1) {
    if (fam == F_A) PAT_COLF(1, 1, F_A, 1, 2);
    else if (fam == F_B) PAT_COLF(1, 1, F_B, 1, 2);
    else PAT_COLF(1, 1, F_ABS, 1, 2);
  } else if (spec.mode == 1 && spec.nfield == 2 && fpb == 2) {
    if (fam == F_A) PAT_COLF(1, 2, F_A, 2, 1);
    else if (fam == F_B) PAT_COLF(1, 2, F_B, 2, 1);
    else PAT_COLF(1, 2, F_ABS, 2, 1);
  } else if (spec.mode == 2 && spec.nfield == 2 && fam == F_B && fpb == 1) {
    PAT_COLF(2, 2, F_B, 1, 1);
  } else if (spec.mode == 1 && spec.nfield == 1 && fam == F_WIN && fpb == 1) {
    PAT_COLF(1, 1, F_WIN, 1, 1);
  } else if (spec.mode == 1 && spec.nfield == 1 && fam == F_ABS && fpb == 1) {
    PAT_COLF(1, 1, F_ABS, 1, 1);  // L2 alone: the initial density's fixed-point steps
  } else {
    return hipErrorInvalidValue;
  }
#undef PAT_COLF
  return hipGetLastError();
}
}  // namespace

hipError_t launch_col_fused(const ColSpec& spec, ColVariant v, const Launch& L, StepArg s) {
  if (v.tile == 8) return launch_colf<512>(spec, v.fpb, L, s);
  if (v.tile == 4) return launch_colf<256>(spec, v.fpb, L, s);
  return hipErrorInvalidValue;
}

hipError_t upload_twiddles_fused(const Tw* host) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tw), host, sizeof(Tw) * TWN, 0, hipMemcpyHostToDevice);
}

}  // namespace pat
