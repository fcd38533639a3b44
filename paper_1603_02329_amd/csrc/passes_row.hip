// Time-step passes of the k-space scheme on gfx950: the per-length row pass
// kernels (bodies in passes_row.h), the sensor-sum reduction and the
// launchers.
#include <algorithm>

#include "passes_row.h"

namespace pat {

template <int N, int D, int K>
__global__ void __launch_bounds__(RowGeo<N>::NTH) k_row(const DevPlan* __restrict__ plans,
                                                        const int2* __restrict__ table, StepArg sa) {
  using G = RowGeo<N>;
  __shared__ float2 lds[G::ROWS * G::LDR];
  __shared__ RowTw<N> tws;
  const int2 job = table ? table[blockIdx.x] : make_int2(0, (int)blockIdx.x);
  row_pass<N, D, K, G::ROWS>(plans[job.x], job.y, step_of(sa), lds, tws);
}

// ------------------------------------------------------------------ gather reduction
// data[n][s] = sum of the sensor's partial row sums, for samples n0 <= n < n1
// (n1 <= 0 selects nt)
__global__ void __launch_bounds__(256) k_reduce(const DevPlan* __restrict__ plans, const int2* __restrict__ table,
                                                int n0, int n1) {
  const int2 job = table ? table[blockIdx.x] : make_int2(0, (int)blockIdx.x);
  const DevPlan& P = plans[job.x];
  const int nend = n1 > 0 ? n1 : P.nt;
  const long idx = (long)n0 * P.ns + (long)job.y * 256 + threadIdx.x;
  const long total = (long)nend * P.ns;
  if (idx >= total) return;
  const int n = (int)(idx / P.ns);
  const int s = (int)(idx - (long)n * P.ns);
  const float* part = P.partial + (long)n * P.nslots;
  const int k0 = gld(P.slot_ptr, s), k1 = gld(P.slot_ptr, s + 1);
  float acc = gld(part, k0);
  for (int k = k0 + 1; k < k1; ++k) acc += gld(part, k);
  gst(P.out, idx, acc);
}

// ------------------------------------------------------------------ launchers
int row_tile_rows(int nx) {
  switch (nx) {
    case 16: return RowGeo<16>::ROWS;
    case 32: return RowGeo<32>::ROWS;
    case 64: return RowGeo<64>::ROWS;
    case 128: return RowGeo<128>::ROWS;
    case 256: return RowGeo<256>::ROWS;
    case 512: return RowGeo<512>::ROWS;
    case 1024: return RowGeo<1024>::ROWS;
  }
  return 0;
}

template <int N, int D>
static hipError_t launch_row_nd(RowKind kind, const Launch& L, StepArg s) {
  // the velocity passes run one axis component per block row (grid.y)
  const bool per_axis = (kind == R_FWD_1 || kind == R_ADJ_1);
  const dim3 grid(L.nblocks, per_axis ? D : 1), block(RowGeo<N>::NTH);
#define PAT_ROW_CASE(KK) \
  case KK:                                                                                        \
    hipExtLaunchKernelGGL((k_row<N, D, KK>), grid, block, 0, L.stream, L.ev0, L.ev1, 0, L.plans, L.table, s); \
    break;
  switch (kind) {
    PAT_ROW_CASE(R_FWD_INIT)
    PAT_ROW_CASE(R_FWD_1)
    PAT_ROW_CASE(R_FWD_2)
    PAT_ROW_CASE(R_FWD_2LL)
    PAT_ROW_CASE(R_FWD_3)
    PAT_ROW_CASE(R_ADJ_3)
    PAT_ROW_CASE(R_ADJ_32LL)
    PAT_ROW_CASE(R_ADJ_2)
    PAT_ROW_CASE(R_ADJ_1)
    PAT_ROW_CASE(R_ADJ_FINAL)
    PAT_ROW_CASE(R_ADJ_SCATTER_ONLY)
    PAT_ROW_CASE(R_ATD_2)
    PAT_ROW_CASE(R_ATD_2LL)
    PAT_ROW_CASE(R_ATD_3)
    PAT_ROW_CASE(R_ATD_FINAL)
    PAT_ROW_CASE(R_FILT_IN)
    PAT_ROW_CASE(R_FWD_INIT_F)
    PAT_ROW_CASE(R_FILT_RE)
    PAT_ROW_CASE(R_FILT_OUT)
    PAT_ROW_CASE(R_EOS_FWD_IN)
    PAT_ROW_CASE(R_EOS_FWD)
    PAT_ROW_CASE(R_EOS_ADJ_IN)
    PAT_ROW_CASE(R_EOS_ADJ)
    default: return hipErrorInvalidValue;
  }
#undef PAT_ROW_CASE
  return hipGetLastError();
}

hipError_t launch_row(RowKind kind, int ndim, int nx, const Launch& L, StepArg s) {
  if (ndim == 2) {
    switch (nx) {
      case 16: return launch_row_nd<16, 2>(kind, L, s);
      case 32: return launch_row_nd<32, 2>(kind, L, s);
      case 64: return launch_row_nd<64, 2>(kind, L, s);
      case 128: return launch_row_nd<128, 2>(kind, L, s);
      case 256: return launch_row_nd<256, 2>(kind, L, s);
      case 512: return launch_row_nd<512, 2>(kind, L, s);
      case 1024: return launch_row_nd<1024, 2>(kind, L, s);
    }
  } else if (ndim == 3) {
    switch (nx) {
      case 16: return launch_row_nd<16, 3>(kind, L, s);
      case 32: return launch_row_nd<32, 3>(kind, L, s);
      case 64: return launch_row_nd<64, 3>(kind, L, s);
      case 128: return launch_row_nd<128, 3>(kind, L, s);
      case 256: return launch_row_nd<256, 3>(kind, L, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(const Launch& L, int n0, int n1) {
  hipLaunchKernelGGL(k_reduce, dim3(L.nblocks), dim3(256), 0, L.stream, L.plans, L.table, n0, n1);
  return hipGetLastError();
}

hipError_t upload_twiddles_rows(const Tw* host) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tw), host, sizeof(Tw) * TWN, 0, hipMemcpyHostToDevice);
}

}  // namespace pat
