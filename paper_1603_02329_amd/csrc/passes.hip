// Time-step passes of the k-space scheme on gfx950.
//
// Each spectral operator F^-1[m F f] of the scheme is split into two kinds
// of passes over HBM:
//   row pass    : per grid row (x fastest), inverse real FFT along x of the
//                 incoming packed spectra -> the pointwise part of the step
//                 (velocity, density, state or their transposes, PML, sensor
//                 gather/scatter) -> forward real FFT along x of the fields the
//                 next spectral operator needs;
//   column pass : per tile of x-frequency columns, FFT along y (and z), the
//                 k-space multiplier, inverse FFT along y (and z).
// Between passes only packed x-spectra (4 bytes per grid point and field)
// and the state fields travel through memory; the pressure itself never
// does.  The multipliers are formed on the fly from 1-D per-axis tables.
//
// The forward step (equations mom, mass, state of section II-A, split per
// axis for the PML) is
//   col  : S1,S2 <- a_x, a_y applied to S0 = F_x p             (gradient)
//   row 1: u_j   <- Qsg_j (Qsg_j u_j - B_j d_j p);  S_j <- F_x u_j
//   col  : S_j   <- b_j applied to S_j                          (divergence)
//   row 2: rho_j <- Q_j (Q_j rho_j - dt rho0 g_j);  S1 <- F_x(dt rho0 sum g),
//                                                   S2 <- F_x(sum rho)
//   col  : S1 <- |k|^(y-2)/dt S1, S2 <- |k|^(y-1) S2            (absorption)
//   row 3: p = c0^2 sum rho + c0^2 tau A1 - c0^2 eta A2; gather; S0 <- F_x p
// and the adjoint runs the transposed passes in reverse order.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fft.h"
#include "pat_internal.h"

namespace pat {

__device__ Tw g_tw[TWN];

// ------------------------------------------------------------------ geometry
template <int N>
struct RowGeo {
  static constexpr int M = N / 2;             // packed complex bins per row
  static constexpr int E = (M < 8) ? M : 8;   // values per thread
  static constexpr int T = M / E;             // threads per row
  static constexpr int ROWS = (256 / T) < 16 ? (256 / T) : 16;
  static constexpr int NTH = ROWS * T;
};

template <int NY>
struct ColGeo {
  static constexpr int E = 8;
  static constexpr int TC = NY / E;                          // threads per column
  static constexpr int TILE = (1024 / TC) < 16 ? (1024 / TC) : 16;
  static constexpr int NTH = TILE * TC;
  static constexpr int LD = NY + 1;                          // padded LDS column stride
};

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ float2 ld2(const float* a, long i) { return reinterpret_cast<const float2*>(a)[i]; }
__device__ __forceinline__ void st2(float* a, long i, float2 v) { reinterpret_cast<float2*>(a)[i] = v; }
__device__ __forceinline__ float2 f2(float a, float b) { return make_float2(a, b); }
__device__ __forceinline__ float2 mul2(float2 a, float2 b) { return make_float2(a.x * b.x, a.y * b.y); }
__device__ __forceinline__ float2 scl2(float s, float2 a) { return make_float2(s * a.x, s * a.y); }

// Packed half spectrum of one row -> real row, as pairs (x[2n], x[2n+1]) at
// n = t + T m.  Unnormalised inverse real DFT.
// r holds the packed bins X[t + T m] on entry (already loaded) and the real
// pairs on exit.
template <int N>
__device__ __forceinline__ void c2r(float2 (&r)[RowGeo<N>::E], float2* L, int t, const Tw* tw) {
  using G = RowGeo<N>;
  constexpr int M = G::M, E = G::E, T = G::T;
#pragma unroll
  for (int m = 0; m < E; ++m) L[t + T * m] = r[m];
  WaveSync::sync();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    const float2 X = L[k];
    if (k == 0) {
      r[m] = f2(X.x + X.y, X.x - X.y);
    } else {
      const float2 Y = conjf2(L[M - k]);
      const float2 A = X + Y;
      const float2 B = twmul<+1>(X - Y, tw[k]);
      r[m] = A + mul_si<+1>(B);
    }
  }
  WaveSync::sync();
  fft<M, E, +1, WaveSync, 2>(r, L, t, tw);
}

// Real row held as pairs (x[2n], x[2n+1]) -> packed half spectrum stored at dst.
template <int N>
__device__ __forceinline__ void r2c(float2 (&r)[RowGeo<N>::E], float2* __restrict__ dst, float2* L, int t,
                                    bool valid, const Tw* tw) {
  using G = RowGeo<N>;
  constexpr int M = G::M, E = G::E, T = G::T;
  fft<M, E, -1, WaveSync, 2>(r, L, t, tw);
#pragma unroll
  for (int m = 0; m < E; ++m) L[t + T * m] = r[m];
  WaveSync::sync();
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    const float2 Z = L[k];
    float2 X;
    if (k == 0) {
      X = f2(Z.x + Z.y, Z.x - Z.y);
    } else {
      const float2 Y = conjf2(L[M - k]);
      const float2 A = Z + Y;
      const float2 B = twmul<-1>(Z - Y, tw[k]);
      X = 0.5f * (A + mul_si<-1>(B));
    }
    if (valid) dst[k] = X;
  }
  WaveSync::sync();
}

// Sensor gather of sample `n` from the real row p held in LDS (as floats).
template <int N>
__device__ __forceinline__ void gather_row(const DevPlan& P, int n, const float* Lf, int row, int t, bool valid) {
  using G = RowGeo<N>;
  WaveSync::sync();
  if (valid) {
    const int e1 = P.g_ptr[row + 1];
    float* out = P.partial + (long)n * P.nslots;
    for (int e = P.g_ptr[row] + t; e < e1; e += G::T) {
      const GTap tap = P.g_tap[e];
      out[tap.slot] = fmaf(tap.w0, Lf[tap.x0], tap.w1 * Lf[tap.x0 + 1]);
    }
  }
  WaveSync::sync();
}

// Add W^T h[n] for this row to the real row held in LDS (as floats).
template <int N>
__device__ __forceinline__ void scatter_row(const DevPlan& P, int n, float* Lf, int row, int t, bool valid) {
  using G = RowGeo<N>;
  WaveSync::sync();
  if (valid) {
    const int g1 = P.s_ptr[row + 1];
    const float* h = P.in + (long)n * P.ns;
    for (int g = P.s_ptr[row] + t; g < g1; g += G::T) {
      const SGroup grp = P.s_grp[g];
      float acc = 0.f;
      for (int e = grp.beg; e < grp.end; ++e) {
        const STap tp = P.s_tap[e];
        acc = fmaf(tp.w, h[tp.s], acc);
      }
      Lf[grp.x] += acc;
    }
  }
  WaveSync::sync();
}

// c0^2 tau and c0^2 eta from c0^2 when alpha0 is uniform (equation Twelve:
// tau = -2 a0 c0^(y-1), eta = 2 a0 c0^y tan(pi y / 2))
template <int E>
__device__ __forceinline__ void absorption_coefs(const DevPlan& P, const float2 (&c2)[E], float2 (&ct)[E],
                                                 float2 (&ce)[E]) {
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const float lx = __builtin_amdgcn_logf(c2[m].x), ly = __builtin_amdgcn_logf(c2[m].y);
    ct[m] = f2(P.ktau * __builtin_amdgcn_exp2f(P.etau * lx), P.ktau * __builtin_amdgcn_exp2f(P.etau * ly));
    ce[m] = f2(P.keta * __builtin_amdgcn_exp2f(P.eeta * lx), P.keta * __builtin_amdgcn_exp2f(P.eeta * ly));
  }
}

__device__ __forceinline__ void check_finite(const DevPlan& P, float2 v) {
  if ((P.flags & PAT_CHECK_FINITE) && !(isfinite(v.x) && isfinite(v.y))) atomicOr(P.bad, 1);
}

// ------------------------------------------------------------------ row passes
// Each row pass first issues every global load it needs (the packed input
// spectra and the per-point state and medium values of its rows) so that the
// memory latency is paid once per block, then runs the transforms from
// registers.  The velocity passes treat one axis component per block
// (blockIdx.y): the components are independent, and the split halves the
// registers a block holds.
template <int N>
struct RowIo {
  static constexpr int E = RowGeo<N>::E, T = RowGeo<N>::T;
  const long base;
  const int t;
  const bool valid;
  __device__ __forceinline__ void ld(const float* a, float2 (&v)[E]) const {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = valid ? ld2(a, base + t + T * m) : f2(0.f, 0.f);
  }
  __device__ __forceinline__ void ld(const float2* a, float2 (&v)[E]) const {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = valid ? a[base + t + T * m] : f2(0.f, 0.f);
  }
  // 1-D x table (PML factor along x), pairs at n = t + T m
  __device__ __forceinline__ void ldx(const float* a, float2 (&v)[E]) const {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = ld2(a, t + T * m);
  }
  __device__ __forceinline__ void st(float* a, const float2 (&v)[E]) const {
    if (!valid) return;
#pragma unroll
    for (int m = 0; m < E; ++m) st2(a, base + t + T * m, v[m]);
  }
  __device__ __forceinline__ void zero(float2 (&v)[E]) const {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = f2(0.f, 0.f);
  }
};

template <int N, int D, int K>
__global__ void __launch_bounds__(RowGeo<N>::NTH) k_row(const DevPlan* __restrict__ plans,
                                                        const int2* __restrict__ table, StepArg sa) {
  using G = RowGeo<N>;
  constexpr int M = G::M, E = G::E, T = G::T;
  __shared__ float2 lds[G::ROWS * M];
  __shared__ Tw tws[N];
  load_twiddles<N, G::NTH>(tws, g_tw);
  const int2 job = table ? table[blockIdx.x] : make_int2(0, (int)blockIdx.x);
  const DevPlan& P = plans[job.x];
  const int rl = threadIdx.x / T, t = threadIdx.x % T;
  const int row = job.y * G::ROWS + rl;
  const bool valid = row < P.nrows;
  const int rowc = valid ? row : 0;
  const int ny = P.n[1];
  const int yy = rowc % ny, zz = rowc / ny;
  float2* L = lds + rl * M;
  float* Lf = reinterpret_cast<float*>(L);
  const RowIo<N> io{(long)rowc * M, t, valid};
  const int it = step_of(sa);  // forward step n / adjoint iteration i

  // per-row PML factors of the y and z axes
  float qrow[3] = {1.f, P.Q[1][yy], 1.f};
  float qsrow[3] = {1.f, P.Qsg[1][yy], 1.f};
  if constexpr (D == 3) {
    qrow[2] = P.Q[2][zz];
    qsrow[2] = P.Qsg[2][zz];
  }
  auto qpair = [&](int j, const float2& qx) { return j == 0 ? qx : f2(qrow[j], qrow[j]); };
  auto qspair = [&](int j, const float2& qx) { return j == 0 ? qx : f2(qsrow[j], qsrow[j]); };

  if constexpr (K == R_FWD_INIT) {
    float2 p[E], ic[E];
    io.ld(P.in, p);
    io.ld(P.inv_dc2, ic);
    __syncthreads();  // twiddles
    float2 rr[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      rr[m] = mul2(p[m], ic[m]);
      L[t + T * m] = p[m];
    }
#pragma unroll
    for (int j = 0; j < D; ++j) io.st(P.r[j], rr);
    gather_row<N>(P, 0, Lf, rowc, t, valid);
    r2c<N>(p, P.S[0] + io.base, L, t, valid, tws);
  } else if constexpr (K == R_FWD_1 || K == R_ADJ_1) {
    // one axis component j per block
    const int j = (int)blockIdx.y;
    const bool first = (it == 0);
    const bool last = (K == R_ADJ_1) && (it == P.nt - 2);
    float2 d[E], b[E], u[E], qx[E];
    io.ld(P.S[1 + j], d);
    io.ld(P.B[j], b);
    if (first) io.zero(u); else io.ld(P.u[j], u);
    if (j == 0) io.ldx(P.Qsg[0], qx);
    __syncthreads();  // twiddles
    c2r<N>(d, L, t, tws);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const float2 qs = qspair(j, qx[m]);
      if constexpr (K == R_FWD_1) {
        // u <- Qsg (Qsg u - B d p); the first step starts from u = (B/2) d p
        const float2 db = mul2(b[m], d[m]);
        const float2 u0 = first ? scl2(0.5f, db) : u[m];
        u[m] = mul2(qs, mul2(qs, u0) - db);
        d[m] = u[m];
      } else {
        // ubar -= d+ gbar; feed B Qsg ubar (last step: B Qsg ubar (1 - Qsg/2)), ubar <- Qsg^2 ubar
        const float2 ub = u[m] - d[m];
        const float2 bq = mul2(b[m], mul2(qs, ub));
        d[m] = last ? mul2(bq, f2(1.f - 0.5f * qs.x, 1.f - 0.5f * qs.y)) : bq;
        u[m] = mul2(mul2(qs, qs), ub);
      }
    }
    if (K == R_FWD_1 || !last) io.st(P.u[j], u);
    r2c<N>(d, P.S[1 + j] + io.base, L, t, valid, tws);
  } else if constexpr (K == R_FWD_2 || K == R_FWD_2LL) {
    float2 g[D][E], r[D][E], dr[E], c2[E], qx[E];
#pragma unroll
    for (int j = 0; j < D; ++j) io.ld(P.S[1 + j], g[j]);
#pragma unroll
    for (int j = 0; j < D; ++j) io.ld(P.r[j], r[j]);
    io.ld(P.dtr0, dr);
    if constexpr (K == R_FWD_2LL) io.ld(P.c2, c2);
    io.ldx(P.Q[0], qx);
    __syncthreads();  // twiddles
#pragma unroll
    for (int j = 0; j < D; ++j) c2r<N>(g[j], L, t, tws);
    float2 sdiv[E], srho[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      sdiv[m] = f2(0.f, 0.f);
      srho[m] = f2(0.f, 0.f);
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const float2 q = qpair(j, qx[m]);
        const float2 tj = mul2(dr[m], g[j][m]);
        r[j][m] = mul2(q, mul2(q, r[j][m]) - tj);
        sdiv[m] = sdiv[m] + tj;
        srho[m] = srho[m] + r[j][m];
      }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) io.st(P.r[j], r[j]);
    if constexpr (K == R_FWD_2) {
      r2c<N>(sdiv, P.S[1] + io.base, L, t, valid, tws);
      r2c<N>(srho, P.S[2] + io.base, L, t, valid, tws);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        srho[m] = mul2(c2[m], srho[m]);
        if (valid) check_finite(P, srho[m]);
        L[t + T * m] = srho[m];
      }
      gather_row<N>(P, it + 1, Lf, rowc, t, valid);
      r2c<N>(srho, P.S[0] + io.base, L, t, valid, tws);
    }
  } else if constexpr (K == R_FWD_3) {
    // the spectra first; the pointwise operands after the transforms (loading
    // all of them up front would double the registers held across the FFTs)
    float2 a1[E], a2[E], rs[E], c2[E], ct[E], ce[E];
    io.ld(P.S[1], a1);
    io.ld(P.S[2], a2);
    __syncthreads();  // twiddles
    c2r<N>(a1, L, t, tws);
    c2r<N>(a2, L, t, tws);
    io.ld(P.r[0], rs);
#pragma unroll
    for (int j = 1; j < D; ++j) {
      float2 rj[E];
      io.ld(P.r[j], rj);
#pragma unroll
      for (int m = 0; m < E; ++m) rs[m] = rs[m] + rj[m];
    }
    io.ld(P.c2, c2);
    if (P.alpha_uniform) {
      absorption_coefs<E>(P, c2, ct, ce);
    } else {
      io.ld(P.c2tau, ct);
      io.ld(P.c2eta, ce);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const float2 p = mul2(c2[m], rs[m]) + mul2(ct[m], a1[m]) - mul2(ce[m], a2[m]);
      if (valid) check_finite(P, p);
      a1[m] = p;
      L[t + T * m] = p;
    }
    gather_row<N>(P, it + 1, Lf, rowc, t, valid);
    r2c<N>(a1, P.S[0] + io.base, L, t, valid, tws);
  } else if constexpr (K == R_ADJ_3 || K == R_ADJ_32LL) {
    const bool first = (it == 0);
    const int nsamp = P.nt - 1 - it;  // h[n+1] with n = nt-2-it
    float2 v[E], c2[E], e1[E], e2[E], dr[E], qx[E];
    if (first) io.zero(v); else io.ld(P.S[0], v);
    io.ld(P.c2, c2);
    if constexpr (K == R_ADJ_3) {
      if (P.alpha_uniform) {
        absorption_coefs<E>(P, c2, e2, e1);
      } else {
        io.ld(P.c2eta, e1);
        io.ld(P.c2tau, e2);
      }
    } else {
      io.ld(P.dtr0, dr);
      io.ldx(P.Q[0], qx);
    }
    float2 rb[D][E];
    if constexpr (K == R_ADJ_32LL) {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        if (first) io.zero(rb[j]); else io.ld(P.r[j], rb[j]);
      }
    }
    __syncthreads();  // twiddles
    if (!first) c2r<N>(v, L, t, tws);
#pragma unroll
    for (int m = 0; m < E; ++m) L[t + T * m] = v[m];
    scatter_row<N>(P, nsamp, Lf, rowc, t, valid);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = L[t + T * m];
    WaveSync::sync();
    if constexpr (K == R_ADJ_3) {
      float2 q[E];
#pragma unroll
      for (int m = 0; m < E; ++m) {
        q[m] = mul2(c2[m], v[m]);
        e1[m] = mul2(e1[m], v[m]);
        e2[m] = mul2(e2[m], v[m]);
      }
      io.st(P.q, q);
      r2c<N>(e1, P.S[1] + io.base, L, t, valid, tws);
      r2c<N>(e2, P.S[2] + io.base, L, t, valid, tws);
    } else {
      float2 g[D][E];
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const float2 q = mul2(c2[m], v[m]);
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const float2 qq = qpair(j, qx[m]);
          const float2 r1 = rb[j][m] + q;
          g[j][m] = f2(0.f, 0.f) - mul2(dr[m], mul2(qq, r1));
          rb[j][m] = mul2(mul2(qq, qq), r1);
        }
      }
#pragma unroll
      for (int j = 0; j < D; ++j) io.st(P.r[j], rb[j]);
#pragma unroll
      for (int j = 0; j < D; ++j) r2c<N>(g[j], P.S[1 + j] + io.base, L, t, valid, tws);
    }
  } else if constexpr (K == R_ADJ_2) {
    const bool first = (it == 0);
    float2 a2[E], a1[E], q[E], dr[E], qx[E], rb[D][E];
    io.ld(P.S[1], a2);
    io.ld(P.S[2], a1);
    __syncthreads();  // twiddles
    c2r<N>(a2, L, t, tws);
    c2r<N>(a1, L, t, tws);
    io.ld(P.q, q);
    io.ld(P.dtr0, dr);
    io.ldx(P.Q[0], qx);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (first) io.zero(rb[j]); else io.ld(P.r[j], rb[j]);
    }
    float2 g[D][E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const float2 qa = q[m] - a2[m];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const float2 qq = qpair(j, qx[m]);
        const float2 r1 = rb[j][m] + qa;
        g[j][m] = mul2(dr[m], a1[m] - mul2(qq, r1));
        rb[j][m] = mul2(mul2(qq, qq), r1);
      }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) io.st(P.r[j], rb[j]);
#pragma unroll
    for (int j = 0; j < D; ++j) r2c<N>(g[j], P.S[1 + j] + io.base, L, t, valid, tws);
  } else if constexpr (K == R_ADJ_FINAL || K == R_ADJ_SCATTER_ONLY) {
    float2 v[E], rs[E], ic[E];
    if constexpr (K == R_ADJ_FINAL) {
      io.ld(P.S[0], v);
      io.ld(P.r[0], rs);
#pragma unroll
      for (int j = 1; j < D; ++j) {
        float2 rj[E];
        io.ld(P.r[j], rj);
#pragma unroll
        for (int m = 0; m < E; ++m) rs[m] = rs[m] + rj[m];
      }
      io.ld(P.inv_dc2, ic);
    } else {
      io.zero(v);
    }
    __syncthreads();  // twiddles
    if constexpr (K == R_ADJ_FINAL) c2r<N>(v, L, t, tws);
#pragma unroll
    for (int m = 0; m < E; ++m) L[t + T * m] = v[m];
    scatter_row<N>(P, 0, Lf, rowc, t, valid);
#pragma unroll
    for (int m = 0; m < E; ++m) {
      v[m] = L[t + T * m];
      if constexpr (K == R_ADJ_FINAL) v[m] = v[m] + mul2(rs[m], ic[m]);
    }
    io.st(P.out, v);
  }
}

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
template <int NA, int MODE, int NF, int FAM>
__global__ void __launch_bounds__(ColGeo<NA>::NTH) k_col(const DevPlan* __restrict__ plans,
                                                         const int2* __restrict__ table, ColSpec spec) {
  using G = ColGeo<NA>;
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
  const int k0 = P.slot_ptr[s], k1 = P.slot_ptr[s + 1];
  float acc = part[k0];
  for (int k = k0 + 1; k < k1; ++k) acc += part[k];
  P.out[idx] = acc;
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

static int col_tile_width(int na) {
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

// blocks of one column-pass launch of one instance (the maximum over the
// passes of the step: y-axis passes use nz groups, z-axis passes ny groups)
int col_tiles(int ndim, int nx, int ny, int nz) {
  const int M = nx / 2;
  int best = 0;
  for (int pass = 0; pass < (ndim == 3 ? 2 : 1); ++pass) {
    const int na = (ndim == 2 || pass == 0) ? ny : nz;
    const int other = (ndim == 2) ? 1 : (pass == 0 ? nz : ny);
    const int tile = col_tile_width(na);
    if (!tile) return 0;
    best = std::max(best, other * ((M + tile - 1) / tile));
  }
  return best;
}

template <int NA>
static hipError_t launch_col_n(const ColSpec& spec, const Launch& L) {
  const dim3 block(ColGeo<NA>::NTH);
  const dim3 grid1(L.nblocks), gridf(L.nblocks, spec.nfield);
  // multiplier family from the kinds: derivatives a_j / b_j listed in axis
  // order, or the two fractional Laplacians
  int fam;
  if (spec.mode >= 3)
    fam = F_A;
  else if (spec.mult[0] == M_L1DT || spec.mult[0] == M_L2)
    fam = F_ABS;
  else
    fam = (spec.mult[0] >= M_BX) ? F_B : F_A;
#define PAT_COL(MODE, NF, FAMV, GRID) \
  hipExtLaunchKernelGGL((k_col<NA, MODE, NF, FAMV>), GRID, block, 0, L.stream, L.ev0, L.ev1, 0, L.plans, L.table, \
                        spec)
#define PAT_COL_FAM(MODE, NF, GRID)              \
  do {                                           \
    if (fam == F_A) PAT_COL(MODE, NF, F_A, GRID);     \
    else if (fam == F_B) PAT_COL(MODE, NF, F_B, GRID); \
    else PAT_COL(MODE, NF, F_ABS, GRID);              \
  } while (0)
  switch (spec.mode) {
    case 0:
      if (spec.nfield == 2) PAT_COL_FAM(0, 2, grid1);
      else if (spec.nfield == 3) PAT_COL_FAM(0, 3, grid1);
      else return hipErrorInvalidValue;
      break;
    case 1: PAT_COL_FAM(1, 1, gridf); break;
    case 2:
      if (spec.nfield == 2) PAT_COL_FAM(2, 2, grid1);
      else if (spec.nfield == 3) PAT_COL_FAM(2, 3, grid1);
      else return hipErrorInvalidValue;
      break;
    case 3: PAT_COL(3, 1, F_A, gridf); break;
    case 4: PAT_COL(4, 1, F_A, gridf); break;
    default: return hipErrorInvalidValue;
  }
#undef PAT_COL_FAM
#undef PAT_COL
  return hipGetLastError();
}

hipError_t launch_col(const ColSpec& spec, int ndim, int nx, int ny, int nz, const Launch& L) {
  (void)nx;
  const int na = (ndim == 2 || spec.mode >= 3) ? ny : nz;
  switch (na) {
    case 16: return launch_col_n<16>(spec, L);
    case 32: return launch_col_n<32>(spec, L);
    case 64: return launch_col_n<64>(spec, L);
    case 128: return launch_col_n<128>(spec, L);
    case 256: return launch_col_n<256>(spec, L);
    case 512: return launch_col_n<512>(spec, L);
    case 1024: return launch_col_n<1024>(spec, L);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(const Launch& L, int n0, int n1) {
  hipLaunchKernelGGL(k_reduce, dim3(L.nblocks), dim3(256), 0, L.stream, L.plans, L.table, n0, n1);
  return hipGetLastError();
}

hipError_t upload_twiddles(const Tw* host) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tw), host, sizeof(Tw) * TWN, 0, hipMemcpyHostToDevice);
}

}  // namespace pat
