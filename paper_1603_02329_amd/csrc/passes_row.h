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
#pragma once

#include "passes_common.h"

namespace pat {

// ------------------------------------------------------------------ geometry
template <int N>
struct RowGeo {
  static constexpr int M = N / 2;             // packed complex bins per row
  static constexpr int E = (M < 8) ? M : 8;   // values per thread
  static constexpr int T = M / E;             // threads per row
  static constexpr int ROWS = (256 / T) < 16 ? (256 / T) : 16;
  static constexpr int NTH = ROWS * T;
  static constexpr int LDR = M + M / 8;       // LDS slots per row (padded FFT exchange)
  static constexpr int TWS = staged_len(M, E);  // staged FFT twiddles
};

// LDS twiddles of a row pass: the untangling factors exp(-2 pi i k / N),
// k < M, then the staged FFT tables
template <int N>
struct RowTw {
  Tw u[N / 2];
  Tw s[RowGeo<N>::TWS > 0 ? RowGeo<N>::TWS : 1];
};
// Both tables in one pass (u then s, contiguous in RowTw): one memory round
// trip, issued after the pass's own loads.
template <int N, int NTH = RowGeo<N>::NTH>
__device__ __forceinline__ void load_row_twiddles(RowTw<N>& tw, const Tw* __restrict__ g) {
  using G = RowGeo<N>;
  static_assert(sizeof(RowTw<N>) == sizeof(Tw) * (G::M + (G::TWS > 0 ? G::TWS : 1)), "RowTw is not contiguous");
  load_table<G::M + G::TWS, NTH>(reinterpret_cast<Tw*>(&tw), g, [](int q) {
    return q < G::M ? q * (TWN / N) : staged_src<G::M, G::E>(q - G::M);
  });
}

// The mirror bins of a row's packed spectrum: for element k = t + T m
// (k != 0), element M - k, held by lane (T - t) mod T of the row's T lanes in
// register E - 1 - m (t != 0), or by this lane in register (E - m) mod E
// (t = 0).  Fetched by a cross-lane permute within the wavefront
// (ds_bpermute) rather than a round trip through the row's LDS region.
// Every lane of the wavefront must call it; the rows' lanes are aligned to
// T within the wavefront.
template <int T, int E>
__device__ __forceinline__ void row_mirror(const float2 (&r)[E], float2 (&y)[E], int t) {
  static_assert(T <= 64 && (T & (T - 1)) == 0 && (E & (E - 1)) == 0, "row lanes must tile the wavefront");
  const int lane = (int)(threadIdx.x & 63);
  const int src = ((lane & ~(T - 1)) | ((T - t) & (T - 1))) << 2;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const float2 v = r[E - 1 - m];
    const float px = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v.x)));
    const float py = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(v.y)));
    y[m] = (t == 0) ? r[(E - m) & (E - 1)] : f2(px, py);
  }
}

// Packed half spectrum of one row -> real row, as pairs (x[2n], x[2n+1]) at
// n = t + T m.  Unnormalised inverse real DFT.
// r holds the packed bins X[t + T m] on entry (already loaded) and the real
// pairs on exit.
template <int N>
__device__ __forceinline__ void c2r(float2 (&r)[RowGeo<N>::E], float2* L, int t, const RowTw<N>& tw) {
  using G = RowGeo<N>;
  constexpr int M = G::M, E = G::E, T = G::T;
  float2 y[E];
  row_mirror<T, E>(r, y, t);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    const float2 X = r[m];
    if (k == 0) {
      r[m] = f2(X.x + X.y, X.x - X.y);
    } else {
      const float2 Y = conjf2(y[m]);
      const float2 A = X + Y;
      const float2 B = twmul<+1>(X - Y, tw.u[k]);
      r[m] = A + mul_si<+1>(B);
    }
  }
  WaveSync::sync();  // earlier readers of the row's region are done
  fft<M, E, +1, WaveSync, 1, TwStaged, true>(r, L, t, tw.s);
}

// Real row held as pairs (x[2n], x[2n+1]) -> packed half spectrum stored at dst.
template <int N>
__device__ __forceinline__ void r2c(float2 (&r)[RowGeo<N>::E], float2* __restrict__ dst, float2* L, int t,
                                    bool valid, const RowTw<N>& tw) {
  using G = RowGeo<N>;
  constexpr int M = G::M, E = G::E, T = G::T;
  fft<M, E, -1, WaveSync, 1, TwStaged, true>(r, L, t, tw.s);
  float2 y[E];
  row_mirror<T, E>(r, y, t);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + T * m;
    const float2 Z = r[m];
    float2 X;
    if (k == 0) {
      X = f2(Z.x + Z.y, Z.x - Z.y);
    } else {
      const float2 Y = conjf2(y[m]);
      const float2 A = Z + Y;
      const float2 B = twmul<-1>(Z - Y, tw.u[k]);
      X = 0.5f * (A + mul_si<-1>(B));
    }
    if (valid) gst(dst, k, X);
  }
  WaveSync::sync();
}

// Sensor gather of sample `n` from the real row p held in LDS (as floats).
template <int N>
__device__ __forceinline__ void gather_row(const DevPlan& P, int n, const float* Lf, int row, int t, bool valid) {
  using G = RowGeo<N>;
  WaveSync::sync();
  if (valid) {
    const int e1 = gld(P.g_ptr, row + 1);
    float* out = P.partial + (long)n * P.nslots;
    const int e = gld(P.g_ptr, row) + t;
    if (e < e1) {
      const GTap tap = gld(P.g_tap, e);
      gst(out, tap.slot, fmaf(tap.w0, Lf[tap.x0], tap.w1 * Lf[tap.x0 + 1]));
    }
    // further taps four per round, their loads issued together (a row of a
    // planar sensor holds a tap at every node: 16 per lane at 128 points)
    for (int e0 = e + G::T; e0 < e1; e0 += 4 * G::T) {
      GTap tp[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) tp[u] = gld(P.g_tap, e0 + u * G::T < e1 ? e0 + u * G::T : e0);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u * G::T < e1) gst(out, tp[u].slot, fmaf(tp[u].w0, Lf[tp[u].x0], tp[u].w1 * Lf[tp[u].x0 + 1]));
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
    const int g1 = gld(P.s_ptr, row + 1);
    const float* h = P.in + (long)n * P.ns;
    for (int g = gld(P.s_ptr, row) + t; g < g1; g += G::T) {
      const SGroup grp = gld(P.s_grp, g);
      float acc = 0.f;
      for (int e = grp.beg; e < grp.end; ++e) {
        const STap tp = gld(P.s_tap, e);
        acc = fmaf(tp.w, gld(h, tp.s), acc);
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
  // loads are issued for every lane (base is that of a valid row) and
  // zeroed for lanes past the last row: no branch between them
  __device__ __forceinline__ void ld(const float* a, float2 (&v)[E]) const {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const float2 x = ld2(a, base + t + T * m);
      v[m] = valid ? x : f2(0.f, 0.f);
    }
  }
  __device__ __forceinline__ void ld(const float2* a, float2 (&v)[E]) const {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const float2 x = gld(a, base + t + T * m);
      v[m] = valid ? x : f2(0.f, 0.f);
    }
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

// One row pass of kind K over the row tile `tile` of instance P (ROWS rows
// of T lanes each, ROWS * T threads), at forward step / adjoint iteration
// `it`; lds holds ROWS * LDR values, tws the block's twiddles.
template <int N, int D, int K, int ROWS>
__device__ __forceinline__ void row_pass(const DevPlan& P, int tile, int it, float2* lds, RowTw<N>& tws) {
  using G = RowGeo<N>;
  constexpr int M = G::M, E = G::E, T = G::T;
  const int rl = threadIdx.x / T, t = threadIdx.x % T;
  const int row = tile * ROWS + rl;
  const bool valid = row < P.nrows;
  const int rowc = valid ? row : 0;
  const int ny = P.n[1];
  const int yy = rowc % ny, zz = rowc / ny;
  float2* L = lds + rl * G::LDR;
  float* Lf = reinterpret_cast<float*>(L);
  const RowIo<N> io{(long)rowc * M, t, valid};

  // per-row PML factors of the y and z axes
  float qrow[3] = {1.f, gld(P.Q[1], yy), 1.f};
  float qsrow[3] = {1.f, gld(P.Qsg[1], yy), 1.f};
  if constexpr (D == 3) {
    qrow[2] = gld(P.Q[2], zz);
    qsrow[2] = gld(P.Qsg[2], zz);
  }
  auto qpair = [&](int j, const float2& qx) { return j == 0 ? qx : f2(qrow[j], qrow[j]); };
  auto qspair = [&](int j, const float2& qx) { return j == 0 ? qx : f2(qsrow[j], qsrow[j]); };

  if constexpr (K == R_FWD_INIT || K == R_FWD_INIT_F) {
    float2 p[E], ic[E];
    if constexpr (K == R_FWD_INIT) io.ld(P.in, p);
    else io.ld(P.S[0], p);  // the windowed spectrum of p0
    io.ld(P.inv_dc2, ic);
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
    if constexpr (K == R_FWD_INIT_F) {
      c2r<N>(p, L, t, tws);  // the smoothed p0 (the window pass holds the 1/N)
      WaveSync::sync();
    }
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
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
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
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
#pragma unroll
    for (int j = 0; j < D; ++j) c2r<N>(g[j], L, t, tws);
#pragma unroll
    for (int j = 0; j < D; ++j) io.ld(P.r[j], r[j]);
    io.ld(P.dtr0, dr);
    if constexpr (K == R_FWD_2LL) io.ld(P.c2, c2);
    io.ldx(P.Q[0], qx);
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
    float2 a1[E], a2[E], rs[E], c2[E];
    io.ld(P.S[1], a1);
    io.ld(P.S[2], a2);
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
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
    // p = c0^2 sum rho + c0^2 tau A1 - c0^2 eta A2, term by term so that no
    // more than one coefficient array is live at a time
    if (P.alpha_uniform) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        float2 ct[1], ce[1];
        const float2 cm[1] = {c2[m]};
        absorption_coefs<1>(P, cm, ct, ce);
        a1[m] = mul2(c2[m], rs[m]) + mul2(ct[0], a1[m]) - mul2(ce[0], a2[m]);
      }
    } else {
      float2 cf[E];
      io.ld(P.c2tau, cf);
#pragma unroll
      for (int m = 0; m < E; ++m) a1[m] = mul2(c2[m], rs[m]) + mul2(cf[m], a1[m]);
      io.ld(P.c2eta, cf);
#pragma unroll
      for (int m = 0; m < E; ++m) a1[m] = a1[m] - mul2(cf[m], a2[m]);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) {
      if (valid) check_finite(P, a1[m]);
      L[t + T * m] = a1[m];
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
    // W^T h[nsamp] for this row: the sums of the row's node groups, formed
    // before the time loop (k_scatter_sums).  The group range is loaded with
    // the pass's inputs, this lane's first group and its sum once they have
    // arrived, so that those loads complete during the transform.
    int sp0 = 0, sp1 = 0;
    if (valid) {
      sp0 = gld(P.s_ptr, rowc) + t;
      sp1 = gld(P.s_ptr, rowc + 1);
    }
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
    const float* sc = P.sc + (long)nsamp * P.ngroups;
    int sx = -1;
    float sv = 0.f;
    if (valid && sp0 < sp1) {
      sx = gld(P.s_grp, sp0).x;
      sv = gld(sc, sp0);
    }
    if (!first) c2r<N>(v, L, t, tws);
#pragma unroll
    for (int m = 0; m < E; ++m) L[t + T * m] = v[m];
    WaveSync::sync();
    if (sx >= 0) {
      Lf[sx] += sv;
      // the remaining groups four per round, their loads issued together
      for (int g0 = sp0 + T; g0 < sp1; g0 += 4 * T) {
        int gx[4];
        float gs[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int g = g0 + u * T < sp1 ? g0 + u * T : sp0;
          gx[u] = gld(P.s_grp, g).x;
          gs[u] = gld(sc, g);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (g0 + u * T < sp1) Lf[gx[u]] += gs[u];
      }
    }
    WaveSync::sync();
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
    float2 a2[E], a1[E], q[E], dr[E], qx[E];
    io.ld(P.S[1], a2);
    io.ld(P.S[2], a1);
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
    c2r<N>(a2, L, t, tws);
    c2r<N>(a1, L, t, tws);
    io.ld(P.q, q);
    io.ld(P.dtr0, dr);
    io.ldx(P.Q[0], qx);
#pragma unroll
    for (int m = 0; m < E; ++m) a2[m] = q[m] - a2[m];  // q - A2, shared by every axis
    // one axis component at a time: its density, then its transform
#pragma unroll
    for (int j = 0; j < D; ++j) {
      float2 rb[E], g[E];
      if (first) io.zero(rb); else io.ld(P.r[j], rb);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const float2 qq = qpair(j, qx[m]);
        const float2 r1 = rb[m] + a2[m];
        g[m] = mul2(dr[m], a1[m] - mul2(qq, r1));
        rb[m] = mul2(mul2(qq, qq), r1);
      }
      io.st(P.r[j], rb);
      r2c<N>(g, P.S[1 + j] + io.base, L, t, valid, tws);
    }
  } else if constexpr (K == R_ATD_2 || K == R_ATD_2LL) {
    // adjoint-then-discretize step `it` (adjoint time it dt, forward time
    // T - it dt): rho*_j <- Q_j (Q_j rho*_j + rho0 (sigma / d - dt g_j)) with
    // sigma = (W^T h[nt-1-it] + W^T h[nt-2-it]) / 2; lossy: S1 <- F_x(c0^2 tau
    // (sigma - dt sum g)) and S2 <- F_x(c0^2 eta / rho0 sum rho*) for the
    // absorption pass; lossless: S0 <- F_x(c0^2 sum rho*)
    const bool first = (it == 0);
    float2 g[D][E], r[D][E], dr[E], c2[E], qx[E];
#pragma unroll
    for (int j = 0; j < D; ++j) io.ld(P.S[1 + j], g[j]);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (first) io.zero(r[j]); else io.ld(P.r[j], r[j]);
    }
    io.ld(P.dtr0, dr);
    io.ld(P.c2, c2);
    io.ldx(P.Q[0], qx);
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
#pragma unroll
    for (int j = 0; j < D; ++j) c2r<N>(g[j], L, t, tws);
#pragma unroll
    for (int m = 0; m < E; ++m) L[t + T * m] = f2(0.f, 0.f);
    scatter_row<N>(P, P.nt - 1 - it, Lf, rowc, t, valid);
    scatter_row<N>(P, P.nt - 2 - it, Lf, rowc, t, valid);
    float2 sg[E], sdiv[E], srho[E];
#pragma unroll
    for (int m = 0; m < E; ++m) sg[m] = 0.5f * L[t + T * m];
    WaveSync::sync();
    const float invd = 1.0f / (float)D;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const float2 r0 = P.inv_dt * dr[m];  // rho0
      const float2 src = mul2(r0, invd * sg[m]);
      sdiv[m] = f2(0.f, 0.f);
      srho[m] = f2(0.f, 0.f);
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const float2 q = qpair(j, qx[m]);
        r[j][m] = mul2(q, mul2(q, r[j][m]) + src - mul2(dr[m], g[j][m]));
        sdiv[m] = sdiv[m] + g[j][m];
        srho[m] = srho[m] + r[j][m];
      }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) io.st(P.r[j], r[j]);
    if constexpr (K == R_ATD_2) {
      float2 ct[E], ce[E];
      if (P.alpha_uniform) {
        absorption_coefs<E>(P, c2, ct, ce);
      } else {
        io.ld(P.c2tau, ct);
        io.ld(P.c2eta, ce);
      }
#pragma unroll
      for (int m = 0; m < E; ++m) {
        sdiv[m] = mul2(ct[m], sg[m] - P.dt * sdiv[m]);
        srho[m] = mul2(ce[m], f2(P.dt * srho[m].x / dr[m].x, P.dt * srho[m].y / dr[m].y));
      }
      r2c<N>(sdiv, P.S[1] + io.base, L, t, valid, tws);
      r2c<N>(srho, P.S[2] + io.base, L, t, valid, tws);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) srho[m] = mul2(c2[m], srho[m]);
      r2c<N>(srho, P.S[0] + io.base, L, t, valid, tws);
    }
  } else if constexpr (K == R_ATD_3) {
    // p* = c0^2 sum rho* - rho0 (A1 + A2), the fractional Laplacians already
    // applied to c0^2 tau (...) and c0^2 eta / rho0 (...) (statea); S0 <- F_x p*
    float2 a1[E], a2[E], rs[E], c2[E], dr[E];
    io.ld(P.S[1], a1);
    io.ld(P.S[2], a2);
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
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
    io.ld(P.dtr0, dr);
#pragma unroll
    for (int m = 0; m < E; ++m) a1[m] = mul2(c2[m], rs[m]) - mul2(P.inv_dt * dr[m], a1[m] + a2[m]);
    r2c<N>(a1, P.S[0] + io.base, L, t, valid, tws);
  } else if constexpr (K == R_ATD_FINAL) {
    // image = sum_j rho*_j / rho0 (eq. adjj), rho0 = (dt rho0) / dt
    float2 rs[E], dr[E];
    io.ld(P.r[0], rs);
#pragma unroll
    for (int j = 1; j < D; ++j) {
      float2 rj[E];
      io.ld(P.r[j], rj);
#pragma unroll
      for (int m = 0; m < E; ++m) rs[m] = rs[m] + rj[m];
    }
    io.ld(P.dtr0, dr);
#pragma unroll
    for (int m = 0; m < E; ++m) rs[m] = f2(P.dt * rs[m].x / dr[m].x, P.dt * rs[m].y / dr[m].y);
    io.st(P.out, rs);
  } else if constexpr (K == R_FILT_IN || K == R_FILT_RE) {
    // x-spectrum of a real field: p0 (forward) or the image (adjoint)
    float2 v[E];
    io.ld(K == R_FILT_IN ? P.in : P.out, v);
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
    r2c<N>(v, P.S[0] + io.base, L, t, valid, tws);
  } else if constexpr (K == R_FILT_OUT) {
    float2 v[E];
    io.ld(P.S[0], v);
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
    c2r<N>(v, L, t, tws);
    io.st(P.out, v);
  } else if constexpr (K == R_EOS_FWD_IN || K == R_EOS_FWD || K == R_EOS_ADJ_IN || K == R_EOS_ADJ) {
    // eta = (c0^2 eta) / c0^2 at this row's points
    auto eta_row = [&](float2 (&e)[E]) {
      float2 c2[E], ce[E];
      io.ld(P.c2, c2);
      if (P.alpha_uniform) {
        float2 ct[E];
        absorption_coefs<E>(P, c2, ct, ce);
      } else {
        io.ld(P.c2eta, ce);
      }
#pragma unroll
      for (int m = 0; m < E; ++m) e[m] = f2(ce[m].x / c2[m].x, ce[m].y / c2[m].y);
    };
    const bool last = (it == 1);
    float2 x[E];
    if constexpr (K == R_EOS_FWD_IN) {
      io.ld(P.r[0], x);
    } else if constexpr (K == R_EOS_ADJ_IN) {
      io.ld(P.r[0], x);
#pragma unroll
      for (int j = 1; j < D; ++j) {
        float2 rj[E];
        io.ld(P.r[j], rj);
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = x[m] + rj[m];
      }
#pragma unroll
      for (int m = 0; m < E; ++m) x[m] = (1.f / (float)D) * x[m];
      io.st(P.q, x);
      io.st(P.r[0], x);
    } else {
      io.ld(P.S[1], x);
    }
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
    if constexpr (K == R_EOS_FWD || K == R_EOS_ADJ) {
      // x <- b + [eta] F_x^-1 S1, b = r_1 (forward: p0 / (d c0^2)) or q
      c2r<N>(x, L, t, tws);
      float2 b[E];
      io.ld(K == R_EOS_FWD ? P.r[1] : P.q, b);
      if constexpr (K == R_EOS_FWD) {
        float2 e[E];
        eta_row(e);
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = b[m] + mul2(e[m], x[m]);
      } else {
#pragma unroll
        for (int m = 0; m < E; ++m) x[m] = b[m] + x[m];
      }
      if (last) {
        if constexpr (K == R_EOS_FWD) {
#pragma unroll
          for (int j = 0; j < D; ++j) io.st(P.r[j], x);
        } else {
          float2 z[E];
#pragma unroll
          for (int m = 0; m < E; ++m) {
            z[m] = f2(0.f, 0.f);
            x[m] = (float)D * x[m];
          }
          io.st(P.r[0], x);
#pragma unroll
          for (int j = 1; j < D; ++j) io.st(P.r[j], z);
        }
        return;  // block-uniform (it)
      }
      io.st(P.r[0], x);
    }
    // S1 <- F_x x (forward) or F_x (eta x) (adjoint)
    if constexpr (K == R_EOS_ADJ_IN || K == R_EOS_ADJ) {
      float2 e[E];
      eta_row(e);
#pragma unroll
      for (int m = 0; m < E; ++m) x[m] = mul2(e[m], x[m]);
    }
    WaveSync::sync();
    r2c<N>(x, P.S[1] + io.base, L, t, valid, tws);
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
    load_row_twiddles<N, ROWS * T>(tws, g_tw);  // after the pass's own loads
    __syncthreads();
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

}  // namespace pat
