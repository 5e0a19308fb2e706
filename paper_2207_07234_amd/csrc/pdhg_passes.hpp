// Device bodies of the three fused passes of one iteration of Algorithm 1
// (Section 3.3), shared by the single-problem kernels (pdhg_fused.hip) and the
// batched persistent kernels (pdhg_batch.hip).
//
//   A  dual_fft_pair     one pair of dual rows: inverse FFT of the
//                        preconditioned residual, dual step and extrapolation
//   B  primal_res_pair   one pair of implicit rows: primal step on the levels
//                        the rows touch, dual residual of the owned levels,
//                        implicit residual of the two rows and its forward FFT
//   C  colsolve_group    eight halfcomplex spectrum columns: banded Cholesky
//                        solve along t (the preconditioner K_d^{-1}, Section 2.2)
//
// A and B run on a sub-group of W threads (tid = 0..W-1, a multiple of 64) of a
// block of TB threads (gtid = 0..TB-1); all sub-groups of a block work on rows
// of the same length nx, share the LDS twiddle table, and call the bodies
// together (the FFT synchronises the whole block).  A pair whose first row is
// >= nt is idle: it takes part in the barriers and stores nothing.
#pragma once

#include <type_traits>

#include "pdhg_device.hpp"

namespace pdhg {

// ------------------------------------------------------------------ A
// EPT = nx / W points per thread.  All global loads (twiddles, the two spectrum
// rows and the two dual rows) are issued before the first LDS write so that
// their latencies overlap.  S is the type of the spectrum and of the FFT (T,
// or float under an FP64 state with a single-precision preconditioner).
template <typename T, int EPT, typename S = T>
__device__ __forceinline__ void dual_fft_pair(const S* __restrict__ spec, int nt, int lqb, int nx,
                                              const C2<S>* __restrict__ tw, T* __restrict__ phi,
                                              T* __restrict__ phibar, T tau, int a, int tid, int W, int gtid, int TB,
                                              C2<S>* buf, C2<S>* twl, C2<S>* alt = nullptr,
                                              const T* __restrict__ s0 = nullptr) {
  const int b = a + 1;
  const bool act = a < nt, hasb = b < nt;
  const int half = nx >> 1;
  const int ar = act ? a : 0, br = hasb ? b : 0;
  T* pa = phi + (size_t)ar * nx;
  T* qa = phibar + (size_t)ar * nx;
  T* pb = phi + (size_t)br * nx;
  T* qb = phibar + (size_t)br * nx;
  // ---- loads
  C2<S> twv[EPT];
  T fa[EPT], fb[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int xt = gtid + e * TB;
    twv[e] = (xt < nx) ? tw[xt] : C2<S>{S(0), S(0)};
    const int x = tid + e * W;
    fa[e] = act ? pa[x] : T(0);
    fb[e] = hasb ? pb[x] : T(0);
  }
  // halfcomplex pair: thread handles modes k = tid + e W, k <= nx/2 (EPT/2 + 1 of them)
  constexpr int KPT = EPT / 2 + 1;
  S sar[KPT], sai[KPT], sbr[KPT], sbi[KPT];
#pragma unroll
  for (int e = 0; e < KPT; ++e) {
    const int k = tid + e * W;
    sar[e] = sai[e] = sbr[e] = sbi[e] = S(0);
    if (act && k <= half) {
      if (k == 0 || k == half) {
        const int q = (k == 0) ? 0 : 1;
        if (k == half || !s0) {
          sar[e] = spec[spec_index(a, q, nt, lqb)];
          if (hasb) sbr[e] = spec[spec_index(b, q, nt, lqb)];
        }
      } else {
        sar[e] = spec[spec_index(a, 2 * k, nt, lqb)];
        sai[e] = spec[spec_index(a, 2 * k + 1, nt, lqb)];
        if (hasb) {
          sbr[e] = spec[spec_index(b, 2 * k, nt, lqb)];
          sbi[e] = spec[spec_index(b, 2 * k + 1, nt, lqb)];
        }
      }
    }
  }
  // ---- LDS: twiddles and Z_k = A_k + i B_k (A_{N-k} = conj A_k)
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int xt = gtid + e * TB;
    if (xt < nx) twl[lpad(xt)] = twv[e];
  }
#pragma unroll
  for (int e = 0; e < KPT; ++e) {
    const int k = tid + e * W;
    if (k <= half) {
      buf[lpad(k)] = {sar[e] - sbi[e], sai[e] + sbr[e]};
      if (k != 0 && k != half) buf[lpad(nx - k)] = {sar[e] + sbi[e], sbr[e] - sai[e]};
    }
  }
  const C2<S>* res = fft_lds<true, EPT>(buf, nx, twl, tid, W, alt);
  const S sc = S(1) / S(nx);
  // with s0: the row means (mode 0) come from s0 in T, not from the float FFT
  const T inv_nx = T(1) / T(nx);
  const T ma = (s0 && act) ? s0[a] * inv_nx : T(0), mb = (s0 && hasb) ? s0[b] * inv_nx : T(0);
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int x = tid + e * W;
    const C2<S> z = res[lpad(x)];
    if (act) {
      const T ta = tau * (T(z.x * sc) + ma);
      const T p = fa[e] + ta;
      pa[x] = p;
      qa[x] = p + ta;
    }
    if (hasb) {
      const T tb = tau * (T(z.y * sc) + mb);
      const T q = fb[e] + tb;
      pb[x] = q;
      qb[x] = q + tb;
    }
  }
}

// ------------------------------------------------------------------ B
// Load one row for this lane (x = seg0 + lane + 64 e) and the two values just
// outside the wave's segment; rows outside [0, nrows) read as zero.
template <typename T, int E>
__device__ __forceinline__ void load_row_wave(const T* __restrict__ base, int r, int nrows, int nx, int seg0,
                                              int lane, T* v, T& prev, T& next) {
  if (r < 0 || r >= nrows) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = T(0);
    prev = next = T(0);
    return;
  }
  const T* row = base + (size_t)r * nx;
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = row[seg0 + lane + 64 * e];
  prev = row[(seg0 - 1) & (nx - 1)];
  next = row[(seg0 + 64 * E) & (nx - 1)];
}

// J(u)^T psi at unknown level m from registers: c = psi^{m-1} (with segment
// edges), t1 = psi^m, t2 = psi^{m+1} (zero where absent), uv = u^m.
template <typename T, int E>
__device__ __forceinline__ void dual_op_regs(const Consts<T>& C, int m, const T* c, T prev, T next, const T* t1,
                                             const T* t2, const T* uv, T* out) {
  T cm[E], cp[E];
  wave_row_neighbours<T, E>(c, prev, next, cm, cp);
#pragma unroll
  for (int e = 0; e < E; ++e) out[e] = C.JtTime(m, c[e], t1[e], t2[e]) + C.JtF(uv[e], cm[e], c[e], cp[e]);
}

// E = nx / W points per thread; wave v of the sub-group owns x in
// [v 64E, (v+1) 64E), lane l element e at x = v 64E + l + 64 e.  The pair
// reads u^{n-1} on levels a-1..a+2, phibar on rows a-2..a+3 and phi on rows
// a..a+3.  STREAM = false: every row is loaded up front, so that all load
// latencies overlap (a block that has its CU to itself).  STREAM = true: the
// levels are stepped in order and each step loads the rows of the next one,
// so that only a sliding window of rows is held in registers (fewer VGPRs, so
// that several blocks share a CU and hide each other's latencies).  The
// arithmetic is the same either way.  Returns this thread's contributions to
// ||A(u^n)||^2 (rows a, a+1) and ||J(u^{n-1})^T phi^{n-1}||^2 (levels a+1, a+2).
// edge: 4 (W / 64) values of LDS for this sub-group.  alt (optional): a second
// N-point LDS array for the FFT.  wsum (optional, 2 W / 64 doubles of LDS): the
// per-wave sums of the two contributions, stored before the FFT.
template <typename T, int E, typename S = T, bool STREAM = false>
__device__ __forceinline__ void primal_res_pair(const Consts<T>& C, const T* __restrict__ u_in,
                                                T* __restrict__ u_out, const T* __restrict__ phibar,
                                                const T* __restrict__ phi, T tau_u, S* __restrict__ spec, int lqb,
                                                const C2<S>* __restrict__ tw, int a, int tid, int W, int gtid,
                                                int TB, C2<S>* buf, C2<S>* twl, T* edge, double& rp_out,
                                                double& rd_out, C2<S>* alt = nullptr, double* wsum = nullptr,
                                                bool want_rd = true, const LamArgs<T>* lam = nullptr) {
  const int nx = C.nx, nt = C.nt;
  const int lane = tid & 63, wv = tid >> 6, nw = W >> 6;
  const int seg0 = wv * 64 * E;
  const int b = a + 1;
  const bool act = a < nt;
  const bool bdf2 = C.time == kTimeBDF2;
  // ---- all global loads first
  C2<S> twv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int xt = gtid + e * TB;
    twv[e] = (xt < nx) ? tw[xt] : C2<S>{S(0), S(0)};
  }
  T U0[4][E], U[4][E];                 // u^{n-1} and u^n on levels a-1+i
  T PB[6][E], PBp[4], PBn[4];          // phibar rows a-2+j (edges for j = 0..3)
  T PH[4][E], PHp[2], PHn[2];          // phi rows a+j (edges for j = 0, 1)
  auto load_u0 = [&](int i) __attribute__((always_inline)) {
    const int m = a - 1 + i;
    const bool ok = m >= 0 && m <= nt && (bdf2 || i > 0);
#pragma unroll
    for (int e = 0; e < E; ++e) U0[i][e] = ok ? u_in[(size_t)m * nx + seg0 + lane + 64 * e] : T(0);
  };
  auto load_pb = [&](int j) __attribute__((always_inline)) {
    T pv, nv;
    load_row_wave<T, E>(phibar, a - 2 + j, nt, nx, seg0, lane, PB[j], pv, nv);
    if (j < 4) { PBp[j] = pv; PBn[j] = nv; }
  };
  auto load_ph = [&](int j) __attribute__((always_inline)) {
    T pv, nv;
    load_row_wave<T, E>(phi, a + j, nt, nx, seg0, lane, PH[j], pv, nv);
    if (j < 2) { PHp[j] = pv; PHn[j] = nv; }
  };
  if constexpr (!STREAM) {
#pragma unroll
    for (int i = 0; i < 4; ++i) load_u0(i);
#pragma unroll
    for (int j = 0; j < 6; ++j) load_pb(j);
    if (want_rd) {   // phi is read only for the dual residual
#pragma unroll
      for (int j = 0; j < 4; ++j) load_ph(j);
    }
  } else {
    load_u0(0);
    load_pb(0);
    load_pb(1);
    load_pb(2);
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int xt = gtid + e * TB;
    if (xt < nx) twl[lpad(xt)] = twv[e];
  }
  // ---- primal step on the four levels, dual residual on the two owned ones
  double rd = 0.0, rp = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = a - 1 + i;
    if constexpr (STREAM) {   // the rows of the next level
      if (i + 3 <= 5) load_pb(i + 3);
      if (i + 1 <= 3) load_u0(i + 1);
    }
    if (m < 0 || m > nt || (!bdf2 && i == 0)) continue;
    if (m == 0) {
      if (lam && lam->u0) {   // multiplier form: u^0 and lambda step (this pair holds rows 0 and 1)
        const T c1 = C.c1(0), c2 = C.c2(1);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int x = seg0 + lane + 64 * e;
          const T lb = lam->lambar[x], lo = lam->lam[x];
          U[i][e] = U0[i][e] - lam->tau_u0 * (c1 * PB[i + 1][e] + c2 * PB[i + 2][e] + lb);
          const T dl = lam->tau_lam * (U[i][e] - lam->u0[x]);
          lam->lam[x] = lo + dl;
          lam->lambar[x] = lo + T(2) * dl;
          u_out[x] = U[i][e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) U[i][e] = U0[i][e];
      }
      continue;
    }
    T g[E];
    dual_op_regs<T, E>(C, m, PB[i], PBp[i], PBn[i], PB[i + 1], PB[i + 2], U0[i], g);
#pragma unroll
    for (int e = 0; e < E; ++e) U[i][e] = U0[i][e] - tau_u * g[e];
    if (i >= 2) {   // owned level: store u^n and the dual residual of (u^{n-1}, phi^{n-1})
      T* uw = u_out + (size_t)m * nx + seg0 + lane;
#pragma unroll
      for (int e = 0; e < E; ++e) uw[64 * e] = U[i][e];
      if (!STREAM && want_rd) {
        dual_op_regs<T, E>(C, m, PH[i - 2], PHp[i - 2], PHn[i - 2], PH[i - 1], PH[i], U0[i], g);
#pragma unroll
        for (int e = 0; e < E; ++e) rd += (double)g[e] * (double)g[e];
      }
    }
  }
  if constexpr (STREAM) {
    // the dual residual of the owned levels, from reloaded inputs (u^{n-1} is
    // still intact in u_in); it is needed only near convergence, and holding
    // its four phi rows through the primal step would widen the window
    if (want_rd) {
      load_u0(2);
      load_u0(3);
#pragma unroll
      for (int j = 0; j < 4; ++j) load_ph(j);
#pragma unroll
      for (int i = 2; i < 4; ++i) {
        const int m = a - 1 + i;
        if (m < 1 || m > nt) continue;
        T g[E];
        dual_op_regs<T, E>(C, m, PH[i - 2], PHp[i - 2], PHn[i - 2], PH[i - 1], PH[i], U0[i], g);
#pragma unroll
        for (int e = 0; e < E; ++e) rd += (double)g[e] * (double)g[e];
      }
    }
  }
  // segment-edge values of the two levels whose flux differences are taken
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (lane == 0) edge[(2 * s + 0) * nw + wv] = U[2 + s][0];
    if (lane == 63) edge[(2 * s + 1) * nw + wv] = U[2 + s][E - 1];
  }
  __syncthreads();
  T R[2][E];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int l = a + s;
    if (l < nt) {
      const int ms = 2 + s;
      T vm[E], vp[E];
      const T prev = edge[(2 * s + 1) * nw + ((wv - 1 + nw) % nw)];
      const T next = edge[(2 * s + 0) * nw + ((wv + 1) % nw)];
      wave_row_neighbours<T, E>(U[ms], prev, next, vm, vp);
      const T c0 = C.c0(l), c1 = C.c1(l), c2 = C.c2(l);
      const bool use2 = bdf2 && l >= 1;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        T t = c0 * U[ms][e] + c1 * U[ms - 1][e];
        if (use2) t += c2 * U[ms - 2][e];
        const T r = t * C.inv_ht + C.F(vm[e], U[ms][e], vp[e]);
        R[s][e] = r;
        rp += (double)r * (double)r;
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) R[s][e] = T(0);
    }
  }
  if (wsum) {
    // per-wave sums now (the FFT's barriers publish them); the caller adds
    // them up in wave order, as block_sum_waves would
    const double sp = wave_sum(rp), sd = wave_sum(rd);
    if (lane == 0) {
      wsum[wv] = sp;
      wsum[nw + wv] = sd;
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) buf[lpad(seg0 + lane + 64 * e)] = {S(R[0][e]), S(R[1][e])};
  const C2<S>* res = fft_lds<false, E>(buf, nx, twl, tid, W, alt);
  if (act) store_halfcomplex_pair(res, nx, spec, nt, lqb, a, b < nt, tid, W);
  rp_out = rp;
  rd_out = rd;
}

// Sum of v over the W threads of a sub-group whose first wave is wave w0 of the
// block: wave reductions, then the sub-group's first thread adds the per-wave
// sums in order (the order of block_sum_waves).  Result valid in that thread.
// red: LDS, one double per wave of the block.  All threads of the block call it.
__device__ __forceinline__ double subgroup_sum(double v, double* red, int w0, int nw) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (wid == w0 && lane == 0) {
    // reads issued together (unrolled to 16 waves), added in wave order
    double r[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) r[i] = i < nw ? red[w0 + i] : 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i < nw) s += r[i];
  }
  return s;
}

// ------------------------------------------------------------------ C
// Banded Cholesky solve along t.  One wavefront per halfcomplex column (the
// column's Fourier mode selects the factor; columns 0 and 1 are the real
// columns of modes 0 and nx/2).  Lane j owns levels [j LPL, (j+1) LPL).  Each
// lane computes the affine map of its segment (particular solution and the
// responses to the two incoming values), an inclusive scan of the maps across
// the 64 lanes (shuffles, no barriers) gives every lane its incoming state, and
// the segment is re-run from it.  The block stages a [nt][8-column] tile of the
// spectrum through LDS (lane-major, padded) so that global accesses are
// coalesced and LDS accesses conflict-free.
constexpr int kColCols = 8;                // spectrum columns per block
constexpr int kFdColWaves = kColCols;      // finite differences: one wave per column
constexpr int kColWaves = 4;               // DG: one wave per mode (its Re and Im columns)
constexpr int kColLongLpl = 16;            // levels per lane when a column spans several waves

// (H, P) <- (H, P) o (H', P') : apply (H', P') first, then (H, P).
// Complex value of the full-symbol column solve: the scan helpers below are
// generic in the arithmetic type; cross-lane moves act per component.
template <typename T>
struct Cx {
  T re, im;
  __device__ __forceinline__ Cx() : re(T(0)), im(T(0)) {}
  __device__ __forceinline__ Cx(T r) : re(r), im(T(0)) {}
  __device__ __forceinline__ Cx(T r, T i) : re(r), im(i) {}
};
template <typename T>
__device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ Cx<T> operator-(Cx<T> a) { return {-a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ Cx<T> operator*(Cx<T> a, Cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ Cx<T> operator*(T a, Cx<T> b) { return {a * b.re, a * b.im}; }
template <int CTRL, typename T>
__device__ __forceinline__ Cx<T> dpp_move(Cx<T> v, Cx<T> fill) {
  return {dpp_move<CTRL>(v.re, fill.re), dpp_move<CTRL>(v.im, fill.im)};
}
template <typename T>
__device__ __forceinline__ Cx<T> read_lane(Cx<T> v, int src) { return {read_lane(v.re, src), read_lane(v.im, src)}; }
template <typename T>
__device__ __forceinline__ Cx<T> from_lane_below(Cx<T> v, Cx<T> fill) {
  return {from_lane_below(v.re, fill.re), from_lane_below(v.im, fill.im)};
}
template <typename T>
__device__ __forceinline__ Cx<T> from_lane_above(Cx<T> v, Cx<T> fill) {
  return {from_lane_above(v.re, fill.re), from_lane_above(v.im, fill.im)};
}

template <typename T>
__device__ __forceinline__ void compose(T* H, T* P, const T* H2, const T* P2) {
  const T h0 = H[0] * H2[0] + H[1] * H2[2];
  const T h1 = H[0] * H2[1] + H[1] * H2[3];
  const T h2 = H[2] * H2[0] + H[3] * H2[2];
  const T h3 = H[2] * H2[1] + H[3] * H2[3];
  const T p0 = H[0] * P2[0] + H[1] * P2[1] + P[0];
  const T p1 = H[2] * P2[0] + H[3] * P2[1] + P[1];
  H[0] = h0; H[1] = h1; H[2] = h2; H[3] = h3;
  P[0] = p0; P[1] = p1;
}

// One Kogge-Stone step inside rows of 16 lanes by DPP: compose with the map of
// lane l - D (forward) or l + D (backward); lanes without such a lane in their
// row compose with the identity map.
template <typename T, bool FWD, int D>
__device__ __forceinline__ void scan_step_row(T* H, T* P) {
  constexpr int CTRL = FWD ? (0x110 + D) : (0x100 + D);
  T H2[4], P2[2];
  H2[0] = dpp_move<CTRL>(H[0], T(1));
  H2[1] = dpp_move<CTRL>(H[1], T(0));
  H2[2] = dpp_move<CTRL>(H[2], T(0));
  H2[3] = dpp_move<CTRL>(H[3], T(1));
  P2[0] = dpp_move<CTRL>(P[0], T(0));
  P2[1] = dpp_move<CTRL>(P[1], T(0));
  compose(H, P, H2, P2);
}

// Combine row `row` with the prefix held by lane `src` (read as a uniform value).
template <typename T>
__device__ __forceinline__ void scan_step_cross(T* H, T* P, int lane, int row, int src) {
  T H2[4], P2[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) H2[k] = read_lane(H[k], src);
  P2[0] = read_lane(P[0], src);
  P2[1] = read_lane(P[1], src);
  if ((lane >> 4) == row) compose(H, P, H2, P2);
}

// Inclusive scan of segment maps over the 64 lanes, forward (from lane 0) or
// backward (from lane 63); returns the state entering this lane's segment.
// Within each row of 16 lanes: DPP row shifts by 1, 2, 4, 8 (VALU, no LDS);
// across rows: each row in turn composes with the full prefix of the rows
// before it (forward) or after it (backward), read from one lane.
template <typename T, bool FWD>
__device__ __forceinline__ void scan_inclusive(T* H, T* P, int lane) {
  scan_step_row<T, FWD, 1>(H, P);
  scan_step_row<T, FWD, 2>(H, P);
  scan_step_row<T, FWD, 4>(H, P);
  scan_step_row<T, FWD, 8>(H, P);
  if (FWD) {
    scan_step_cross(H, P, lane, 1, 15);
    scan_step_cross(H, P, lane, 2, 31);
    scan_step_cross(H, P, lane, 3, 47);
  } else {
    scan_step_cross(H, P, lane, 2, 48);
    scan_step_cross(H, P, lane, 1, 32);
    scan_step_cross(H, P, lane, 0, 16);
  }
}

template <typename T, bool FWD>
__device__ __forceinline__ void scan_incoming(T* H, T* P, int lane, T& in2, T& in1) {
  scan_inclusive<T, FWD>(H, P, lane);
  if (FWD) {
    in2 = from_lane_below(P[0], T(0));
    in1 = from_lane_below(P[1], T(0));
  } else {
    in2 = from_lane_above(P[0], T(0));
    in1 = from_lane_above(P[1], T(0));
  }
}

// The same for four independent 16-lane columns per wavefront (one DPP row
// each): only the row steps; the first lane of each column (forward) or its
// last lane (backward) enters with zero.
template <typename T, bool FWD>
__device__ __forceinline__ void scan_incoming_quarter(T* H, T* P, int lane, T& in2, T& in1) {
  scan_step_row<T, FWD, 1>(H, P);
  scan_step_row<T, FWD, 2>(H, P);
  scan_step_row<T, FWD, 4>(H, P);
  scan_step_row<T, FWD, 8>(H, P);
  const bool edge = FWD ? ((lane & 15) == 0) : ((lane & 15) == 15);
  if (FWD) {
    in2 = from_lane_below(P[0], T(0));
    in1 = from_lane_below(P[1], T(0));
  } else {
    in2 = from_lane_above(P[0], T(0));
    in1 = from_lane_above(P[1], T(0));
  }
  if (edge) {
    in2 = T(0);
    in1 = T(0);
  }
}

// The same over a column shared by WPC consecutive waves of the block (wave j
// of the column holds lanes 64 j .. 64 j + 63 of it): each wave's inclusive
// scan, then the wave totals (the map of its last lane forward, of its first
// lane backward) are exchanged through LDS (xch: 6 values per wave of the
// block) and each wave applies the totals of the waves before it (forward) or
// after it (backward) to the zero state; the lane's exclusive prefix map,
// applied to that state, gives the state entering its segment.
template <typename T, bool FWD, int WPC>
__device__ __forceinline__ void scan_incoming_multi(T* H, T* P, int lane, int wv, T* xch, T& in2, T& in1) {
  scan_inclusive<T, FWD>(H, P, lane);
  if (lane == (FWD ? 63 : 0)) {
#pragma unroll
    for (int k = 0; k < 4; ++k) xch[wv * 6 + k] = H[k];
    xch[wv * 6 + 4] = P[0];
    xch[wv * 6 + 5] = P[1];
  }
  __syncthreads();
  const int j = wv % WPC, w0 = wv - j;
  T s2 = 0, s1 = 0;
#pragma unroll
  for (int jj = 0; jj < WPC; ++jj) {
    const int src = FWD ? jj : WPC - 1 - jj;   // waves nearer the column's start first
    if (FWD ? (src < j) : (src > j)) {
      const T* X = xch + (w0 + src) * 6;
      const T n2 = X[0] * s2 + X[1] * s1 + X[4];
      const T n1 = X[2] * s2 + X[3] * s1 + X[5];
      s2 = n2;
      s1 = n1;
    }
  }
  __syncthreads();   // xch is reused by the next scan
  T E[4], F[2];
  if (FWD) {
    E[0] = from_lane_below(H[0], T(1));
    E[1] = from_lane_below(H[1], T(0));
    E[2] = from_lane_below(H[2], T(0));
    E[3] = from_lane_below(H[3], T(1));
    F[0] = from_lane_below(P[0], T(0));
    F[1] = from_lane_below(P[1], T(0));
  } else {
    E[0] = from_lane_above(H[0], T(1));
    E[1] = from_lane_above(H[1], T(0));
    E[2] = from_lane_above(H[2], T(0));
    E[3] = from_lane_above(H[3], T(1));
    F[0] = from_lane_above(P[0], T(0));
    F[1] = from_lane_above(P[1], T(0));
  }
  in2 = E[0] * s2 + E[1] * s1 + F[0];
  in1 = E[2] * s2 + E[3] * s1 + F[1];
}

// The same for two independent 32-lane columns per wavefront (lanes 0..31 and
// 32..63): the row steps never cross a row, and across rows only row 1 (row 3)
// composes with the prefix ending in lane 15 (47), forward, or row 0 (row 2)
// with the suffix starting in lane 16 (48), backward.  The first lane of each
// column (forward) or its last lane (backward) enters with zero.
template <typename T>
__device__ __forceinline__ void scan_cross_half(T* H, T* P, int lane, bool fwd) {
  const int sa = fwd ? 15 : 16, sb = fwd ? 47 : 48;
  T Ha[4], Pa[2], Hb[4], Pb[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    Ha[k] = read_lane(H[k], sa);
    Hb[k] = read_lane(H[k], sb);
  }
  Pa[0] = read_lane(P[0], sa);
  Pa[1] = read_lane(P[1], sa);
  Pb[0] = read_lane(P[0], sb);
  Pb[1] = read_lane(P[1], sb);
  const int row = lane >> 4;
  if (row == (fwd ? 1 : 0)) compose(H, P, Ha, Pa);
  if (row == (fwd ? 3 : 2)) compose(H, P, Hb, Pb);
}

template <typename T, bool FWD>
__device__ __forceinline__ void scan_incoming_half(T* H, T* P, int lane, T& in2, T& in1) {
  scan_step_row<T, FWD, 1>(H, P);
  scan_step_row<T, FWD, 2>(H, P);
  scan_step_row<T, FWD, 4>(H, P);
  scan_step_row<T, FWD, 8>(H, P);
  scan_cross_half(H, P, lane, FWD);
  const bool edge = FWD ? ((lane & 31) == 0) : ((lane & 31) == 31);
  if (FWD) {
    in2 = from_lane_below(P[0], T(0));
    in1 = from_lane_below(P[1], T(0));
  } else {
    in2 = from_lane_above(P[0], T(0));
    in1 = from_lane_above(P[1], T(0));
  }
  if (edge) {
    in2 = T(0);
    in1 = T(0);
  }
}

// Solve L M y = z in place for NC columns sharing the coefficient rows, L lower
// triangular (inverse diagonal invd, sub-diagonals e1, e2) and M = the upper
// triangular with inverse diagonal invb and the transposed sub-diagonals; z[c][i]
// is level l0 + i of column c.  L L^T (Cholesky factor) is invb = invd.  T is
// the value type (real, or Cx for complex right-hand sides and diagonals), E
// the type of the sub-diagonals.
template <typename T, typename E, int BW, int LPL, int NC, int CW = 64>
__device__ __forceinline__ void tri_solve_wave(T (&z)[NC][LPL], const T* invd, const T* invb, const E* e1,
                                               const E* e2, int lane, int l0, int nt) {
  // forward: z_l = invd_l (rhs_l - e1_l z_{l-1} - e2_l z_{l-2})
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    T p2 = 0, p1 = 0, a2 = 1, a1 = 0, b2 = 0, b1 = 1;
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
      if (l0 + i < nt) {
        const T pz = invd[i] * (z[c][i] - e1[i] * p1 - (BW == 2 ? e2[i] * p2 : T(0)));
        const T az = invd[i] * (-(e1[i] * a1) - (BW == 2 ? e2[i] * a2 : T(0)));
        const T bz = invd[i] * (-(e1[i] * b1) - (BW == 2 ? e2[i] * b2 : T(0)));
        p2 = p1; p1 = pz; a2 = a1; a1 = az; b2 = b1; b1 = bz;
      }
    }
    T H[4] = {a2, b2, a1, b1}, P[2] = {p2, p1};
    T zm2, zm1;
    if (CW == 64) scan_incoming<T, true>(H, P, lane, zm2, zm1);
    else if (CW == 32) scan_incoming_half<T, true>(H, P, lane, zm2, zm1);
    else scan_incoming_quarter<T, true>(H, P, lane, zm2, zm1);
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
      if (l0 + i < nt) {
        const T zz = invd[i] * (z[c][i] - e1[i] * zm1 - (BW == 2 ? e2[i] * zm2 : T(0)));
        z[c][i] = zz;
        zm2 = zm1; zm1 = zz;
      }
    }
  }
  // backward: y_l = invb_l (z_l - e1_{l+1} y_{l+1} - e2_{l+2} y_{l+2})
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    T p2 = 0, p1 = 0, a2 = 1, a1 = 0, b2 = 0, b1 = 1;
#pragma unroll
    for (int ii = 0; ii < LPL; ++ii) {
      const int i = LPL - 1 - ii;
      if (l0 + i < nt) {
        const E f1 = e1[i + 1], f2 = (BW == 2) ? e2[i + 2] : E(0);
        const T pz = invb[i] * (z[c][i] - f1 * p1 - f2 * p2);
        const T az = invb[i] * (-(f1 * a1) - f2 * a2);
        const T bz = invb[i] * (-(f1 * b1) - f2 * b2);
        p2 = p1; p1 = pz; a2 = a1; a1 = az; b2 = b1; b1 = bz;
      }
    }
    T H[4] = {a2, b2, a1, b1}, P[2] = {p2, p1};
    T ym2, ym1;
    if (CW == 64) scan_incoming<T, false>(H, P, lane, ym2, ym1);
    else if (CW == 32) scan_incoming_half<T, false>(H, P, lane, ym2, ym1);
    else scan_incoming_quarter<T, false>(H, P, lane, ym2, ym1);
#pragma unroll
    for (int ii = 0; ii < LPL; ++ii) {
      const int i = LPL - 1 - ii;
      if (l0 + i < nt) {
        const E f1 = e1[i + 1], f2 = (BW == 2) ? e2[i + 2] : E(0);
        const T yy = invb[i] * (z[c][i] - f1 * ym1 - f2 * ym2);
        z[c][i] = yy;
        ym2 = ym1; ym1 = yy;
      }
    }
  }
}

// Solve L L^T y = z in place (banded Cholesky factor L) for one column per
// lane group of WPC waves (64 WPC lanes, LPL levels each); every wave of the
// block takes part in both exchanges.
template <typename T, int BW, int LPL, int WPC>
__device__ __forceinline__ void cholesky_solve_multi(T (&z)[LPL], const T* invd, const T* e1, const T* e2, int lane,
                                                     int wv, int l0, int nt, T* xch) {
  {
    T p2 = 0, p1 = 0, a2 = 1, a1 = 0, b2 = 0, b1 = 1;
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
      if (l0 + i < nt) {
        const T pz = invd[i] * (z[i] - e1[i] * p1 - (BW == 2 ? e2[i] * p2 : T(0)));
        const T az = invd[i] * (-(e1[i] * a1) - (BW == 2 ? e2[i] * a2 : T(0)));
        const T bz = invd[i] * (-(e1[i] * b1) - (BW == 2 ? e2[i] * b2 : T(0)));
        p2 = p1; p1 = pz; a2 = a1; a1 = az; b2 = b1; b1 = bz;
      }
    }
    T H[4] = {a2, b2, a1, b1}, P[2] = {p2, p1};
    T zm2, zm1;
    scan_incoming_multi<T, true, WPC>(H, P, lane, wv, xch, zm2, zm1);
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
      if (l0 + i < nt) {
        const T zz = invd[i] * (z[i] - e1[i] * zm1 - (BW == 2 ? e2[i] * zm2 : T(0)));
        z[i] = zz;
        zm2 = zm1; zm1 = zz;
      }
    }
  }
  {
    T p2 = 0, p1 = 0, a2 = 1, a1 = 0, b2 = 0, b1 = 1;
#pragma unroll
    for (int ii = 0; ii < LPL; ++ii) {
      const int i = LPL - 1 - ii;
      if (l0 + i < nt) {
        const T f1 = e1[i + 1], f2 = (BW == 2) ? e2[i + 2] : T(0);
        const T pz = invd[i] * (z[i] - f1 * p1 - f2 * p2);
        const T az = invd[i] * (-(f1 * a1) - f2 * a2);
        const T bz = invd[i] * (-(f1 * b1) - f2 * b2);
        p2 = p1; p1 = pz; a2 = a1; a1 = az; b2 = b1; b1 = bz;
      }
    }
    T H[4] = {a2, b2, a1, b1}, P[2] = {p2, p1};
    T ym2, ym1;
    scan_incoming_multi<T, false, WPC>(H, P, lane, wv, xch, ym2, ym1);
#pragma unroll
    for (int ii = 0; ii < LPL; ++ii) {
      const int i = LPL - 1 - ii;
      if (l0 + i < nt) {
        const T f1 = e1[i + 1], f2 = (BW == 2) ? e2[i + 2] : T(0);
        const T yy = invd[i] * (z[i] - f1 * ym1 - f2 * ym2);
        z[i] = yy;
        ym2 = ym1; ym1 = yy;
      }
    }
  }
}

// Solve L L^T y = z in place (banded Cholesky factor L); CW lanes per column.
template <typename T, int BW, int LPL, int NC, int CW = 64>
__device__ __forceinline__ void cholesky_solve_wave(T (&z)[NC][LPL], const T* invd, const T* e1, const T* e2,
                                                    int lane, int l0, int nt) {
  tri_solve_wave<T, T, BW, LPL, NC, CW>(z, invd, invd, e1, e2, lane, l0, nt);
}

template <typename T, int LPL>
__device__ __forceinline__ void load_factor_rows(const FacTab<T>& fac, int kmode, int l0, T* invd, T* e1, T* e2) {
  const FacRow<T>* rows = fac.rows + fac.off[kmode];
  const int last = fac.last[kmode];
#pragma unroll
  for (int i = 0; i < LPL; ++i) {
    const FacRow<T> fr = rows[min(l0 + i, last)];
    invd[i] = fr.invd;
    e1[i] = fr.e1;
    e2[i] = fr.e2;
  }
  e1[LPL] = rows[min(l0 + LPL, last)].e1;
  e2[LPL] = rows[min(l0 + LPL, last)].e2;
  e2[LPL + 1] = rows[min(l0 + LPL + 1, last)].e2;
}

// Norms and stopping decision of iteration n from the nparts partial sums of
// each norm (part[0..nparts) for the residual, part[stride..stride+nparts) for
// the dual residual), reduced in a fixed order by one wavefront.
__device__ __forceinline__ void finalize_wave(Ctrl* ctrl, const double* __restrict__ part, int nparts, int stride,
                                              double wscale, double* hist) {
  const int lane = threadIdx.x & 63;
  double a = 0.0, b = 0.0;
  for (int i = lane; i < nparts; i += 64) {
    a += part[i];
    b += part[stride + i];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) finalize_body(ctrl, a, b, wscale, hist);
}

// Mode 0 of a float spectrum under an FP64 state: the row means of s = K_d^{-1} r
// are kept in the arithmetic type A (s0[l], l < nt) besides the float
// spectrum.  Mode 0 of K_d is the bare time Gram B_t B_t^T, whose solution is
// large and smooth in t, and the primal step takes its time difference: float
// rounding of it would be amplified by up to N_t there.
template <typename A, int LPL>
__device__ __forceinline__ void store_mode0(const A (&z)[LPL], A* __restrict__ s0, int l0, int nt) {
#pragma unroll
  for (int i = 0; i < LPL; ++i)
    if (l0 + i < nt) s0[l0 + i] = z[i];
}

// Column solve of spectrum columns q0..q0+7 (q0 a multiple of 8) by the 8
// waves of the calling block, one column each.  tile: kColCols * LPL * 65
// elements of LDS.
template <typename T, int BW, int LPL, typename A = T>
__device__ __forceinline__ void colsolve_group(T* __restrict__ spec, const FacTab<A>& fac, int nt, int nx, int lqb,
                                               int q0, T* tile, A* __restrict__ s0 = nullptr) {
  const int QB = 1 << lqb;
  T* base = spec + (size_t)(q0 >> lqb) * nt * QB + (q0 & (QB - 1));
  const int tid = threadIdx.x;
  constexpr int kThreads = 64 * kFdColWaves;
  constexpr int kPer = 64 * LPL * kColCols / kThreads;   // tile elements per thread
  const int wv = tid >> 6, lane = tid & 63;
  const int kmode = spec_mode(q0 + wv, nx);
  const int l0 = lane * LPL;
  // factor rows of this wave's mode first, so their latency overlaps the tile loads
  A invd[LPL], e1[LPL + 1], e2[LPL + 2];
  load_factor_rows<A, LPL>(fac, kmode, l0, invd, e1, e2);
  // all tile loads in flight before the first LDS write
  T stage[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / kColCols, c = idx % kColCols;
    stage[r] = (l < nt) ? base[(size_t)l * QB + c] : T(0);
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / kColCols, c = idx % kColCols;
    tile[(c * LPL + l % LPL) * 65 + l / LPL] = stage[r];
  }
  __syncthreads();
  A z[1][LPL];
#pragma unroll
  for (int i = 0; i < LPL; ++i) z[0][i] = A(tile[(wv * LPL + i) * 65 + lane]);
  cholesky_solve_wave<A, BW, LPL, 1>(z, invd, e1, e2, lane, l0, nt);
  if (s0 && q0 + wv == 0) store_mode0<A, LPL>(z[0], s0, l0, nt);
#pragma unroll
  for (int i = 0; i < LPL; ++i) tile[(wv * LPL + i) * 65 + lane] = T(z[0][i]);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / kColCols, c = idx % kColCols;
    stage[r] = tile[(c * LPL + l % LPL) * 65 + l / LPL];
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / kColCols, c = idx % kColCols;
    if (l < nt) base[(size_t)l * QB + c] = stage[r];
  }
}

// The same for N_t <= 512 on NCOL columns q0..q0+NCOL-1 (q0 a multiple of
// NCOL) by the calling block, CW = 32 lanes per column (two columns per wave,
// N_t <= 512) or 16 (four per wave, N_t <= 256), LPL <= 16 levels per lane: a
// wave's scans run over CW lanes, and a SIMD holds one wave with 64 / CW
// columns instead of as many waves with one each, which cuts the scan work
// per column.  tile: NCOL * LPL * (CW + 1) elements of LDS.
constexpr int kColHalfThreads = 256;
template <typename T, int BW, int LPL, int NCOL = kColCols, int CW = 32, typename A = T>
__device__ __forceinline__ void colsolve_group_half(T* __restrict__ spec, const FacTab<A>& fac, int nt, int nx,
                                                    int lqb, int q0, T* tile, A* __restrict__ s0 = nullptr) {
  constexpr int kThreads = CW * NCOL;
  constexpr int TS = CW + 1;   // tile row stride
  const int QB = 1 << lqb;
  T* base = spec + (size_t)(q0 >> lqb) * nt * QB + (q0 & (QB - 1));
  const int tid = threadIdx.x;
  constexpr int kPer = LPL;   // tile elements per thread (CW LPL NCOL / kThreads)
  const int wv = tid >> 6, lane = tid & 63;
  const int col = wv * (64 / CW) + lane / CW, q = lane % CW;
  const int kmode = spec_mode(q0 + col, nx);
  const int l0 = q * LPL;
  A invd[LPL], e1[LPL + 1], e2[LPL + 2];
  load_factor_rows<A, LPL>(fac, kmode, l0, invd, e1, e2);
  T stage[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / NCOL, c = idx % NCOL;
    stage[r] = (l < nt) ? base[(size_t)l * QB + c] : T(0);
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / NCOL, c = idx % NCOL;
    tile[(c * LPL + l % LPL) * TS + l / LPL] = stage[r];
  }
  __syncthreads();
  A z[1][LPL];
#pragma unroll
  for (int i = 0; i < LPL; ++i) z[0][i] = A(tile[(col * LPL + i) * TS + q]);
  cholesky_solve_wave<A, BW, LPL, 1, CW>(z, invd, e1, e2, lane, l0, nt);
  if (s0 && q0 + col == 0) store_mode0<A, LPL>(z[0], s0, l0, nt);
#pragma unroll
  for (int i = 0; i < LPL; ++i) tile[(col * LPL + i) * TS + q] = T(z[0][i]);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / NCOL, c = idx % NCOL;
    stage[r] = tile[(c * LPL + l % LPL) * TS + l / LPL];
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / NCOL, c = idx % NCOL;
    if (l < nt) base[(size_t)l * QB + c] = stage[r];
  }
}

// The same for 1024 < N_t <= 64 WPC LPL on 8 / WPC columns q0.. (q0 a multiple
// of 8 / WPC) by the block's 8 waves, WPC consecutive waves per column and
// LPL levels per lane.  Wave v of the block holds levels 64 LPL (v % WPC) ..
// of column v / WPC.  tile: 8 * LPL * 65 elements of LDS, xch: 48 more.
template <typename T, int BW, int LPL, int WPC, typename A = T>
__device__ __forceinline__ void colsolve_group_long(T* __restrict__ spec, const FacTab<A>& fac, int nt, int nx,
                                                    int lqb, int q0, T* tile, A* xch, A* __restrict__ s0 = nullptr) {
  constexpr int kWaves = 8;
  constexpr int kThreads = 64 * kWaves;
  constexpr int NCB = kWaves / WPC;   // columns per block
  constexpr int kPer = LPL;           // tile elements per thread (64 LPL kWaves / kThreads)
  const int QB = 1 << lqb;
  T* base = spec + (size_t)(q0 >> lqb) * nt * QB + (q0 & (QB - 1));
  const int tid = threadIdx.x;
  const int wv = tid >> 6, lane = tid & 63;
  const int col = wv / WPC;
  const int kmode = spec_mode(q0 + col, nx);
  const int l0 = ((wv % WPC) * 64 + lane) * LPL;
  A invd[LPL], e1[LPL + 1], e2[LPL + 2];
  load_factor_rows<A, LPL>(fac, kmode, l0, invd, e1, e2);
  T stage[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / NCB, c = idx % NCB;
    stage[r] = (l < nt) ? base[(size_t)l * QB + c] : T(0);
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / NCB, c = idx % NCB;
    const int g = l / LPL;   // lane of the column's lane group
    tile[((c * WPC + (g >> 6)) * LPL + l % LPL) * 65 + (g & 63)] = stage[r];
  }
  __syncthreads();
  A z[LPL];
#pragma unroll
  for (int i = 0; i < LPL; ++i) z[i] = A(tile[(wv * LPL + i) * 65 + lane]);
  cholesky_solve_multi<A, BW, LPL, WPC>(z, invd, e1, e2, lane, wv, l0, nt, xch);
  if (s0 && q0 + col == 0) store_mode0<A, LPL>(z, s0, l0, nt);
#pragma unroll
  for (int i = 0; i < LPL; ++i) tile[(wv * LPL + i) * 65 + lane] = T(z[i]);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / NCB, c = idx % NCB;
    const int g = l / LPL;
    stage[r] = tile[((c * WPC + (g >> 6)) * LPL + l % LPL) * 65 + (g & 63)];
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * kThreads;
    const int l = idx / NCB, c = idx % NCB;
    if (l < nt) base[(size_t)l * QB + c] = stage[r];
  }
}

// ------------------------------------------------------------------ C, chunked (long time axes)
// For N_t > 4096 the solve L L^T y = r of every spectrum column runs on chunks
// of kChunkLevels levels.  Both substitutions are linear, so the state entering
// chunk c of a column (forward: t_c = (z_{s-2}, z_{s-1}) at its first level s;
// backward: h_c = (y_{e+1}, y_e) at its end e) is an affine function of the
// neighbouring chunk's:
//   t_{c+1} = H_c t_c + P_c
//   h_{c-1} = G_c h_c + K_c t_c + R_c
// H_c, G_c (the homogeneous responses over the chunk) and K_c (the backward
// particular response to the forward homogeneous responses) depend only on the
// factor rows: 12 values per mode and chunk, computed once with the factor
// table (k_colchunk_maps).  P_c and R_c are the forward and backward states
// leaving the chunk when it is solved from zero entering states.  Pass 1 solves
// every chunk from zero and records P_c, R_c; the carry pass runs the two
// recurrences per column; pass 2 solves every chunk again from its entering
// states and stores y.  Every load and store of a block moves whole lines: a
// block holds the kChunkCols columns of one column block of the spectrum.

// Inclusive scan of segment maps over the 32-lane columns of a wavefront
// (H, P in place), and the state entering this lane's segment when the
// column's segment chain is entered with state (x2, x1).
template <typename T, bool FWD>
__device__ __forceinline__ void scan_half_from(T* H, T* P, int lane, T x2, T x1, T& in2, T& in1) {
  scan_step_row<T, FWD, 1>(H, P);
  scan_step_row<T, FWD, 2>(H, P);
  scan_step_row<T, FWD, 4>(H, P);
  scan_step_row<T, FWD, 8>(H, P);
  scan_cross_half(H, P, lane, FWD);
  T E[4], F[2];
  if (FWD) {
    E[0] = from_lane_below(H[0], T(1));
    E[1] = from_lane_below(H[1], T(0));
    E[2] = from_lane_below(H[2], T(0));
    E[3] = from_lane_below(H[3], T(1));
    F[0] = from_lane_below(P[0], T(0));
    F[1] = from_lane_below(P[1], T(0));
  } else {
    E[0] = from_lane_above(H[0], T(1));
    E[1] = from_lane_above(H[1], T(0));
    E[2] = from_lane_above(H[2], T(0));
    E[3] = from_lane_above(H[3], T(1));
    F[0] = from_lane_above(P[0], T(0));
    F[1] = from_lane_above(P[1], T(0));
  }
  if (FWD ? ((lane & 31) == 0) : ((lane & 31) == 31)) {   // the column's first segment: the identity
    E[0] = T(1); E[1] = T(0); E[2] = T(0); E[3] = T(1);
    F[0] = T(0); F[1] = T(0);
  }
  in2 = E[0] * x2 + E[1] * x1 + F[0];
  in1 = E[2] * x2 + E[3] * x1 + F[1];
}

// Entries of a block's LDS table at p + o, read where they are used: the
// offset is hidden from the compiler so that it neither hoists the reads nor
// keeps the values in registers across the scans.
template <typename A>
__device__ __forceinline__ const A* lds_at(const A* p, int o) {
  asm volatile("" : "+v"(o));
  return p + o;
}

// Row-local inclusive scan of the particular parts P of lane maps that all
// share the homogeneous part M (rows of 16 lanes, forward from the row's first
// lane or backward from its last): at distance d = 2^s a lane that spans d
// lanes takes in the lane d before (after) it, P += M^d P'.  pw: M^(2^s),
// s = 0..3, 4 values each (the layout of the scan's H).
template <typename A, bool FWD>
__device__ __forceinline__ void pow_scan_row(A* P, const A* pw) {
  auto step = [&](auto dd) __attribute__((always_inline)) {
    constexpr int S = decltype(dd)::value;
    constexpr int CTRL = FWD ? (0x110 + (1 << S)) : (0x100 + (1 << S));
    const A* m = lds_at(pw, 4 * S);
    const A q2 = dpp_move<CTRL>(P[0], A(0)), q1 = dpp_move<CTRL>(P[1], A(0));
    P[0] += m[0] * q2 + m[1] * q1;
    P[1] += m[2] * q2 + m[3] * q1;
  };
  step(std::integral_constant<int, 0>{});
  step(std::integral_constant<int, 1>{});
  step(std::integral_constant<int, 2>{});
  step(std::integral_constant<int, 3>{});
}

// scan_half_from for a column (32 lanes) whose lane maps all have the
// homogeneous part M: the row scan of P, then each second row (forward: lanes
// 16..31; backward: lanes 0..15) adds M^s S, S the total of the row it
// follows and s the lanes it spans, as a second row scan started from M S in
// its first lane.  The entering state x is folded into the first lane's P
// (M x), so no prefix powers are needed: the state entering lane q is the
// inclusive P of the lane before it, x for the first lane.
template <typename A, bool FWD>
__device__ __forceinline__ void scan_half_const(A* P, const A* pw, int lane, A x2, A x1, bool fold, A& in2,
                                                A& in1) {
  const int q = lane & 31, r = lane & 15, row = lane >> 4;
  const bool first = FWD ? q == 0 : q == 31;
  if (fold && first) {
    const A* m = lds_at(pw, 0);
    P[0] += m[0] * x2 + m[1] * x1;
    P[1] += m[2] * x2 + m[3] * x1;
  }
  pow_scan_row<A, FWD>(P, pw);
  {
    const int sa = FWD ? 15 : 16, sb = FWD ? 47 : 48;   // the first row's total, per column
    const A a2 = read_lane(P[0], sa), a1 = read_lane(P[1], sa);
    const A b2 = read_lane(P[0], sb), b1 = read_lane(P[1], sb);
    const bool second = (row & 1) == (FWD ? 1 : 0);
    const bool head = second && r == (FWD ? 0 : 15);
    const A s2 = row < 2 ? a2 : b2, s1 = row < 2 ? a1 : b1;
    A D[2] = {A(0), A(0)};
    if (head) {
      const A* m = lds_at(pw, 0);
      D[0] = m[0] * s2 + m[1] * s1;
      D[1] = m[2] * s2 + m[3] * s1;
    }
    pow_scan_row<A, FWD>(D, pw);
    P[0] += D[0];
    P[1] += D[1];
  }
  if (FWD) {
    in2 = from_lane_below(P[0], A(0));
    in1 = from_lane_below(P[1], A(0));
  } else {
    in2 = from_lane_above(P[0], A(0));
    in1 = from_lane_above(P[1], A(0));
  }
  if (first) {
    in2 = x2;
    in1 = x1;
  }
}

// One tile of the chunked solve: kChunkCols columns x kChunkLevels levels of
// column block g from level ls, contiguous in the spectrum (QB = kChunkCols),
// moved in 16-byte pieces; levels at or past nt read as zero and are not
// stored.
template <typename T>
struct ChunkTile {
  static constexpr int VW = 16 / (int)sizeof(T);
  static constexpr int kVec = kChunkCols * kChunkLevels / (kChunkThreads * VW);
  static constexpr int TS = kChunkCw + 1;
  typedef typename std::conditional<sizeof(T) == 8, double2, float4>::type V;
  V v[kVec];
  // unconditional loads (from the last level for levels past nt, then zeroed), so that no branch
  // separates them and the waits for the loads issued around them stay exact
  __device__ __forceinline__ void load(const T* __restrict__ spec, int nt, int g, int ls) {
    const V* base = reinterpret_cast<const V*>(spec + (size_t)g * nt * kChunkCols);
#pragma unroll
    for (int r = 0; r < kVec; ++r) {
      const int e = (threadIdx.x + r * kChunkThreads) * VW;
      const int l = ls + e / kChunkCols;
      v[r] = base[((size_t)(l < nt ? l : nt - 1) * kChunkCols + e % kChunkCols) / VW];
    }
#pragma unroll
    for (int r = 0; r < kVec; ++r) {
      const int e = (threadIdx.x + r * kChunkThreads) * VW;
      if (ls + e / kChunkCols >= nt) v[r] = V{};
    }
  }
  // LDS tile: element (level l, column c) at (c * kChunkLpl + l % kChunkLpl) * TS + l / kChunkLpl
  __device__ __forceinline__ void to_lds(T* tile) const {
#pragma unroll
    for (int r = 0; r < kVec; ++r) {
      const int e = (threadIdx.x + r * kChunkThreads) * VW;
      const int l = e / kChunkCols, c0 = e % kChunkCols;
      const T* x = reinterpret_cast<const T*>(&v[r]);
#pragma unroll
      for (int k = 0; k < VW; ++k) tile[((c0 + k) * kChunkLpl + l % kChunkLpl) * TS + l / kChunkLpl] = x[k];
    }
  }
  static __device__ __forceinline__ void store_from_lds(const T* tile, T* __restrict__ spec, int nt, int g, int ls) {
    V* base = reinterpret_cast<V*>(spec + ((size_t)g * nt + ls) * kChunkCols);
#pragma unroll
    for (int r = 0; r < kVec; ++r) {
      const int e = (threadIdx.x + r * kChunkThreads) * VW;
      const int l = e / kChunkCols, c0 = e % kChunkCols;
      V w;
      T* x = reinterpret_cast<T*>(&w);
#pragma unroll
      for (int k = 0; k < VW; ++k) x[k] = tile[((c0 + k) * kChunkLpl + l % kChunkLpl) * TS + l / kChunkLpl];
      if (ls + l < nt) base[e / VW] = w;
    }
  }
};

// The solve of one tile held in LDS (column block g, chunk c) by a block of
// kChunkThreads threads, arithmetic type A on the factor rows fac.
// SOLVE = false: pass 1 (records P_c, R_c in ca.cwork[0][c]); true: pass 2
// (reads the entering states from ca.cwork[1][c] and writes the solution back
// into the tile).
// A lane's share of a tile: column j of the tile, levels l0 .. l0 + kChunkLpl
// - 1, and its factor rows.  lookup() issues the loads of the mode's row
// offset, load_rows() those of the rows: the tile's loads go in between, so
// that all of them are in flight together (a wait for a load also waits for
// every load issued before it).
template <typename A>
struct ChunkLane {
  int col, q, j, l0, off, last;
  A invd[kChunkLpl], e1[kChunkLpl + 1], e2[kChunkLpl + 2];
  __device__ __forceinline__ void lookup(const FacTab<A>& fac, int nx, int g, int c) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    col = wv * (64 / kChunkCw) + lane / kChunkCw;
    q = lane % kChunkCw;
    j = g * kChunkCols + col;
    l0 = c * kChunkLevels + q * kChunkLpl;
    const int k = spec_mode(j, nx);
    off = fac.off[k];
    last = fac.last[k];
  }
  __device__ __forceinline__ void load_rows(const FacTab<A>& fac) {
    const FacRow<A>* rows = fac.rows + off;
#pragma unroll
    for (int i = 0; i < kChunkLpl; ++i) {
      const FacRow<A> fr = rows[min(l0 + i, last)];
      invd[i] = fr.invd;
      e1[i] = fr.e1;
      e2[i] = fr.e2;
    }
    e1[kChunkLpl] = rows[min(l0 + kChunkLpl, last)].e1;
    e2[kChunkLpl] = rows[min(l0 + kChunkLpl, last)].e2;
    e2[kChunkLpl + 1] = rows[min(l0 + kChunkLpl + 1, last)].e2;
  }
  // a tile past the last distinct row: every level uses row `last`
  __device__ __forceinline__ void load_row_last(const FacTab<A>& fac) {
    const FacRow<A> fr = fac.rows[off + last];
#pragma unroll
    for (int i = 0; i < kChunkLpl; ++i) {
      invd[i] = fr.invd;
      e1[i] = fr.e1;
      e2[i] = fr.e2;
    }
    e1[kChunkLpl] = fr.e1;
    e2[kChunkLpl] = fr.e2;
    e2[kChunkLpl + 1] = fr.e2;
  }
};

template <typename T, int BW, typename A, bool SOLVE, bool CST>
__device__ __forceinline__ void colchunk_tile(const ChunkLane<A>& ln, const ChunkArgs& ca, int nt, int nx, int c,
                                              T* tile, const A* pw, const A* st, double* __restrict__ s0) {
  constexpr int LPL = kChunkLpl, CW = kChunkCw, TS = CW + 1;
  const int lane = threadIdx.x & 63;
  const int col = ln.col, q = ln.q, j = ln.j, l0 = ln.l0;
  const A* invd = ln.invd;
  const A* e1 = ln.e1;
  const A* e2 = ln.e2;
  A z[LPL];
#pragma unroll
  for (int i = 0; i < LPL; ++i) z[i] = A(tile[(col * LPL + i) * TS + q]);
  // CST: a full chunk past the last distinct factor row of every column of the tile, so that every lane map
  // has the homogeneous part M, whose powers come from the block's table
  constexpr bool cst = CST;
  // forward: z_l = invd_l (r_l - e1_l z_{l-1} - e2_l z_{l-2})
  {
    A P[2], zm2, zm1, x2 = A(0), x1 = A(0);
    if (SOLVE) {   // the state entering the chunk, read from the block's copy where it is needed
      const A* x = lds_at(st, 0);
      x2 = x[0];
      x1 = x[1];
    }
    if (cst) {
      A p2 = 0, p1 = 0;
#pragma unroll
      for (int i = 0; i < LPL; ++i) {
        const A pz = invd[i] * (z[i] - e1[i] * p1 - (BW == 2 ? e2[i] * p2 : A(0)));
        p2 = p1; p1 = pz;
      }
      P[0] = p2; P[1] = p1;
      scan_half_const<A, true>(P, pw, lane, x2, x1, SOLVE, zm2, zm1);
    } else {
      A p2 = 0, p1 = 0, a2 = 1, a1 = 0, b2 = 0, b1 = 1;
#pragma unroll
      for (int i = 0; i < LPL; ++i) {
        if (l0 + i < nt) {
          const A pz = invd[i] * (z[i] - e1[i] * p1 - (BW == 2 ? e2[i] * p2 : A(0)));
          const A az = invd[i] * (-(e1[i] * a1) - (BW == 2 ? e2[i] * a2 : A(0)));
          const A bz = invd[i] * (-(e1[i] * b1) - (BW == 2 ? e2[i] * b2 : A(0)));
          p2 = p1; p1 = pz; a2 = a1; a1 = az; b2 = b1; b1 = bz;
        }
      }
      A H[4] = {a2, b2, a1, b1};
      P[0] = p2; P[1] = p1;
      scan_half_from<A, true>(H, P, lane, x2, x1, zm2, zm1);
    }
    if (!SOLVE && q == CW - 1) {   // state leaving the chunk (from zero)
      double* rec = ca.cwork + ((size_t)c * nx + j) * 4;
      rec[0] = double(P[0]);
      rec[1] = double(P[1]);
    }
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
      if (l0 + i < nt) {
        const A zz = invd[i] * (z[i] - e1[i] * zm1 - (BW == 2 ? e2[i] * zm2 : A(0)));
        z[i] = zz;
        zm2 = zm1; zm1 = zz;
      }
    }
  }
  // backward: y_l = invd_l (z_l - e1_{l+1} y_{l+1} - e2_{l+2} y_{l+2})
  {
    A P[2], ym2, ym1, w2 = A(0), w1 = A(0);
    if (SOLVE) {
      const A* w = lds_at(st, 2);
      w2 = w[0];
      w1 = w[1];
    }
    if (cst) {
      A p2 = 0, p1 = 0;
#pragma unroll
      for (int ii = 0; ii < LPL; ++ii) {
        const int i = LPL - 1 - ii;
        const A f1 = e1[i + 1], f2 = (BW == 2) ? e2[i + 2] : A(0);
        const A pz = invd[i] * (z[i] - f1 * p1 - f2 * p2);
        p2 = p1; p1 = pz;
      }
      P[0] = p2; P[1] = p1;
      scan_half_const<A, false>(P, pw, lane, w2, w1, SOLVE, ym2, ym1);
    } else {
      A p2 = 0, p1 = 0, a2 = 1, a1 = 0, b2 = 0, b1 = 1;
#pragma unroll
      for (int ii = 0; ii < LPL; ++ii) {
        const int i = LPL - 1 - ii;
        if (l0 + i < nt) {
          const A f1 = e1[i + 1], f2 = (BW == 2) ? e2[i + 2] : A(0);
          const A pz = invd[i] * (z[i] - f1 * p1 - f2 * p2);
          const A az = invd[i] * (-(f1 * a1) - f2 * a2);
          const A bz = invd[i] * (-(f1 * b1) - f2 * b2);
          p2 = p1; p1 = pz; a2 = a1; a1 = az; b2 = b1; b1 = bz;
        }
      }
      A H[4] = {a2, b2, a1, b1};
      P[0] = p2; P[1] = p1;
      scan_half_from<A, false>(H, P, lane, w2, w1, ym2, ym1);
    }
    if (!SOLVE) {
      if (q == 0) {   // state leaving the chunk backwards (forward values from zero)
        double* rec = ca.cwork + ((size_t)c * nx + j) * 4;
        rec[2] = double(P[0]);
        rec[3] = double(P[1]);
      }
      return;
    }
#pragma unroll
    for (int ii = 0; ii < LPL; ++ii) {
      const int i = LPL - 1 - ii;
      if (l0 + i < nt) {
        const A f1 = e1[i + 1], f2 = (BW == 2) ? e2[i + 2] : A(0);
        const A yy = invd[i] * (z[i] - f1 * ym1 - f2 * ym2);
        z[i] = yy;
        ym2 = ym1; ym1 = yy;
      }
    }
  }
  if (s0 && j == 0) {
#pragma unroll
    for (int i = 0; i < LPL; ++i)
      if (l0 + i < nt) s0[l0 + i] = double(z[i]);
  }
#pragma unroll
  for (int i = 0; i < LPL; ++i) tile[(col * LPL + i) * TS + q] = T(z[i]);
}

// One tile (column block g, chunk c) by the calling block: the lookup of the
// mode's row offset and the entering states, the tile's loads and the factor
// rows are issued in that order, so that their latencies overlap.
// tile: kChunkCols * kChunkLpl * (kChunkCw + 1) elements of LDS.
// One tile (column block g, chunk c) of either pass; CST: a tile whose every
// column lies past its last distinct factor row (only row `last` is loaded,
// and the scans use the powers of M).
template <typename T, int BW, typename A, bool SOLVE, bool CST>
__device__ __forceinline__ void colchunk_item(T* __restrict__ spec, const FacTab<A>& fac, const ChunkArgs& ca,
                                              int nt, int nx, int g, int c, T* tile, double* __restrict__ s0) {
  ChunkLane<A> ln;
  ln.lookup(fac, nx, g, c);
  ChunkTile<T> buf;
  buf.load(spec, nt, g, c * kChunkLevels);
  // the power table of the block's columns, after the tile in LDS: [kChunkCols][kChunkPow][4] (every thread
  // loads, the first kChunkCols * kChunkPow * 4 store)
  constexpr int NPW = kChunkCols * kChunkPow * 4;
  static_assert(NPW <= kChunkThreads, "one power entry per thread");
  A* pwl = reinterpret_cast<A*>(tile + kChunkCols * kChunkLpl * (kChunkCw + 1));
  double pv = 0.0;
  if (CST) {
    const int pe = threadIdx.x % NPW;
    pv = ca.cpow[(size_t)spec_mode(g * kChunkCols + pe / (kChunkPow * 4), nx) * (kChunkPow * 4) + pe % (kChunkPow * 4)];
  }
  // pass 2: the states entering the chunk (t, h) of the block's columns, after the powers: [kChunkCols][4]
  A* stl = pwl + NPW;
  const double sv = SOLVE ? ca.cwork[((size_t)(ca.nchunk + c) * nx + g * kChunkCols) * 4 + threadIdx.x % (4 * kChunkCols)]
                          : 0.0;
  if (CST) ln.load_row_last(fac);
  else ln.load_rows(fac);
  buf.to_lds(tile);
  if (CST && threadIdx.x < NPW) pwl[threadIdx.x] = A(pv);
  if (SOLVE && threadIdx.x < 4 * kChunkCols) stl[threadIdx.x] = A(sv);
  __syncthreads();
  colchunk_tile<T, BW, A, SOLVE, CST>(ln, ca, nt, nx, c, tile, pwl + ln.col * (kChunkPow * 4), stl + ln.col * 4, s0);
  if (SOLVE) {
    __syncthreads();
    ChunkTile<T>::store_from_lds(tile, spec, nt, g, c * kChunkLevels);
  }
}

// Dynamic LDS above 64 KiB needs an explicit opt-in per kernel.
template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace pdhg
