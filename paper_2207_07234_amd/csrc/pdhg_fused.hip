// Fused passes of one iteration of Algorithm 1 (Section 3.3) on gfx950.
//
// One iteration n = three kernels:
//   A  k_dual_fft      per pair of dual rows: inverse FFT of the preconditioned
//                      residual shat^{n-1}, dual step phi^{n-1} = phi^{n-2} + tau s,
//                      extrapolation phibar = phi^{n-1} + tau s            (in place on phi)
//   B  k_primal_res    per pair of implicit rows (2w, 2w+1): primal step
//                      u^n = u^{n-1} - tau_u J(u^{n-1})^T phibar on the levels the rows
//                      touch, the dual residual ||J(u^{n-1})^T phi^{n-1}|| of the owned
//                      levels, the implicit residual A(u^n) of the two rows, its
//                      forward FFT (halfcomplex spectrum, column-block layout), the
//                      primal residual ||A(u^n)||, and, in the last block to finish,
//                      the convergence decision (Section 3.3 stopping rule)
//   C  k_colsolve_wave per Fourier mode: banded Cholesky solve along t
//                      (the preconditioner K_d^{-1} of Section 2.2)
// Halo levels of u^n needed by the time stencil of A are recomputed by each
// block from the same inputs (bitwise identical to the owner's values); u is
// ping-ponged between two buffers so no block reads a level another block has
// already overwritten.
#include "pdhg_internal.hpp"

namespace pdhg {

constexpr int kRowThreadsMax = 512;

// ------------------------------------------------------------------ A
// W = nx / EPT threads.  All global loads (twiddles, the two spectrum rows and
// the two dual rows) are issued before the first LDS write so that their
// latencies overlap; the twiddle table and the FFT buffer live in LDS.
template <typename T, int EPT>
__global__ void __launch_bounds__(kRowThreadsMax)
k_dual_fft(const T* __restrict__ spec, int nt, int lqb, int nx, const C2<T>* __restrict__ tw, T* __restrict__ phi,
           T* __restrict__ phibar, T tau, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  extern __shared__ char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(nx);
  const int tid = threadIdx.x, W = blockDim.x;
  const int a = 2 * xcd_block(blockIdx.x, gridDim.x), b = a + 1;
  const bool hasb = b < nt;
  const int half = nx >> 1;
  T* pa = phi + (size_t)a * nx;
  T* qa = phibar + (size_t)a * nx;
  T* pb = phi + (size_t)b * nx;
  T* qb = phibar + (size_t)b * nx;
  // ---- loads
  C2<T> twv[EPT];
  T fa[EPT], fb[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int x = tid + e * W;
    twv[e] = tw[x];
    fa[e] = pa[x];
    fb[e] = hasb ? pb[x] : T(0);
  }
  // halfcomplex pair: thread handles modes k = tid + e W, k <= nx/2 (EPT/2 + 1 of them)
  constexpr int KPT = EPT / 2 + 1;
  T sar[KPT], sai[KPT], sbr[KPT], sbi[KPT];
#pragma unroll
  for (int e = 0; e < KPT; ++e) {
    const int k = tid + e * W;
    sar[e] = sai[e] = sbr[e] = sbi[e] = T(0);
    if (k <= half) {
      if (k == 0 || k == half) {
        const int q = (k == 0) ? 0 : 1;
        sar[e] = spec[spec_index(a, q, nt, lqb)];
        if (hasb) sbr[e] = spec[spec_index(b, q, nt, lqb)];
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
  for (int e = 0; e < EPT; ++e) twl[lpad(tid + e * W)] = twv[e];
#pragma unroll
  for (int e = 0; e < KPT; ++e) {
    const int k = tid + e * W;
    if (k <= half) {
      buf[lpad(k)] = {sar[e] - sbi[e], sai[e] + sbr[e]};
      if (k != 0 && k != half) buf[lpad(nx - k)] = {sar[e] + sbi[e], sbr[e] - sai[e]};
    }
  }
  fft_lds<true, EPT>(buf, nx, twl, tid, W);
  const T sc = T(1) / T(nx);
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int x = tid + e * W;
    const C2<T> z = buf[lpad(x)];
    const T ta = tau * (z.x * sc);
    const T p = fa[e] + ta;
    pa[x] = p;
    qa[x] = p + ta;
    if (hasb) {
      const T tb = tau * (z.y * sc);
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

// W = 64 nw threads; wave v owns x in [v 64E, (v+1) 64E), lane l element e at
// x = v 64E + l + 64 e.  Every global row the block needs is loaded up front:
// u^{n-1} on levels a-1..a+2, phibar on rows a-2..a+3, phi on rows a..a+3.
template <typename T, int E>
__global__ void __launch_bounds__(kRowThreadsMax)
k_primal_res(Scheme sch, const T* __restrict__ u_in, T* __restrict__ u_out, const T* __restrict__ phibar,
             const T* __restrict__ phi, T tau_u, T* __restrict__ spec, int lqb, const C2<T>* __restrict__ tw,
             double* __restrict__ part, const Ctrl* ctrl) {
  if (ctrl->status != 0) return;
  extern __shared__ char smem[];
  const Consts<T> C(sch);
  const int nx = sch.nx, nt = sch.nt, W = blockDim.x, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, nw = W >> 6;
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(nx);
  T* edge = reinterpret_cast<T*>(twl + lds_fft_points(nx));   // [2 rows][first, last][nw]
  __shared__ double red[kRowThreadsMax / 64];
  const int seg0 = wv * 64 * E;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int a = 2 * blk, b = a + 1;                            // implicit rows of this block
  const bool bdf2 = C.time == kTimeBDF2;
  // ---- all global loads first
  constexpr int TPT = (E < 1) ? 1 : E;                         // twiddles per thread (nx / W)
  C2<T> twv[TPT];
#pragma unroll
  for (int e = 0; e < TPT; ++e) twv[e] = tw[tid + e * W];
  T U0[4][E], U[4][E];                 // u^{n-1} and u^n on levels a-1+i
  T PB[6][E], PBp[4], PBn[4];          // phibar rows a-2+j (edges for j = 0..3)
  T PH[4][E], PHp[2], PHn[2];          // phi rows a+j (edges for j = 0, 1)
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = a - 1 + i;
    const bool ok = m >= 0 && m <= nt && (bdf2 || i > 0);
#pragma unroll
    for (int e = 0; e < E; ++e) U0[i][e] = ok ? u_in[(size_t)m * nx + seg0 + lane + 64 * e] : T(0);
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    T pv, nv;
    load_row_wave<T, E>(phibar, a - 2 + j, nt, nx, seg0, lane, PB[j], pv, nv);
    if (j < 4) { PBp[j] = pv; PBn[j] = nv; }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    T pv, nv;
    load_row_wave<T, E>(phi, a + j, nt, nx, seg0, lane, PH[j], pv, nv);
    if (j < 2) { PHp[j] = pv; PHn[j] = nv; }
  }
#pragma unroll
  for (int e = 0; e < TPT; ++e) twl[lpad(tid + e * W)] = twv[e];
  // ---- primal step on the four levels, dual residual on the two owned ones
  double rd = 0.0, rp = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = a - 1 + i;
    if (m < 0 || m > nt || (!bdf2 && i == 0)) continue;
    if (m == 0) {
#pragma unroll
      for (int e = 0; e < E; ++e) U[i][e] = U0[i][e];
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
      dual_op_regs<T, E>(C, m, PH[i - 2], PHp[i - 2], PHn[i - 2], PH[i - 1], PH[i], U0[i], g);
#pragma unroll
      for (int e = 0; e < E; ++e) rd += (double)g[e] * (double)g[e];
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
#pragma unroll
  for (int e = 0; e < E; ++e) buf[lpad(seg0 + lane + 64 * e)] = {R[0][e], R[1][e]};
  fft_lds<false, E>(buf, nx, twl, tid, W);
  store_halfcomplex_pair(buf, nx, spec, nt, lqb, a, b < nt, tid, W);

  // per-block partial sums; the column-solve kernel of this iteration reduces them
  const double srp = block_sum_waves(rp, red);
  const double srd = block_sum_waves(rd, red);
  if (tid == 0) {
    part[blk] = srp;
    part[gridDim.x + blk] = srd;
  }
}

// ------------------------------------------------------------------ C
// Banded Cholesky solve along t.  One wavefront per Fourier mode k handles the
// two halfcomplex columns of that mode (Re and Im share the factor; the first
// wave of the spectrum handles the real columns of modes 0 and nx/2).  Lane j
// owns levels [j LPL, (j+1) LPL).  Each lane computes the affine map of its
// segment (particular solution and the responses to the two incoming values),
// an inclusive scan of the maps across the 64 lanes (shuffles, no barriers)
// gives every lane its incoming state, and the segment is re-run from it.
// The block stages a [nt][8-column] tile of the spectrum through LDS (lane-major,
// padded) so that global accesses are coalesced and LDS accesses conflict-free.
constexpr int kColWaves = 4;
constexpr int kColCols = 2 * kColWaves;

template <typename T>
__device__ __forceinline__ T shfl_up_T(T v, int d) { return __shfl_up(v, d, 64); }
template <typename T>
__device__ __forceinline__ T shfl_down_T(T v, int d) { return __shfl_down(v, d, 64); }

// (H, P) <- (H, P) o (H', P') : apply (H', P') first, then (H, P).
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

// Inclusive scan of segment maps over the lanes, forward (from lane 0) or
// backward (from lane 63); returns the state entering this lane's segment.
template <typename T, bool FWD>
__device__ __forceinline__ void scan_incoming(T* H, T* P, int lane, T& in2, T& in1) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T H2[4], P2[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) H2[k] = FWD ? shfl_up_T(H[k], d) : shfl_down_T(H[k], d);
    P2[0] = FWD ? shfl_up_T(P[0], d) : shfl_down_T(P[0], d);
    P2[1] = FWD ? shfl_up_T(P[1], d) : shfl_down_T(P[1], d);
    if (FWD ? (lane >= d) : (lane + d < 64)) compose(H, P, H2, P2);
  }
  in2 = FWD ? shfl_up_T(P[0], 1) : shfl_down_T(P[0], 1);
  in1 = FWD ? shfl_up_T(P[1], 1) : shfl_down_T(P[1], 1);
  if (FWD ? (lane == 0) : (lane == 63)) { in2 = T(0); in1 = T(0); }
}

// Solve L L^T y = z in place for NC columns sharing the factor rows; z[c][i]
// is level l0 + i of column c.
template <typename T, int BW, int LPL, int NC>
__device__ __forceinline__ void cholesky_solve_wave(T (&z)[NC][LPL], const T* invd, const T* e1, const T* e2,
                                                    int lane, int l0, int nt) {
  // forward: z_l = invd_l (rhs_l - e1_l z_{l-1} - e2_l z_{l-2})
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    T p2 = 0, p1 = 0, a2 = 1, a1 = 0, b2 = 0, b1 = 1;
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
      if (l0 + i < nt) {
        const T pz = invd[i] * (z[c][i] - e1[i] * p1 - (BW == 2 ? e2[i] * p2 : T(0)));
        const T az = invd[i] * (-e1[i] * a1 - (BW == 2 ? e2[i] * a2 : T(0)));
        const T bz = invd[i] * (-e1[i] * b1 - (BW == 2 ? e2[i] * b2 : T(0)));
        p2 = p1; p1 = pz; a2 = a1; a1 = az; b2 = b1; b1 = bz;
      }
    }
    T H[4] = {a2, b2, a1, b1}, P[2] = {p2, p1};
    T zm2, zm1;
    scan_incoming<T, true>(H, P, lane, zm2, zm1);
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
      if (l0 + i < nt) {
        const T zz = invd[i] * (z[c][i] - e1[i] * zm1 - (BW == 2 ? e2[i] * zm2 : T(0)));
        z[c][i] = zz;
        zm2 = zm1; zm1 = zz;
      }
    }
  }
  // backward: y_l = invd_l (z_l - e1_{l+1} y_{l+1} - e2_{l+2} y_{l+2})
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    T p2 = 0, p1 = 0, a2 = 1, a1 = 0, b2 = 0, b1 = 1;
#pragma unroll
    for (int ii = 0; ii < LPL; ++ii) {
      const int i = LPL - 1 - ii;
      if (l0 + i < nt) {
        const T f1 = e1[i + 1], f2 = (BW == 2) ? e2[i + 2] : T(0);
        const T pz = invd[i] * (z[c][i] - f1 * p1 - f2 * p2);
        const T az = invd[i] * (-f1 * a1 - f2 * a2);
        const T bz = invd[i] * (-f1 * b1 - f2 * b2);
        p2 = p1; p1 = pz; a2 = a1; a1 = az; b2 = b1; b1 = bz;
      }
    }
    T H[4] = {a2, b2, a1, b1}, P[2] = {p2, p1};
    T ym2, ym1;
    scan_incoming<T, false>(H, P, lane, ym2, ym1);
#pragma unroll
    for (int ii = 0; ii < LPL; ++ii) {
      const int i = LPL - 1 - ii;
      if (l0 + i < nt) {
        const T f1 = e1[i + 1], f2 = (BW == 2) ? e2[i + 2] : T(0);
        const T yy = invd[i] * (z[c][i] - f1 * ym1 - f2 * ym2);
        z[c][i] = yy;
        ym2 = ym1; ym1 = yy;
      }
    }
  }
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

// Norms and stopping decision of iteration n from the nparts per-block partial
// sums written by k_primal_res (first wave of the block only; fixed order).
__device__ __forceinline__ void finalize_wave(Ctrl* ctrl, const double* __restrict__ part, int nparts,
                                              double wscale, double* hist) {
  const int lane = threadIdx.x & 63;
  double a = 0.0, b = 0.0;
  for (int i = lane; i < nparts; i += 64) {
    a += part[i];
    b += part[nparts + i];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) finalize_body(ctrl, a, b, wscale, hist);
}

template <typename T, int BW, int LPL>
__global__ void __launch_bounds__(64 * kColWaves)
k_colsolve_wave(T* __restrict__ spec, FacTab<T> fac, int nt, int nx, int lqb, Ctrl* ctrl, const double* part,
                int nparts, double wscale, double* hist) {
  if (ctrl && ctrl->status != 0) return;
  if (part && blockIdx.x == 0 && threadIdx.x < 64) finalize_wave(ctrl, part, nparts, wscale, hist);
  extern __shared__ char smem[];
  T* tile = reinterpret_cast<T*>(smem);   // [kColCols][LPL][65], level l of column c at (c LPL + l % LPL) 65 + l / LPL
  const int QB = 1 << lqb;
  const int q0 = xcd_block(blockIdx.x, gridDim.x) * kColCols;   // first spectrum column of this block
  T* base = spec + (size_t)(q0 >> lqb) * nt * QB + (q0 & (QB - 1));
  const int tid = threadIdx.x;
  constexpr int kPer = 64 * LPL * kColCols / (64 * kColWaves);   // tile elements per thread
  const int wv = tid >> 6, lane = tid & 63;
  const int qa = q0 + 2 * wv, qb = qa + 1;
  const int ka = spec_mode(qa, nx), kb = spec_mode(qb, nx);
  const int l0 = lane * LPL;
  // factor rows of this wave's mode first, so their latency overlaps the tile loads
  T invd[LPL], e1[LPL + 1], e2[LPL + 2];
  load_factor_rows<T, LPL>(fac, ka, l0, invd, e1, e2);
  // all tile loads in flight before the first LDS write
  T stage[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * 64 * kColWaves;
    const int l = idx / kColCols, c = idx % kColCols;
    stage[r] = (l < nt) ? base[(size_t)l * QB + c] : T(0);
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * 64 * kColWaves;
    const int l = idx / kColCols, c = idx % kColCols;
    tile[(c * LPL + l % LPL) * 65 + l / LPL] = stage[r];
  }
  __syncthreads();
  T z[2][LPL];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < LPL; ++i) z[c][i] = tile[((2 * wv + c) * LPL + i) * 65 + lane];
  if (ka == kb) {
    cholesky_solve_wave<T, BW, LPL, 2>(z, invd, e1, e2, lane, l0, nt);
  } else {   // real columns of modes 0 and nx/2
    T za[1][LPL], zb[1][LPL];
#pragma unroll
    for (int i = 0; i < LPL; ++i) { za[0][i] = z[0][i]; zb[0][i] = z[1][i]; }
    cholesky_solve_wave<T, BW, LPL, 1>(za, invd, e1, e2, lane, l0, nt);
    load_factor_rows<T, LPL>(fac, kb, l0, invd, e1, e2);
    cholesky_solve_wave<T, BW, LPL, 1>(zb, invd, e1, e2, lane, l0, nt);
#pragma unroll
    for (int i = 0; i < LPL; ++i) { z[0][i] = za[0][i]; z[1][i] = zb[0][i]; }
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < LPL; ++i) tile[((2 * wv + c) * LPL + i) * 65 + lane] = z[c][i];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * 64 * kColWaves;
    const int l = idx / kColCols, c = idx % kColCols;
    stage[r] = tile[(c * LPL + l % LPL) * 65 + l / LPL];
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int idx = tid + r * 64 * kColWaves;
    const int l = idx / kColCols, c = idx % kColCols;
    if (l < nt) base[(size_t)l * QB + c] = stage[r];
  }
}

// ------------------------------------------------------------------ launchers
static inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Dynamic LDS above 64 KiB needs an explicit opt-in per kernel.
template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <typename T, int EPT>
static hipError_t launch_dual_fft_e(const T* spec, int nt, int lqb, int nx, const void* tw, T* phi, T* phibar, T tau,
                                    const Ctrl* ctrl, hipStream_t st) {
  const int W = nx / EPT;
  const size_t lds = sizeof(C2<T>) * 2 * (size_t)lds_fft_points(nx);
  hipError_t e = allow_lds(k_dual_fft<T, EPT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_dual_fft<T, EPT>), dim3((nt + 1) / 2), dim3(W), lds, st, spec, nt, lqb, nx,
                     (const C2<T>*)tw, phi, phibar, tau, ctrl);
  return hipGetLastError();
}

// A: nx >= 64.
template <typename T>
hipError_t launch_dual_fft(const T* spec, int nt, int lqb, int nx, const void* tw, T* phi, T* phibar, T tau,
                           const Ctrl* ctrl, hipStream_t st) {
  // EPT = nx / W with W = min(512, nx / 2) threads for nx >= 128 (8 waves at nx = 2048)
  const int W = nx >= 1024 ? 512 : (nx >= 128 ? nx / 2 : nx);
  switch (nx / W) {
    case 1: return launch_dual_fft_e<T, 1>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st);
    case 2: return launch_dual_fft_e<T, 2>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st);
    case 4: return launch_dual_fft_e<T, 4>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st);
    case 8: return launch_dual_fft_e<T, 8>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int E>
static hipError_t launch_primal_res_e(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi,
                                      T tau_u, T* spec, int lqb, const void* tw, double* part, const Ctrl* ctrl,
                                      hipStream_t st) {
  const int W = s.nx / E;
  const size_t lds = sizeof(C2<T>) * 2 * (size_t)lds_fft_points(s.nx) + sizeof(T) * 4 * (W / 64);
  hipError_t e = allow_lds(k_primal_res<T, E>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_primal_res<T, E>), dim3((s.nt + 1) / 2), dim3(W), lds, st, s, u_in, u_out, phibar, phi,
                     tau_u, spec, lqb, (const C2<T>*)tw, part, ctrl);
  return hipGetLastError();
}

// B: W = 64 * clamp(nx / 256, 1, 8) threads, E = nx / W points per thread (nx >= 64).
template <typename T>
hipError_t launch_primal_res(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                             T* spec, int lqb, const void* tw, double* part, const Ctrl* ctrl, hipStream_t st) {
  const int W = 64 * clampi(s.nx / 256, 1, 8);
  switch (s.nx / W) {
    case 1: return launch_primal_res_e<T, 1>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, st);
    case 2: return launch_primal_res_e<T, 2>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, st);
    case 4: return launch_primal_res_e<T, 4>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, st);
    case 8: return launch_primal_res_e<T, 8>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int BW, int LPL>
static hipError_t launch_colsolve_wave_l(T* spec, const FacTab<T>& fac, int nt, int nx, int lqb, Ctrl* ctrl,
                                         const double* part, int nparts, double wscale, double* hist,
                                         hipStream_t st) {
  const size_t lds = sizeof(T) * (size_t)kColCols * LPL * 65;
  hipError_t e = allow_lds(k_colsolve_wave<T, BW, LPL>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_colsolve_wave<T, BW, LPL>), dim3(nx / kColCols), dim3(64 * kColWaves), lds, st, spec, fac,
                     nt, nx, lqb, ctrl, part, nparts, wscale, hist);
  return hipGetLastError();
}

// C: nt <= 1024, nx >= 8 (one wavefront per Fourier mode).  With part != NULL the
// first wave of block 0 also reduces the iteration's residual partial sums and
// takes the stopping decision (ctrl must then be non-NULL).
template <typename T>
hipError_t launch_colsolve_wave(T* spec, const FacTab<T>& fac, int bw, int nt, int nx, int lqb, Ctrl* ctrl,
                                const double* part, int nparts, double wscale, double* hist, hipStream_t st) {
  const int lpl = (nt + 63) / 64;
#define PDHG_CW(B, L) \
  return launch_colsolve_wave_l<T, B, L>(spec, fac, nt, nx, lqb, ctrl, part, nparts, wscale, hist, st)
  if (bw == 2) {
    if (lpl <= 1) PDHG_CW(2, 1);
    if (lpl <= 2) PDHG_CW(2, 2);
    if (lpl <= 4) PDHG_CW(2, 4);
    if (lpl <= 8) PDHG_CW(2, 8);
    if (lpl <= 16) PDHG_CW(2, 16);
  } else {
    if (lpl <= 1) PDHG_CW(1, 1);
    if (lpl <= 2) PDHG_CW(1, 2);
    if (lpl <= 4) PDHG_CW(1, 4);
    if (lpl <= 8) PDHG_CW(1, 8);
    if (lpl <= 16) PDHG_CW(1, 16);
  }
#undef PDHG_CW
  return hipErrorInvalidValue;
}

template hipError_t launch_dual_fft<float>(const float*, int, int, int, const void*, float*, float*, float,
                                           const Ctrl*, hipStream_t);
template hipError_t launch_dual_fft<double>(const double*, int, int, int, const void*, double*, double*, double,
                                            const Ctrl*, hipStream_t);
template hipError_t launch_primal_res<float>(const Scheme&, const float*, float*, const float*, const float*, float,
                                             float*, int, const void*, double*, const Ctrl*, hipStream_t);
template hipError_t launch_primal_res<double>(const Scheme&, const double*, double*, const double*, const double*,
                                              double, double*, int, const void*, double*, const Ctrl*, hipStream_t);
template hipError_t launch_colsolve_wave<float>(float*, const FacTab<float>&, int, int, int, int, Ctrl*,
                                                const double*, int, double, double*, hipStream_t);
template hipError_t launch_colsolve_wave<double>(double*, const FacTab<double>&, int, int, int, int, Ctrl*,
                                                 const double*, int, double, double*, hipStream_t);

}  // namespace pdhg
