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
// W = nx / EPT threads; the twiddle table and the FFT buffer live in LDS.
template <typename T, int EPT>
__global__ void __launch_bounds__(kRowThreadsMax)
k_dual_fft(const T* __restrict__ spec, int nt, int lqb, int nx, const C2<T>* __restrict__ tw, T* __restrict__ phi,
           T* __restrict__ phibar, T tau, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  extern __shared__ char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(nx);
  const int tid = threadIdx.x, W = blockDim.x;
  const int a = 2 * blockIdx.x, b = a + 1;
  const bool hasb = b < nt;
  load_twiddles_lds(twl, tw, nx, tid, W);
  load_halfcomplex_pair(buf, nx, spec, nt, lqb, a, hasb, tid, W);
  fft_lds<true, EPT>(buf, nx, twl, tid, W);
  const T sc = T(1) / T(nx);
  T* pa = phi + (size_t)a * nx;
  T* qa = phibar + (size_t)a * nx;
  T* pb = phi + (size_t)b * nx;
  T* qb = phibar + (size_t)b * nx;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int x = tid + e * W;
    const C2<T> z = buf[lpad(x)];
    const T ta = tau * (z.x * sc);
    const T p = pa[x] + ta;
    pa[x] = p;
    qa[x] = p + ta;
    if (hasb) {
      const T tb = tau * (z.y * sc);
      const T q = pb[x] + tb;
      pb[x] = q;
      qb[x] = q + tb;
    }
  }
}

// ------------------------------------------------------------------ B
// Coherent (L1-bypassing) load for the cross-block reduction.
__device__ __forceinline__ double load_coherent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// J(u)^T psi at unknown level m for this lane's points x = seg0 + lane + 64 e.
// psi^{m-1} is loaded once (coalesced) and its x-neighbours come from the
// neighbouring lanes.
template <typename T, int E>
__device__ __forceinline__ void dual_op_wave(const Consts<T>& C, int m, const T* __restrict__ psi, const T* uv,
                                             int seg0, int lane, T* out) {
  const int nx = C.nx, nt = C.nt;
  const T* p0 = psi + (size_t)(m - 1) * nx;
  const bool has1 = m <= nt - 1;
  const bool has2 = (C.time == kTimeBDF2) && (m + 1 <= nt - 1);
  const T* p1 = psi + (size_t)m * nx;
  const T* p2 = psi + (size_t)(m + 1) * nx;
  T c[E], t1[E], t2[E], cm[E], cp[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int x = seg0 + lane + 64 * e;
    c[e] = p0[x];
    t1[e] = has1 ? p1[x] : T(0);
    t2[e] = has2 ? p2[x] : T(0);
  }
  const T prev = p0[(seg0 - 1) & (nx - 1)];
  const T next = p0[(seg0 + 64 * E) & (nx - 1)];
  wave_row_neighbours<T, E>(c, prev, next, cm, cp);
#pragma unroll
  for (int e = 0; e < E; ++e) out[e] = C.JtTime(m, c[e], t1[e], t2[e]) + C.JtF(uv[e], cm[e], c[e], cp[e]);
}

// W = 64 nw threads; wave v owns x in [v 64E, (v+1) 64E), lane l element e at
// x = v 64E + l + 64 e.
template <typename T, int E>
__global__ void __launch_bounds__(kRowThreadsMax)
k_primal_res(Scheme sch, const T* __restrict__ u_in, T* __restrict__ u_out, const T* __restrict__ phibar,
             const T* __restrict__ phi, T tau_u, T* __restrict__ spec, int lqb, const C2<T>* __restrict__ tw,
             double* __restrict__ part, Ctrl* ctrl, double* hist, unsigned* counter) {
  if (ctrl->status != 0) return;
  extern __shared__ char smem[];
  const Consts<T> C(sch);
  const int nx = sch.nx, nt = sch.nt, W = blockDim.x, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, nw = W >> 6;
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(nx);
  T* edge = reinterpret_cast<T*>(twl + lds_fft_points(nx));   // [2 rows][first, last][nw]
  __shared__ double red[kRowThreadsMax];
  __shared__ unsigned ticket;
  const int seg0 = wv * 64 * E;
  const int a = 2 * blockIdx.x, b = a + 1;                     // implicit rows of this block
  const bool bdf2 = C.time == kTimeBDF2;
  load_twiddles_lds(twl, tw, nx, tid, W);
  // slot i holds level a - 1 + i (i = 0..3); rows a, b need slots {2,1,0} and {3,2,1}
  T U[4][E];
  double rd = 0.0, rp = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = a - 1 + i;
    if (m < 0 || m > nt || (!bdf2 && i == 0)) continue;
    const T* uo = u_in + (size_t)m * nx + seg0 + lane;
    T uv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) uv[e] = uo[64 * e];
    if (m == 0) {
#pragma unroll
      for (int e = 0; e < E; ++e) U[i][e] = uv[e];
      continue;
    }
    T g[E];
    dual_op_wave<T, E>(C, m, phibar, uv, seg0, lane, g);
#pragma unroll
    for (int e = 0; e < E; ++e) U[i][e] = uv[e] - tau_u * g[e];
    if (i >= 2) {   // owned level: store u^n and the dual residual of (u^{n-1}, phi^{n-1})
      T* uw = u_out + (size_t)m * nx + seg0 + lane;
#pragma unroll
      for (int e = 0; e < E; ++e) uw[64 * e] = U[i][e];
      dual_op_wave<T, E>(C, m, phi, uv, seg0, lane, g);
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

  // per-block partial sums, then the last block reduces them in a fixed order
  const int nblk = gridDim.x;
  const double srp = block_sum_tree(rp, red);
  const double srd = block_sum_tree(rd, red);
  if (tid == 0) {
    part[blockIdx.x] = srp;
    part[nblk + blockIdx.x] = srd;
    __threadfence();
    ticket = atomicAdd(counter, 1u);
  }
  __syncthreads();
  if (ticket != (unsigned)(nblk - 1)) return;
  __threadfence();
  double ta = 0.0, tb = 0.0;
  for (int i = tid; i < nblk; i += W) {
    ta += load_coherent(part + i);
    tb += load_coherent(part + nblk + i);
  }
  const double sa = block_sum_tree(ta, red);
  const double sb = block_sum_tree(tb, red);
  if (tid == 0) {
    finalize_body(ctrl, sa, sb, sch.ht * sch.hx, hist);
    *counter = 0u;
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

template <typename T, int BW, int LPL>
__global__ void __launch_bounds__(64 * kColWaves)
k_colsolve_wave(T* __restrict__ spec, FacTab<T> fac, int nt, int nx, int lqb, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  extern __shared__ char smem[];
  T* tile = reinterpret_cast<T*>(smem);   // [kColCols][LPL][65], level l of column c at (c LPL + l % LPL) 65 + l / LPL
  const int QB = 1 << lqb;
  const int q0 = blockIdx.x * kColCols;   // first spectrum column of this block
  T* base = spec + (size_t)(q0 >> lqb) * nt * QB + (q0 & (QB - 1));
  const int tid = threadIdx.x;
  for (int idx = tid; idx < nt * kColCols; idx += blockDim.x) {
    const int l = idx / kColCols, c = idx % kColCols;
    tile[(c * LPL + l % LPL) * 65 + l / LPL] = base[(size_t)l * QB + c];
  }
  __syncthreads();
  const int wv = tid >> 6, lane = tid & 63;
  const int qa = q0 + 2 * wv, qb = qa + 1;
  const int ka = spec_mode(qa, nx), kb = spec_mode(qb, nx);
  const int l0 = lane * LPL;
  T z[2][LPL];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int i = 0; i < LPL; ++i) z[c][i] = tile[((2 * wv + c) * LPL + i) * 65 + lane];
  T invd[LPL], e1[LPL + 1], e2[LPL + 2];
  if (ka == kb) {
    load_factor_rows<T, LPL>(fac, ka, l0, invd, e1, e2);
    cholesky_solve_wave<T, BW, LPL, 2>(z, invd, e1, e2, lane, l0, nt);
  } else {   // real columns of modes 0 and nx/2
    T za[1][LPL], zb[1][LPL];
#pragma unroll
    for (int i = 0; i < LPL; ++i) { za[0][i] = z[0][i]; zb[0][i] = z[1][i]; }
    load_factor_rows<T, LPL>(fac, ka, l0, invd, e1, e2);
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
  for (int idx = tid; idx < nt * kColCols; idx += blockDim.x) {
    const int l = idx / kColCols, c = idx % kColCols;
    base[(size_t)l * QB + c] = tile[(c * LPL + l % LPL) * 65 + l / LPL];
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

// A: EPT = clamp(nx / 64, 1, 8) points per thread (nx >= 64).
template <typename T>
hipError_t launch_dual_fft(const T* spec, int nt, int lqb, int nx, const void* tw, T* phi, T* phibar, T tau,
                           const Ctrl* ctrl, hipStream_t st) {
  switch (clampi(nx / 64, 1, 8)) {
    case 1: return launch_dual_fft_e<T, 1>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st);
    case 2: return launch_dual_fft_e<T, 2>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st);
    case 4: return launch_dual_fft_e<T, 4>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st);
    case 8: return launch_dual_fft_e<T, 8>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int E>
static hipError_t launch_primal_res_e(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi,
                                      T tau_u, T* spec, int lqb, const void* tw, double* part, Ctrl* ctrl,
                                      double* hist, unsigned* counter, hipStream_t st) {
  const int W = s.nx / E;
  const size_t lds = sizeof(C2<T>) * 2 * (size_t)lds_fft_points(s.nx) + sizeof(T) * 4 * (W / 64);
  hipError_t e = allow_lds(k_primal_res<T, E>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_primal_res<T, E>), dim3((s.nt + 1) / 2), dim3(W), lds, st, s, u_in, u_out, phibar, phi,
                     tau_u, spec, lqb, (const C2<T>*)tw, part, ctrl, hist, counter);
  return hipGetLastError();
}

// B: W = 64 * clamp(nx / 256, 1, 8) threads, E = nx / W points per thread (nx >= 64).
template <typename T>
hipError_t launch_primal_res(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                             T* spec, int lqb, const void* tw, double* part, Ctrl* ctrl, double* hist,
                             unsigned* counter, hipStream_t st) {
  const int W = 64 * clampi(s.nx / 256, 1, 8);
  switch (s.nx / W) {
    case 1: return launch_primal_res_e<T, 1>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, hist, counter, st);
    case 2: return launch_primal_res_e<T, 2>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, hist, counter, st);
    case 4: return launch_primal_res_e<T, 4>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, hist, counter, st);
    case 8: return launch_primal_res_e<T, 8>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, hist, counter, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int BW, int LPL>
static hipError_t launch_colsolve_wave_l(T* spec, const FacTab<T>& fac, int nt, int nx, int lqb, const Ctrl* ctrl,
                                         hipStream_t st) {
  const size_t lds = sizeof(T) * (size_t)kColCols * LPL * 65;
  hipError_t e = allow_lds(k_colsolve_wave<T, BW, LPL>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_colsolve_wave<T, BW, LPL>), dim3(nx / kColCols), dim3(64 * kColWaves), lds, st, spec, fac,
                     nt, nx, lqb, ctrl);
  return hipGetLastError();
}

// C: nt <= 1024, nx >= 8 (one wavefront per Fourier mode).
template <typename T>
hipError_t launch_colsolve_wave(T* spec, const FacTab<T>& fac, int bw, int nt, int nx, int lqb, const Ctrl* ctrl,
                                hipStream_t st) {
  const int lpl = (nt + 63) / 64;
#define PDHG_CW(B, L) return launch_colsolve_wave_l<T, B, L>(spec, fac, nt, nx, lqb, ctrl, st)
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
                                             float*, int, const void*, double*, Ctrl*, double*, unsigned*,
                                             hipStream_t);
template hipError_t launch_primal_res<double>(const Scheme&, const double*, double*, const double*, const double*,
                                              double, double*, int, const void*, double*, Ctrl*, double*,
                                              unsigned*, hipStream_t);
template hipError_t launch_colsolve_wave<float>(float*, const FacTab<float>&, int, int, int, int, const Ctrl*,
                                                hipStream_t);
template hipError_t launch_colsolve_wave<double>(double*, const FacTab<double>&, int, int, int, int, const Ctrl*,
                                                 hipStream_t);

}  // namespace pdhg
