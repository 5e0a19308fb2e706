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
//                      forward FFT (halfcomplex spectrum, column-block layout), and
//                      per-block partial sums of ||A(u^n)||^2 and of the dual
//                      residual (the latter only where the stopping test needs it)
//   C  k_colsolve_*    per spectrum column: banded Cholesky solve along t (the
//                      preconditioner K_d^{-1} of Section 2.2; k_colsolve_half for
//                      N_t <= 512, k_colsolve_wave up to 1024, k_colsolve_long up
//                      to 4096 (N_x = 8: 8192), beyond that k_colchunk_pass1, the
//                      carry pass and k_colchunk_pass2 on chunks of 256 levels); its
//                      first wave reduces B's partial sums and takes the convergence
//                      decision (Section 3.3 stopping rule)
// The pass bodies live in pdhg_passes.hpp (shared with the batched kernels).
// Halo levels of u^n needed by the time stencil of A are recomputed by each
// block from the same inputs (bitwise identical to the owner's values); u is
// ping-ponged between two buffers so no block reads a level another block has
// already overwritten.
#include "pdhg_internal.hpp"
#include "pdhg_passes.hpp"

namespace pdhg {

constexpr int kRowThreadsMax = 512;
// Row-pair blocks of the primal pass.  The pass holds about 18 E values per
// thread (four u levels twice, six phibar rows, four phi rows), so blocks of up
// to 1024 threads (4 waves per SIMD, <= 128 VGPRs) are possible while E values
// of type T fit in 16 bytes per row (FP32 E <= 4, FP64 E <= 2); larger E keeps
// 512-thread blocks.
template <typename T, int E>
constexpr int row_threads_max() { return E * (int)sizeof(T) <= 16 ? 1024 : 512; }

// A and B take a third N-point LDS array for the FFT (one barrier per stage
// instead of two) when the three arrays fit in 96 KiB: up to nx = 2048 in FP64
// and nx = 4096 in FP32.  The kernels and their launchers decide alike.
template <typename T>
__host__ __device__ constexpr bool fft_pingpong(int nx) { return 3 * (size_t)nx * sizeof(C2<T>) <= 98304; }

// Compute units of the current device (cached per device).
static int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

// Row-pair grids of at least two blocks per CU run their row passes for
// occupancy: A without the third LDS array (two blocks share a CU's LDS), B
// with the streaming body (a sliding window of rows in registers, no third LDS
// array).  A grid of at most one block per CU keeps the one-block layouts,
// whose load-everything-first order suits a block that has its CU to itself.
// Either way the arithmetic, and so every iterate, is the same.
static inline bool rows_for_occupancy(int nt) { return (nt + 1) / 2 >= 2 * device_cus(); }

// A: one block per pair of dual rows, W = nx / EPT threads; S is the type of
// the spectrum and of the FFT.
template <typename T, int EPT, typename S>
__global__ void __launch_bounds__(kRowThreadsMax)
k_dual_fft(const S* __restrict__ spec, int nt, int lqb, int nx, const C2<S>* __restrict__ tw, T* __restrict__ phi,
           T* __restrict__ phibar, T tau, const Ctrl* ctrl, const T* __restrict__ s0, int pp) {
  if (ctrl && ctrl->status != 0) return;
  extern __shared__ char smem[];
  C2<S>* buf = reinterpret_cast<C2<S>*>(smem);
  C2<S>* twl = buf + lds_fft_points(nx);
  const int tid = threadIdx.x, W = blockDim.x;
  const int a = 2 * xcd_block(blockIdx.x, gridDim.x);
  C2<S>* alt = pp ? twl + lds_fft_points(nx) : nullptr;
  dual_fft_pair<T, EPT, S>(spec, nt, lqb, nx, tw, phi, phibar, tau, a, tid, W, tid, W, buf, twl, alt, s0);
}

// B: one block per pair of implicit rows, W = 64 nw threads, E = nx / W.  The
// per-block partial sums go to part[blk] and part[gridDim + blk]; the column
// solve of the same iteration reduces them.  The per-wave sums are taken
// before the FFT, whose barriers publish them, and added up by thread 0 in
// wave order at the end (the order of block_sum_waves).
template <typename T, int E, typename S, bool STREAM>
__global__ void __launch_bounds__((STREAM ? 1024 : row_threads_max<T, E>()))
k_primal_res(Scheme sch, const T* __restrict__ u_in, T* __restrict__ u_out, const T* __restrict__ phibar,
             const T* __restrict__ phi, T tau_u, S* __restrict__ spec, int lqb, const C2<S>* __restrict__ tw,
             double* __restrict__ part, const Ctrl* ctrl, LamArgs<T> lam) {
  if (ctrl->status != 0) return;
  extern __shared__ char smem[];
  const Consts<T> C(sch);
  const int nx = sch.nx, W = blockDim.x, tid = threadIdx.x;
  C2<S>* buf = reinterpret_cast<C2<S>*>(smem);
  C2<S>* twl = buf + lds_fft_points(nx);
  const bool pp = !STREAM && fft_pingpong<S>(nx);
  C2<S>* alt = pp ? twl + lds_fft_points(nx) : nullptr;
  T* edge = reinterpret_cast<T*>(twl + (pp ? 2 : 1) * lds_fft_points(nx));   // [2 rows][first, last][nw]
  constexpr int kMaxWaves = (STREAM ? 1024 : row_threads_max<T, E>()) / 64;
  __shared__ double wsum[2 * kMaxWaves];
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const bool want_rd = rd_needed(ctrl);
  double rp, rd;
  primal_res_pair<T, E, S, STREAM>(C, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, 2 * blk, tid, W, tid, W, buf,
                                   twl, edge, rp, rd, alt, wsum, want_rd, &lam);
  if (tid == 0) {
    const int nw = W >> 6;
    double srp = 0.0, srd = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxWaves; ++i)
      if (i < nw) srp += wsum[i];
#pragma unroll
    for (int i = 0; i < kMaxWaves; ++i)
      if (i < nw) srd += wsum[nw + i];
    part[blk] = srp;
    part[gridDim.x + blk] = srd;
  }
}

// C: 8 waves per block, one spectrum column each.  With part != NULL the
// first wave of block 0 first reduces the iteration's partial sums and takes
// the stopping decision.
template <typename T, int BW, int LPL, typename A>
__global__ void __launch_bounds__(64 * kFdColWaves)
k_colsolve_wave(T* __restrict__ spec, FacTab<A> fac, int nt, int nx, int lqb, Ctrl* ctrl, const double* part,
                int nparts, double wscale, double* hist, A* s0) {
  if (ctrl && ctrl->status != 0) return;
  if (part && blockIdx.x == 0 && threadIdx.x < 64) finalize_wave(ctrl, part, nparts, nparts, wscale, hist);
  extern __shared__ char smem[];
  T* tile = reinterpret_cast<T*>(smem);
  colsolve_group<T, BW, LPL, A>(spec, fac, nt, nx, lqb, xcd_block(blockIdx.x, gridDim.x) * kColCols, tile, s0);
}

// C for N_t <= 512: kColsHalf columns per block, two per wave (32 lanes each).
constexpr int kColsHalf = 4;
template <typename T, int BW, int LPL, typename A>
__global__ void __launch_bounds__(32 * kColsHalf)
k_colsolve_half(T* __restrict__ spec, FacTab<A> fac, int nt, int nx, int lqb, Ctrl* ctrl, const double* part,
                int nparts, double wscale, double* hist, A* s0) {
  if (ctrl && ctrl->status != 0) return;
  if (part && blockIdx.x == 0 && threadIdx.x < 64) finalize_wave(ctrl, part, nparts, nparts, wscale, hist);
  extern __shared__ char smem[];
  T* tile = reinterpret_cast<T*>(smem);
  colsolve_group_half<T, BW, LPL, kColsHalf, 32, A>(spec, fac, nt, nx, lqb,
                                                    xcd_block(blockIdx.x, gridDim.x) * kColsHalf, tile, s0);
}

// C for N_t <= 256: kColsQuarter columns per block, four per wave (16 lanes each).
constexpr int kColsQuarter = 8;
template <typename T, int BW, int LPL, typename A>
__global__ void __launch_bounds__(16 * kColsQuarter)
k_colsolve_quarter(T* __restrict__ spec, FacTab<A> fac, int nt, int nx, int lqb, Ctrl* ctrl, const double* part,
                   int nparts, double wscale, double* hist, A* s0) {
  if (ctrl && ctrl->status != 0) return;
  if (part && blockIdx.x == 0 && threadIdx.x < 64) finalize_wave(ctrl, part, nparts, nparts, wscale, hist);
  extern __shared__ char smem[];
  T* tile = reinterpret_cast<T*>(smem);
  colsolve_group_half<T, BW, LPL, kColsQuarter, 16, A>(spec, fac, nt, nx, lqb,
                                                       xcd_block(blockIdx.x, gridDim.x) * kColsQuarter, tile, s0);
}

// C for 1024 < N_t <= 8192: WPC waves per column, 8 / WPC columns per block.
// Float recurrences are held to 128 VGPRs, so that two blocks share a CU.
template <typename T, int BW, int WPC, typename A>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(A) == 4 ? 4 : 1)))
k_colsolve_long(T* __restrict__ spec, FacTab<A> fac, int nt, int nx, int lqb, Ctrl* ctrl, const double* part,
                int nparts, double wscale, double* hist, A* s0) {
  if (ctrl && ctrl->status != 0) return;
  if (part && blockIdx.x == 0 && threadIdx.x < 64) finalize_wave(ctrl, part, nparts, nparts, wscale, hist);
  extern __shared__ char smem[];
  T* tile = reinterpret_cast<T*>(smem);
  A* xch = reinterpret_cast<A*>(tile + 8 * kColLongLpl * 65);
  colsolve_group_long<T, BW, kColLongLpl, WPC, A>(spec, fac, nt, nx, lqb,
                                                   xcd_block(blockIdx.x, gridDim.x) * (8 / WPC), tile, xch, s0);
}

// C for N_t > 4096 and N_x >= 16, in chunks of kChunkLevels levels (the
// chunked solve above): pass 1, the carry pass and pass 2, one block per
// (column block, chunk) in the passes.  The first wave of block 0 of pass 1
// reduces B's partial sums and takes the stopping decision; once a solve has
// stopped every later launch returns at once.  A float spectrum's column
// blocks below ca.g64 (the slowly decaying low modes) run in FP64.
template <typename A>
__device__ __forceinline__ const FacTab<A>& chunk_fac(const ChunkArgs& ca);
template <>
__device__ __forceinline__ const FacTab<double>& chunk_fac<double>(const ChunkArgs& ca) { return ca.f64; }
template <>
__device__ __forceinline__ const FacTab<float>& chunk_fac<float>(const ChunkArgs& ca) { return ca.f32; }

// Grids over a list of tiles (g nchunk + c), one tile per block, arithmetic
// type A; CST grids hold the tiles past every column's last distinct factor
// row.  The launcher runs FP64 and float recurrences, general and constant
// tiles as separate grids, so that each has its own register budget (a
// constant tile needs one factor row per lane instead of kChunkLpl + 2).
template <typename T, int BW, typename A, bool CST>
__global__ void __launch_bounds__(kChunkThreads)
k_colchunk_pass1(T* __restrict__ spec, ChunkArgs ca, const int* __restrict__ tiles, int nt, int nx, Ctrl* ctrl,
                 const double* part, int nparts, double wscale, double* hist) {
  if (ctrl && ctrl->status != 0) return;
  if (part && blockIdx.x == 0 && threadIdx.x < 64) finalize_wave(ctrl, part, nparts, nparts, wscale, hist);
  extern __shared__ char smem[];
  const int tl = tiles[xcd_block(blockIdx.x, gridDim.x)];
  colchunk_item<T, BW, A, false, CST>(spec, chunk_fac<A>(ca), ca, nt, nx, tl / ca.nchunk, tl % ca.nchunk,
                                      reinterpret_cast<T*>(smem), nullptr);
}

template <typename T, int BW, typename A, bool CST>
__global__ void __launch_bounds__(kChunkThreads)
k_colchunk_pass2(T* __restrict__ spec, ChunkArgs ca, const int* __restrict__ tiles, int nt, int nx, Ctrl* ctrl,
                 double* s0) {
  if (ctrl && ctrl->status != 0) return;
  extern __shared__ char smem[];
  const int tl = tiles[xcd_block(blockIdx.x, gridDim.x)];
  colchunk_item<T, BW, A, true, CST>(spec, chunk_fac<A>(ca), ca, nt, nx, tl / ca.nchunk, tl % ca.nchunk,
                                     reinterpret_cast<T*>(smem), s0);
}

// Entering states of every chunk: one 32-lane group per column, lane c for
// chunk c (nchunk <= 32).  The forward maps (H_c, P_c) are scanned up the
// chunks from t_0 = 0, then the backward maps (G_c, K_c t_c + R_c) down them
// from h_{nchunk-1} = 0; lanes past the last chunk hold the identity.  Writes
// (t_c, h_c) to fac.cwork[1][c].
constexpr int kChunkCarryThreads = 256;
__global__ void __launch_bounds__(kChunkCarryThreads)
k_colchunk_carry(ChunkArgs ca, int nx, Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  typedef double A;
  const int nc = ca.nchunk;
  const int lane = threadIdx.x & 63, c = lane & 31;
  const int j = blockIdx.x * (kChunkCarryThreads / 32) + (threadIdx.x >> 5);
  const bool act = c < nc && j < nx;
  A H[4] = {A(1), A(0), A(0), A(1)}, P[2] = {A(0), A(0)};
  A G[4] = {A(1), A(0), A(0), A(1)}, K[4] = {A(0), A(0), A(0), A(0)}, R[2] = {A(0), A(0)};
  if (act) {
    const A* m = ca.cmap + ((size_t)spec_mode(j, nx) * nc + c) * 12;
    const A* w = ca.cwork + ((size_t)c * nx + j) * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      H[k] = m[k];
      G[k] = m[4 + k];
      K[k] = m[8 + k];
    }
    P[0] = w[0]; P[1] = w[1];
    R[0] = w[2]; R[1] = w[3];
  }
  A t2, t1, h2, h1;
  scan_half_from<A, true>(H, P, lane, A(0), A(0), t2, t1);
  A Q[2] = {K[0] * t2 + K[1] * t1 + R[0], K[2] * t2 + K[3] * t1 + R[1]};
  scan_half_from<A, false>(G, Q, lane, A(0), A(0), h2, h1);
  if (act) {
    A* o = ca.cwork + ((size_t)(nc + c) * nx + j) * 4;
    o[0] = t2; o[1] = t1; o[2] = h2; o[3] = h1;
  }
}

// The maps of mode k and chunk c (one thread each) from the factor rows:
// H (forward homogeneous responses at the chunk's last two levels to the
// entering z_{s-2}, z_{s-1}), G (backward homogeneous responses at its first
// two levels to the entering y_{e+1}, y_e) and K (the backward solve, from
// zero, of the forward homogeneous responses, at the first two levels).  K is
// accumulated in the forward sweep: y_i = <L_c^{-1} e_i, v> for the chunk's
// diagonal block L_c of the factor.  out: [nmodes][nchunk][12] = H, G, K.
template <typename A, int BW>
__global__ void __launch_bounds__(256)
k_colchunk_maps(FacTab<A> fac, int nt, int nmodes, A* __restrict__ out) {
  const int nc = chunk_count(nt);
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nmodes * nc) return;
  const int k = idx / nc, c = idx % nc;
  const FacRow<A>* rows = fac.rows + fac.off[k];
  const int last = fac.last[k];
  const int s = c * kChunkLevels, e = min(nt, s + kChunkLevels);
  A a2 = 1, a1 = 0, b2 = 0, b1 = 1, u2 = 0, u1 = 0, v2 = 0, v1 = 0;
  A k0 = 0, k1 = 0, k2 = 0, k3 = 0;
  for (int l = s; l < e; ++l) {
    const FacRow<A> r = rows[min(l, last)];
    const A f2 = BW == 2 ? r.e2 : A(0);
    const A az = r.invd * (-(r.e1 * a1) - f2 * a2);
    const A bz = r.invd * (-(r.e1 * b1) - f2 * b2);
    const A uz = r.invd * ((l == s ? A(1) : A(0)) - r.e1 * u1 - f2 * u2);       // L_c^{-1} e_s
    const A vz = r.invd * ((l == s + 1 ? A(1) : A(0)) - r.e1 * v1 - f2 * v2);   // L_c^{-1} e_{s+1}
    a2 = a1; a1 = az; b2 = b1; b1 = bz; u2 = u1; u1 = uz; v2 = v1; v1 = vz;
    k0 += vz * az; k1 += vz * bz; k2 += uz * az; k3 += uz * bz;
  }
  A* o = out + (size_t)idx * 12;
  o[0] = a2; o[1] = b2; o[2] = a1; o[3] = b1;
  a2 = 1; a1 = 0; b2 = 0; b1 = 1;
  for (int l = e - 1; l >= s; --l) {
    const A invd = rows[min(l, last)].invd;
    const A f1 = rows[min(l + 1, last)].e1;
    const A f2 = BW == 2 ? rows[min(l + 2, last)].e2 : A(0);
    const A az = invd * (-(f1 * a1) - f2 * a2);
    const A bz = invd * (-(f1 * b1) - f2 * b2);
    a2 = a1; a1 = az; b2 = b1; b1 = bz;
  }
  o[4] = a2; o[5] = b2; o[6] = a1; o[7] = b1;
  o[8] = k0; o[9] = k1; o[10] = k2; o[11] = k3;
}

// C (full-symbol preconditioner): per Fourier mode k, K_k = L_k L_k^* with
// L_k = B_t + g_k I lower triangular (row l: c0(l)/h_t + g_k on the diagonal,
// c1(l)/h_t and c2(l)/h_t below it), g_k = (wr + vr)(1 - cos theta_k) + i ci sin theta_k
// the symbol of the linear-flux spatial operator (theta_k = 2 pi k / nx, from the
// twiddle table).  Forward substitution with L_k, backward with L_k^*.  Block of
// 4 waves = 8 spectrum columns; wave w owns columns 2w (Re) and 2w+1 (Im) of one
// mode as a complex column; the real columns 0 (mode 0) and 1 (mode nx/2) of
// block 0 are solved one after the other as real columns.  With part != NULL the
// first wave of block 0 first reduces the iteration's partial sums and takes the
// stopping decision.
template <typename T, int BW, int LPL>
__device__ __forceinline__ void full_rows(const FullSym& F, const C2<T>* __restrict__ tw, int kmode, int l0,
                                          Cx<T>* invd, Cx<T>* invb, T* e1, T* e2) {
  const C2<T> w = tw[kmode];   // (cos theta, -sin theta)
  const T omc = T(1) - w.x;
  const Cx<T> g((T(F.wr) + T(F.vr)) * omc, -T(F.ci) * w.y);
  const T iht = T(F.inv_ht);
#pragma unroll
  for (int i = 0; i < LPL; ++i) {
    const int l = l0 + i;
    const T c0 = (F.bdf2 && l >= 1) ? T(1.5) : T(1);
    const Cx<T> d(c0 * iht + g.re, g.im);
    const T den = T(1) / (d.re * d.re + d.im * d.im);
    invd[i] = Cx<T>(d.re * den, -d.im * den);
    invb[i] = Cx<T>(d.re * den, d.im * den);
  }
#pragma unroll
  for (int i = 0; i <= LPL; ++i) {
    const int l = l0 + i;
    e1[i] = (l >= 1) ? ((F.bdf2 ? T(-2) : T(-1)) * iht) : T(0);
  }
#pragma unroll
  for (int i = 0; i <= LPL + 1; ++i) {
    const int l = l0 + i;
    e2[i] = (F.bdf2 && l >= 2) ? T(0.5) * iht : T(0);
  }
}

template <typename T, int BW, int LPL>
__global__ void __launch_bounds__(64 * kColWaves)
k_colsolve_full(T* __restrict__ spec, FullSym F, const C2<T>* __restrict__ tw, int nt, int nx, int lqb, Ctrl* ctrl,
                const double* part, int nparts, double wscale, double* hist) {
  if (ctrl && ctrl->status != 0) return;
  if (part && blockIdx.x == 0 && threadIdx.x < 64) finalize_wave(ctrl, part, nparts, nparts, wscale, hist);
  extern __shared__ char smem[];
  T* tile = reinterpret_cast<T*>(smem);   // [8 cols][LPL][65]
  const int QB = 1 << lqb;
  const int q0 = xcd_block(blockIdx.x, gridDim.x) * kColCols;
  T* base = spec + (size_t)(q0 >> lqb) * nt * QB + (q0 & (QB - 1));
  constexpr int kThreads = 64 * kColWaves;
  constexpr int kPer = 64 * LPL * kColCols / kThreads;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int l0 = lane * LPL;
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
  const int ca = 2 * wv, cb = 2 * wv + 1;
  Cx<T> invd[LPL], invb[LPL];
  T e1[LPL + 1], e2[LPL + 2];
  Cx<T> z[1][LPL];
  if (q0 + ca != 0) {   // complex mode (q0 + ca) / 2
    full_rows<T, BW, LPL>(F, tw, (q0 + ca) >> 1, l0, invd, invb, e1, e2);
#pragma unroll
    for (int i = 0; i < LPL; ++i)
      z[0][i] = Cx<T>(tile[(ca * LPL + i) * 65 + lane], tile[(cb * LPL + i) * 65 + lane]);
    tri_solve_wave<Cx<T>, T, BW, LPL, 1>(z, invd, invb, e1, e2, lane, l0, nt);
#pragma unroll
    for (int i = 0; i < LPL; ++i) {
      tile[(ca * LPL + i) * 65 + lane] = z[0][i].re;
      tile[(cb * LPL + i) * 65 + lane] = z[0][i].im;
    }
  } else {              // real columns: mode 0 in column 0, mode nx/2 in column 1
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = h;
      full_rows<T, BW, LPL>(F, tw, h ? nx / 2 : 0, l0, invd, invb, e1, e2);
#pragma unroll
      for (int i = 0; i < LPL; ++i) z[0][i] = Cx<T>(tile[(c * LPL + i) * 65 + lane], T(0));
      tri_solve_wave<Cx<T>, T, BW, LPL, 1>(z, invd, invb, e1, e2, lane, l0, nt);
#pragma unroll
      for (int i = 0; i < LPL; ++i) tile[(c * LPL + i) * 65 + lane] = z[0][i].re;
    }
  }
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

// ------------------------------------------------------------------ launchers
static inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

template <typename T, int BW, int LPL>
static hipError_t launch_colsolve_full_l(T* spec, const FullSym& F, const void* tw, int nt, int nx, int lqb,
                                         Ctrl* ctrl, const double* part, int nparts, double wscale, double* hist,
                                         hipStream_t st) {
  const size_t lds = sizeof(T) * (size_t)kColCols * LPL * 65;
  hipError_t e = allow_lds(k_colsolve_full<T, BW, LPL>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_colsolve_full<T, BW, LPL>), dim3(nx / kColCols), dim3(64 * kColWaves), lds, st, spec, F,
                     (const C2<T>*)tw, nt, nx, lqb, ctrl, part, nparts, wscale, hist);
  return hipGetLastError();
}

// Full-symbol C: nt <= 1024, nx >= 8; part != NULL as for launch_colsolve_wave.
template <typename T>
hipError_t launch_colsolve_full(T* spec, const FullSym& F, const void* tw, int nt, int nx, int lqb, Ctrl* ctrl,
                                const double* part, int nparts, double wscale, double* hist, hipStream_t st) {
  const int lpl = (nt + 63) / 64;
#define PDHG_CF(B, L) \
  return launch_colsolve_full_l<T, B, L>(spec, F, tw, nt, nx, lqb, ctrl, part, nparts, wscale, hist, st)
  if (F.bdf2) {
    if (lpl <= 1) PDHG_CF(2, 1);
    if (lpl <= 2) PDHG_CF(2, 2);
    if (lpl <= 4) PDHG_CF(2, 4);
    if (lpl <= 8) PDHG_CF(2, 8);
    if (lpl <= 16) PDHG_CF(2, 16);
  } else {
    if (lpl <= 1) PDHG_CF(1, 1);
    if (lpl <= 2) PDHG_CF(1, 2);
    if (lpl <= 4) PDHG_CF(1, 4);
    if (lpl <= 8) PDHG_CF(1, 8);
    if (lpl <= 16) PDHG_CF(1, 16);
  }
#undef PDHG_CF
  return hipErrorInvalidValue;
}

template <typename T, int EPT, typename S>
static hipError_t launch_dual_fft_e(const S* spec, int nt, int lqb, int nx, const void* tw, T* phi, T* phibar, T tau,
                                    const Ctrl* ctrl, hipStream_t st, const T* s0) {
  const int W = nx / EPT;
  const int pp = fft_pingpong<S>(nx) && !rows_for_occupancy(nt);
  const size_t lds = sizeof(C2<S>) * (pp ? 3 : 2) * (size_t)lds_fft_points(nx);
  hipError_t e = allow_lds(k_dual_fft<T, EPT, S>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_dual_fft<T, EPT, S>), dim3((nt + 1) / 2), dim3(W), lds, st, spec, nt, lqb, nx,
                     (const C2<S>*)tw, phi, phibar, tau, ctrl, s0, pp);
  return hipGetLastError();
}

// A: nx >= 64.
template <typename T, typename S>
hipError_t launch_dual_fft(const S* spec, int nt, int lqb, int nx, const void* tw, T* phi, T* phibar, T tau,
                           const Ctrl* ctrl, hipStream_t st, const T* s0) {
  // EPT = nx / W with W = min(512, nx / 2) threads for nx >= 128 (8 waves at nx = 2048)
  const int W = nx >= 1024 ? 512 : (nx >= 128 ? nx / 2 : nx);
  switch (nx / W) {
    case 1: return launch_dual_fft_e<T, 1, S>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st, s0);
    case 2: return launch_dual_fft_e<T, 2, S>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st, s0);
    case 4: return launch_dual_fft_e<T, 4, S>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st, s0);
    case 8: return launch_dual_fft_e<T, 8, S>(spec, nt, lqb, nx, tw, phi, phibar, tau, ctrl, st, s0);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int E, typename S, bool STREAM = false>
static hipError_t launch_primal_res_e(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi,
                                      T tau_u, S* spec, int lqb, const void* tw, double* part, const Ctrl* ctrl,
                                      hipStream_t st, const LamArgs<T>& lam) {
  const int W = s.nx / E;
  const bool pp = !STREAM && fft_pingpong<S>(s.nx);
  const size_t lds = sizeof(C2<S>) * (pp ? 3 : 2) * (size_t)lds_fft_points(s.nx) + sizeof(T) * 4 * (W / 64);
  hipError_t e = allow_lds(k_primal_res<T, E, S, STREAM>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_primal_res<T, E, S, STREAM>), dim3((s.nt + 1) / 2), dim3(W), lds, st, s, u_in, u_out,
                     phibar, phi, tau_u, spec, lqb, (const C2<S>*)tw, part, ctrl, lam);
  return hipGetLastError();
}

// B: E = 4 points per thread in FP32 (W = nx / 4 <= 1024 threads); in FP64
// E = 2 up to nx = 2048 (W = nx / 2 <= 1024), E = 8 at nx = 4096 (W = 512);
// W >= 64 (nx >= 64).  Grids of two or more blocks per CU (rows_for_occupancy)
// take the streaming body with E = 8 in FP32 (W = nx / 8) and E = 4 in FP64
// (W = nx / 4), from nx = 512 and 256 on; FP64 at nx = 4096 always streams
// (W = 1024): its load-first body would spill.
template <typename T, typename S>
hipError_t launch_primal_res(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                             S* spec, int lqb, const void* tw, double* part, const Ctrl* ctrl, hipStream_t st,
                             const LamArgs<T>* lam) {
  const LamArgs<T> la = lam ? *lam : LamArgs<T>{nullptr, nullptr, nullptr, T(0), T(0)};
  const bool occ = rows_for_occupancy(s.nt);
  if constexpr (sizeof(T) == 4) {
    if (occ && s.nx >= 512)
      return launch_primal_res_e<T, 8, S, true>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, st,
                                                la);
  } else {
    if ((occ && s.nx >= 256) || s.nx == 4096)
      return launch_primal_res_e<T, 4, S, true>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, st,
                                                la);
  }
  int W;
  if (sizeof(T) == 4) W = clampi(s.nx / 4, 64, 1024);
  else W = s.nx <= 2048 ? clampi(s.nx / 2, 64, 1024) : 512;
  switch (s.nx / W) {
    case 1: return launch_primal_res_e<T, 1, S>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, st, la);
    case 2: return launch_primal_res_e<T, 2, S>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, st, la);
    case 4: return launch_primal_res_e<T, 4, S>(s, u_in, u_out, phibar, phi, tau_u, spec, lqb, tw, part, ctrl, st, la);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int BW, int LPL, typename A>
static hipError_t launch_colsolve_half_l(T* spec, const FacTab<A>& fac, int nt, int nx, int lqb, Ctrl* ctrl,
                                         const double* part, int nparts, double wscale, double* hist,
                                         hipStream_t st, A* s0) {
  const size_t lds = sizeof(T) * (size_t)kColsHalf * LPL * 33;
  hipError_t e = allow_lds(k_colsolve_half<T, BW, LPL, A>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_colsolve_half<T, BW, LPL, A>), dim3(nx / kColsHalf), dim3(32 * kColsHalf), lds, st, spec,
                     fac, nt, nx, lqb, ctrl, part, nparts, wscale, hist, s0);
  return hipGetLastError();
}

template <typename T, int BW, int LPL, typename A>
static hipError_t launch_colsolve_quarter_l(T* spec, const FacTab<A>& fac, int nt, int nx, int lqb, Ctrl* ctrl,
                                            const double* part, int nparts, double wscale, double* hist,
                                            hipStream_t st, A* s0) {
  const size_t lds = sizeof(T) * (size_t)kColsQuarter * LPL * 17;
  hipError_t e = allow_lds(k_colsolve_quarter<T, BW, LPL, A>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_colsolve_quarter<T, BW, LPL, A>), dim3(nx / kColsQuarter), dim3(16 * kColsQuarter), lds, st,
                     spec, fac, nt, nx, lqb, ctrl, part, nparts, wscale, hist, s0);
  return hipGetLastError();
}

template <typename T, int BW, int LPL, typename A>
static hipError_t launch_colsolve_wave_l(T* spec, const FacTab<A>& fac, int nt, int nx, int lqb, Ctrl* ctrl,
                                         const double* part, int nparts, double wscale, double* hist,
                                         hipStream_t st, A* s0) {
  const size_t lds = sizeof(T) * (size_t)kColCols * LPL * 65;
  hipError_t e = allow_lds(k_colsolve_wave<T, BW, LPL, A>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_colsolve_wave<T, BW, LPL, A>), dim3(nx / kColCols), dim3(64 * kFdColWaves), lds, st, spec, fac,
                     nt, nx, lqb, ctrl, part, nparts, wscale, hist, s0);
  return hipGetLastError();
}

template <typename T, int BW, int WPC, typename A>
static hipError_t launch_colsolve_long_l(T* spec, const FacTab<A>& fac, int nt, int nx, int lqb, Ctrl* ctrl,
                                         const double* part, int nparts, double wscale, double* hist,
                                         hipStream_t st, A* s0) {
  const size_t lds = sizeof(T) * (size_t)8 * kColLongLpl * 65 + sizeof(A) * 48;
  hipError_t e = allow_lds(k_colsolve_long<T, BW, WPC, A>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_colsolve_long<T, BW, WPC, A>), dim3(nx / (8 / WPC)), dim3(512), lds, st, spec, fac, nt, nx,
                     lqb, ctrl, part, nparts, wscale, hist, s0);
  return hipGetLastError();
}

template <typename T, int BW>
static hipError_t launch_colsolve_chunk_l(T* spec, const ChunkArgs& ca, int nt, int nx, Ctrl* ctrl,
                                          const double* part, int nparts, double wscale, double* hist,
                                          hipStream_t st, double* s0) {
  const size_t lds = sizeof(T) * (size_t)kChunkCols * kChunkLpl * (kChunkCw + 1) +
                     sizeof(double) * kChunkCols * (kChunkPow + 1) * 4;   // the tile, the powers, the states
  // the four grids of a pass, in order: FP64 general, FP64 constant, float general, float constant (the float
  // grids only for a float spectrum); the first grid launched reduces the partial sums
  auto pass1 = [&](auto tg, auto cg, int k) -> hipError_t {
    using A = decltype(tg);
    constexpr bool CST = decltype(cg)::value;
    if (ca.ntile[k] == 0) return hipSuccess;
    hipError_t r = allow_lds(k_colchunk_pass1<T, BW, A, CST>, lds);
    if (r != hipSuccess) return r;
    hipLaunchKernelGGL((k_colchunk_pass1<T, BW, A, CST>), dim3(ca.ntile[k]), dim3(kChunkThreads), lds, st, spec, ca,
                       ca.tiles + ca.toff[k], nt, nx, ctrl, part, nparts, wscale, hist);
    part = nullptr;
    return hipGetLastError();
  };
  auto pass2 = [&](auto tg, auto cg, int k) -> hipError_t {
    using A = decltype(tg);
    constexpr bool CST = decltype(cg)::value;
    if (ca.ntile[k] == 0) return hipSuccess;
    hipError_t r = allow_lds(k_colchunk_pass2<T, BW, A, CST>, lds);
    if (r != hipSuccess) return r;
    hipLaunchKernelGGL((k_colchunk_pass2<T, BW, A, CST>), dim3(ca.ntile[k]), dim3(kChunkThreads), lds, st, spec, ca,
                       ca.tiles + ca.toff[k], nt, nx, ctrl, s0);
    return hipGetLastError();
  };
  using F = std::false_type;
  using Tr = std::true_type;
  hipError_t e;
  if ((e = pass1(0.0, F{}, 0)) != hipSuccess || (e = pass1(0.0, Tr{}, 1)) != hipSuccess) return e;
  if constexpr (sizeof(T) == 4) {
    if ((e = pass1(0.0f, F{}, 2)) != hipSuccess || (e = pass1(0.0f, Tr{}, 3)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_colchunk_carry, dim3((nx + 7) / 8), dim3(kChunkCarryThreads), 0, st, ca, nx, ctrl);
  if ((e = pass2(0.0, F{}, 0)) != hipSuccess || (e = pass2(0.0, Tr{}, 1)) != hipSuccess) return e;
  if constexpr (sizeof(T) == 4) {
    if ((e = pass2(0.0f, F{}, 2)) != hipSuccess || (e = pass2(0.0f, Tr{}, 3)) != hipSuccess) return e;
  }
  return hipGetLastError();
}

// C in chunks: N_t >= kChunkMinNt, N_x >= 16 (column blocks of 16), at most 32
// chunks.  ctrl, part, nparts, wscale, hist as for launch_colsolve_wave; s0
// (nullable): receives the mode-0 column of the solution in FP64.
template <typename T>
hipError_t launch_colsolve_chunk(T* spec, const ChunkArgs& ca, int bw, int nt, int nx, int lqb, Ctrl* ctrl,
                                 const double* part, int nparts, double wscale, double* hist, hipStream_t st,
                                 double* s0) {
  if (nt < kChunkMinNt || nx < kChunkCols || lqb != 4 || ca.nchunk != chunk_count(nt) || ca.nchunk > 32 ||
      !ca.cmap || !ca.cpow || !ca.cwork || !ca.f64.rows || !ca.tiles ||
      ca.ntile[0] + ca.ntile[1] + ca.ntile[2] + ca.ntile[3] != (nx / kChunkCols) * ca.nchunk ||
      (sizeof(T) == 8 && ca.ntile[2] + ca.ntile[3] != 0))
    return hipErrorInvalidValue;
  if (bw == 2) return launch_colsolve_chunk_l<T, 2>(spec, ca, nt, nx, ctrl, part, nparts, wscale, hist, st, s0);
  return launch_colsolve_chunk_l<T, 1>(spec, ca, nt, nx, ctrl, part, nparts, wscale, hist, st, s0);
}
template hipError_t launch_colsolve_chunk<float>(float*, const ChunkArgs&, int, int, int, int, Ctrl*, const double*,
                                                 int, double, double*, hipStream_t, double*);
template hipError_t launch_colsolve_chunk<double>(double*, const ChunkArgs&, int, int, int, int, Ctrl*,
                                                  const double*, int, double, double*, hipStream_t, double*);

// The segment map M of every mode past its last distinct factor row (one
// thread per mode; kChunkLpl steps of the homogeneous recurrence on row
// `last`, the layout of the scan's H) and its repeated squares.
template <int BW>
__global__ void __launch_bounds__(256)
k_colchunk_powers(FacTab<double> fac, int nmodes, double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nmodes) return;
  const FacRow<double> r = fac.rows[fac.off[k] + fac.last[k]];
  const double e2 = BW == 2 ? r.e2 : 0.0;
  double a2 = 1, a1 = 0, b2 = 0, b1 = 1;
  for (int i = 0; i < kChunkLpl; ++i) {
    const double az = r.invd * (-(r.e1 * a1) - e2 * a2);
    const double bz = r.invd * (-(r.e1 * b1) - e2 * b2);
    a2 = a1; a1 = az; b2 = b1; b1 = bz;
  }
  double m[4] = {a2, b2, a1, b1};
  double* o = out + (size_t)k * kChunkPow * 4;
  for (int s = 0; s < kChunkPow; ++s) {
    for (int i = 0; i < 4; ++i) o[4 * s + i] = m[i];
    const double s0 = m[0] * m[0] + m[1] * m[2], s1 = m[0] * m[1] + m[1] * m[3];
    const double s2 = m[2] * m[0] + m[3] * m[2], s3 = m[2] * m[1] + m[3] * m[3];
    m[0] = s0; m[1] = s1; m[2] = s2; m[3] = s3;
  }
}

hipError_t launch_colchunk_powers(const FacTab<double>& fac, int bw, int nmodes, double* out, hipStream_t st) {
  if (bw == 2)
    hipLaunchKernelGGL(k_colchunk_powers<2>, dim3((nmodes + 255) / 256), dim3(256), 0, st, fac, nmodes, out);
  else
    hipLaunchKernelGGL(k_colchunk_powers<1>, dim3((nmodes + 255) / 256), dim3(256), 0, st, fac, nmodes, out);
  return hipGetLastError();
}

template <typename A>
hipError_t launch_colchunk_maps(const FacTab<A>& fac, int bw, int nt, int nmodes, A* out, hipStream_t st) {
  const int n = nmodes * chunk_count(nt);
  if (bw == 2)
    hipLaunchKernelGGL((k_colchunk_maps<A, 2>), dim3((n + 255) / 256), dim3(256), 0, st, fac, nt, nmodes, out);
  else
    hipLaunchKernelGGL((k_colchunk_maps<A, 1>), dim3((n + 255) / 256), dim3(256), 0, st, fac, nt, nmodes, out);
  return hipGetLastError();
}
template hipError_t launch_colchunk_maps<double>(const FacTab<double>&, int, int, int, double*, hipStream_t);

// C: nt <= 8192, nx >= 8.  With part != NULL the
// first wave of block 0 also reduces the iteration's residual partial sums and
// takes the stopping decision (ctrl must then be non-NULL).  N_t <= 256: four
// 16-lane columns per wave; up to 512: two 32-lane columns per wave; up to
// 1024: one wavefront per column; beyond: 2, 4 or 8 wavefronts per column.
template <typename T, typename A>
hipError_t launch_colsolve_wave(T* spec, const FacTab<A>& fac, int bw, int nt, int nx, int lqb, Ctrl* ctrl,
                                const double* part, int nparts, double wscale, double* hist, hipStream_t st, A* s0) {
  if (nt <= 256) {
    const int lq = (nt + 15) / 16;
#define PDHG_CQ(B, L) \
  return launch_colsolve_quarter_l<T, B, L, A>(spec, fac, nt, nx, lqb, ctrl, part, nparts, wscale, hist, st, s0)
    if (bw == 2) {
      if (lq <= 1) PDHG_CQ(2, 1);
      if (lq <= 2) PDHG_CQ(2, 2);
      if (lq <= 4) PDHG_CQ(2, 4);
      if (lq <= 8) PDHG_CQ(2, 8);
      PDHG_CQ(2, 16);
    } else {
      if (lq <= 1) PDHG_CQ(1, 1);
      if (lq <= 2) PDHG_CQ(1, 2);
      if (lq <= 4) PDHG_CQ(1, 4);
      if (lq <= 8) PDHG_CQ(1, 8);
      PDHG_CQ(1, 16);
    }
#undef PDHG_CQ
  }
  if (nt <= 512) {
    const int lh = (nt + 31) / 32;
#define PDHG_CH(B, L) \
  return launch_colsolve_half_l<T, B, L, A>(spec, fac, nt, nx, lqb, ctrl, part, nparts, wscale, hist, st, s0)
    if (bw == 2) {
      if (lh <= 1) PDHG_CH(2, 1);
      if (lh <= 2) PDHG_CH(2, 2);
      if (lh <= 4) PDHG_CH(2, 4);
      if (lh <= 8) PDHG_CH(2, 8);
      PDHG_CH(2, 16);
    } else {
      if (lh <= 1) PDHG_CH(1, 1);
      if (lh <= 2) PDHG_CH(1, 2);
      if (lh <= 4) PDHG_CH(1, 4);
      if (lh <= 8) PDHG_CH(1, 8);
      PDHG_CH(1, 16);
    }
#undef PDHG_CH
  }
  const int lpl = (nt + 63) / 64;
#define PDHG_CW(B, L) \
  return launch_colsolve_wave_l<T, B, L, A>(spec, fac, nt, nx, lqb, ctrl, part, nparts, wscale, hist, st, s0)
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
#define PDHG_CL(B, W) \
  return launch_colsolve_long_l<T, B, W, A>(spec, fac, nt, nx, lqb, ctrl, part, nparts, wscale, hist, st, s0)
  const int wpc = (nt + 64 * kColLongLpl - 1) / (64 * kColLongLpl);
  if (bw == 2) {
    if (wpc <= 2) PDHG_CL(2, 2);
    if (wpc <= 4) PDHG_CL(2, 4);
    if (wpc <= 8) PDHG_CL(2, 8);
  } else {
    if (wpc <= 2) PDHG_CL(1, 2);
    if (wpc <= 4) PDHG_CL(1, 4);
    if (wpc <= 8) PDHG_CL(1, 8);
  }
#undef PDHG_CL
  return hipErrorInvalidValue;
}

template hipError_t launch_dual_fft<float, float>(const float*, int, int, int, const void*, float*, float*, float,
                                                  const Ctrl*, hipStream_t, const float*);
template hipError_t launch_dual_fft<double, double>(const double*, int, int, int, const void*, double*, double*,
                                                    double, const Ctrl*, hipStream_t, const double*);
template hipError_t launch_dual_fft<double, float>(const float*, int, int, int, const void*, double*, double*,
                                                   double, const Ctrl*, hipStream_t, const double*);
template hipError_t launch_primal_res<float, float>(const Scheme&, const float*, float*, const float*, const float*,
                                                    float, float*, int, const void*, double*, const Ctrl*,
                                                    hipStream_t, const LamArgs<float>*);
template hipError_t launch_primal_res<double, double>(const Scheme&, const double*, double*, const double*,
                                                      const double*, double, double*, int, const void*, double*,
                                                      const Ctrl*, hipStream_t, const LamArgs<double>*);
template hipError_t launch_primal_res<double, float>(const Scheme&, const double*, double*, const double*,
                                                     const double*, double, float*, int, const void*, double*,
                                                     const Ctrl*, hipStream_t, const LamArgs<double>*);
template hipError_t launch_colsolve_wave<float, float>(float*, const FacTab<float>&, int, int, int, int, Ctrl*,
                                                       const double*, int, double, double*, hipStream_t, float*);
template hipError_t launch_colsolve_wave<float, double>(float*, const FacTab<double>&, int, int, int, int, Ctrl*,
                                                        const double*, int, double, double*, hipStream_t, double*);
template hipError_t launch_colsolve_full<float>(float*, const FullSym&, const void*, int, int, int, Ctrl*,
                                                const double*, int, double, double*, hipStream_t);
template hipError_t launch_colsolve_full<double>(double*, const FullSym&, const void*, int, int, int, Ctrl*,
                                                 const double*, int, double, double*, hipStream_t);
template hipError_t launch_colsolve_wave<double, double>(double*, const FacTab<double>&, int, int, int, int, Ctrl*,
                                                         const double*, int, double, double*, hipStream_t, double*);

}  // namespace pdhg
