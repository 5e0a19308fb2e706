// Batched solver: many independent problems of uneven N_x and N_t advance
// together, one launch per pass of the fused iteration (A, B, C of
// pdhg_passes.hpp) for the whole batch.
//
// * Problem table (BatchProb): sizes, scheme, step sizes and the offsets of the
//   problem's slices in the packed u, phi/phibar/spectrum and u0 arrays.
// * Work lists, rebuilt on the device at the end of every graph chunk from the
//   per-problem control blocks (converged problems drop out):
//     row tiles   (p, first pair): S = TB / W row pairs of problem p, one per
//                 sub-group of W = nx / EPT threads (every tile of a block has
//                 the same shape, so all tiles cost the same TB EPT points)
//     col tiles   (p, column group): 8 spectrum columns of problem p
//   Row tiles list the problems of 4 points per thread first (counts[3] of
//   them), then those of 8, so that the primal pass runs one grid for each,
//   each with its own register budget.
// * Persistent grids: blocks take contiguous ranges of row tiles (neighbouring
//   pairs share halo rows; the range of XCD x is contiguous) and strided
//   column tiles (ordered by decreasing N_t, so every block gets a mix of
//   long and short columns).
// * Per-problem convergence: the block that solves column group 0 of problem
//   p first reduces p's partial sums and takes p's stopping decision.
#include "pdhg_internal.hpp"
#include "pdhg_passes.hpp"

namespace pdhg {

// Row tile shape for rows of length nx in a block of TB threads:
// EPT = 4 points per thread when nx <= 4 TB, else 8 (nx = 8 TB).
constexpr int kBatchMaxNx = 4096;
constexpr int kBatchRowThreads = 512;   // threads of a row-pass block, either type
__host__ __device__ constexpr int batch_ept(int nx, int TB) { return nx <= 4 * TB ? 4 : 8; }
// The primal pass runs the streaming body in FP32 (see batch_row_threads).
template <typename T>
constexpr bool batch_stream() { return sizeof(T) == 4; }
// Whether blocks of TB threads ever need the EPT = 8 bodies.
template <int TB>
constexpr bool batch_needs_e8() { return 4 * TB < kBatchMaxNx; }

// LDS of the row kernels: twiddles (max nx) + S FFT buffers + edges.
__host__ __device__ inline size_t batch_row_lds_points(int max_nx, int min_nx, int TB) {
  size_t bufpts = 0;
  for (int nx = min_nx; nx <= max_nx; nx *= 2) {
    const int W = nx / batch_ept(nx, TB);
    const size_t s = (size_t)(TB / W) * lds_fft_points(nx);
    if (s > bufpts) bufpts = s;
  }
  return (size_t)lds_fft_points(max_nx) + bufpts;
}

template <typename T, int TB>
__device__ __forceinline__ void row_tile_geometry(int nx, int& W, int& sg, int& tid, C2<T>*& buf, C2<T>*& twl,
                                                  char* smem, int max_nx) {
  W = nx / batch_ept(nx, TB);
  sg = threadIdx.x / W;
  tid = threadIdx.x - sg * W;
  twl = reinterpret_cast<C2<T>*>(smem);
  buf = twl + lds_fft_points(max_nx) + (size_t)sg * lds_fft_points(nx);
}

// Contiguous range of n items for logical block lb of G.
__device__ __forceinline__ void block_range(int n, int lb, int G, int& t0, int& t1) {
  t0 = (int)((long long)lb * n / G);
  t1 = (int)((long long)(lb + 1) * n / G);
}

// ------------------------------------------------------------------ A
template <typename T, int TB>
__global__ void __launch_bounds__(TB)
kb_dual_fft(const BatchProb* __restrict__ probs, const Ctrl* __restrict__ ctrls, const int2* __restrict__ tiles,
            const int* __restrict__ counts, int max_nx, T* __restrict__ spec, T* __restrict__ phi,
            T* __restrict__ phibar) {
  extern __shared__ char smem[];
  int t0, t1;
  block_range(counts[0], xcd_block(blockIdx.x, gridDim.x), gridDim.x, t0, t1);
  for (int t = t0; t < t1; ++t) {
    const int2 td = tiles[t];
    if (ctrls[td.x].status != 0) continue;   // ctrl is not written during this pass: uniform
    const BatchProb& P = probs[td.x];
    const int nx = P.s.nx, nt = P.s.nt;
    int W, sg, tid;
    C2<T>* buf;
    C2<T>* twl;
    row_tile_geometry<T, TB>(nx, W, sg, tid, buf, twl, smem, max_nx);
    const int a = 2 * (td.y + sg);
    const C2<T>* tw = as_global(static_cast<const C2<T>*>(P.tw));
    __syncthreads();   // LDS of the previous tile is free
    if (!batch_needs_e8<TB>() || batch_ept(nx, TB) == 4)
      dual_fft_pair<T, 4>(spec + P.f_off, nt, P.lqb, nx, tw, phi + P.f_off, phibar + P.f_off, (T)P.tau_phi, a, tid,
                          W, threadIdx.x, TB, buf, twl);
    else if constexpr (batch_needs_e8<TB>())
      dual_fft_pair<T, 8>(spec + P.f_off, nt, P.lqb, nx, tw, phi + P.f_off, phibar + P.f_off, (T)P.tau_phi, a, tid,
                          W, threadIdx.x, TB, buf, twl);
  }
}

// ------------------------------------------------------------------ B
// Partial sums: part[P.part_off + pair] (residual) and part[rd_base + P.part_off
// + pair] (dual residual), one per row pair.
// E: the points per thread of the tiles this grid takes (where problems of
// both kinds can occur, tiles [0, counts[3]) have 4 and the rest 8).
template <typename T, int TB, int E>
__global__ void __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(batch_stream<T>() ? 4 : 1)))
kb_primal_res(const BatchProb* __restrict__ probs, const Ctrl* __restrict__ ctrls, const int2* __restrict__ tiles,
              const int* __restrict__ counts, int max_nx, const T* __restrict__ u_in, T* __restrict__ u_out,
              const T* __restrict__ phibar, const T* __restrict__ phi, T* __restrict__ spec,
              double* __restrict__ part, int rd_base) {
  extern __shared__ char smem[];
  __shared__ double red[TB / 64];
  T* edge_all = reinterpret_cast<T*>(smem + sizeof(C2<T>) * batch_row_lds_points(max_nx, 256, TB));
  const int base = (batch_needs_e8<TB>() && E == 8) ? counts[3] : 0;
  const int n = batch_needs_e8<TB>() ? (E == 4 ? counts[3] : counts[0] - counts[3]) : counts[0];
  int t0, t1;
  block_range(n, xcd_block(blockIdx.x, gridDim.x), gridDim.x, t0, t1);
  for (int t = base + t0; t < base + t1; ++t) {
    const int2 td = tiles[t];
    if (ctrls[td.x].status != 0) continue;
    const BatchProb& P = probs[td.x];
    const int nx = P.s.nx;
    int W, sg, tid;
    C2<T>* buf;
    C2<T>* twl;
    row_tile_geometry<T, TB>(nx, W, sg, tid, buf, twl, smem, max_nx);
    const int nw = W >> 6;
    T* edge = edge_all + sg * 4 * nw;
    const int pair = td.y + sg;
    const Consts<T> C(P.s);
    const C2<T>* tw = as_global(static_cast<const C2<T>*>(P.tw));
    double rp, rd;
    const bool want_rd = rd_needed(ctrls + td.x);
    __syncthreads();
    constexpr bool kStream = batch_stream<T>();
    primal_res_pair<T, E, T, kStream>(C, u_in + P.u_off, u_out + P.u_off, phibar + P.f_off, phi + P.f_off,
                                      (T)P.tau_u, spec + P.f_off, P.lqb, tw, 2 * pair, tid, W, threadIdx.x, TB, buf,
                                      twl, edge, rp, rd, static_cast<C2<T>*>(nullptr), nullptr, want_rd);
    const double srp = subgroup_sum(rp, red, sg * nw, nw);
    const double srd = subgroup_sum(rd, red, sg * nw, nw);
    if (tid == 0 && pair < P.npairs) {
      part[P.part_off + pair] = srp;
      part[rd_base + P.part_off + pair] = srd;
    }
  }
}

// ------------------------------------------------------------------ C
template <typename T>
__global__ void __launch_bounds__(kColHalfThreads)
kb_colsolve(const BatchProb* __restrict__ probs, Ctrl* ctrls, const int2* __restrict__ tiles,
            const int* __restrict__ counts, T* __restrict__ spec, const double* __restrict__ part, int rd_base) {
  extern __shared__ char smem[];
  T* tile = reinterpret_cast<T*>(smem);
  __shared__ int s_status;
  const int n = counts[1];
  for (int t = blockIdx.x; t < n; t += gridDim.x) {
    const int2 td = tiles[t];
    // the stopping decision of another problem may land during this pass:
    // one thread reads the status and the block follows it
    if (threadIdx.x == 0) s_status = ctrls[td.x].status;
    __syncthreads();
    const int st = s_status;
    __syncthreads();
    if (st != 0) continue;
    const BatchProb& P = probs[td.x];
    if (td.y == 0 && threadIdx.x < 64)
      finalize_wave(ctrls + td.x, part + P.part_off, P.npairs, rd_base, P.wscale, nullptr);
    const FacTab<T> fac{as_global(static_cast<const FacRow<T>*>(P.fac_rows)), as_global(P.fac_off),
                        as_global(P.fac_last)};
    const int nt = P.s.nt, nx = P.s.nx;
    T* sp = spec + P.f_off;
    if (nt <= 256) {   // tiles of 16 columns, 16 lanes per column, LPL = ceil(nt / 16) <= 16
      const int q0 = td.y * 16, lq = (nt + 15) / 16;
      if (P.s.time == kTimeBDF2) {
        if (lq <= 1) colsolve_group_half<T, 2, 1, 16, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
        else if (lq <= 2) colsolve_group_half<T, 2, 2, 16, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
        else if (lq <= 4) colsolve_group_half<T, 2, 4, 16, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
        else if (lq <= 8) colsolve_group_half<T, 2, 8, 16, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
        else colsolve_group_half<T, 2, 16, 16, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
      } else {
        if (lq <= 1) colsolve_group_half<T, 1, 1, 16, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
        else if (lq <= 2) colsolve_group_half<T, 1, 2, 16, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
        else if (lq <= 4) colsolve_group_half<T, 1, 4, 16, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
        else if (lq <= 8) colsolve_group_half<T, 1, 8, 16, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
        else colsolve_group_half<T, 1, 16, 16, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
      }
      continue;
    }
    const int q0 = td.y * kColCols;
    // nt <= 512 (checked at set-up): 32 lanes per column, LPL = ceil(nt / 32) <= 16
    const int lpl = (nt + 31) / 32;
    if (P.s.time == kTimeBDF2) {
      if (lpl <= 1) colsolve_group_half<T, 2, 1>(sp, fac, nt, nx, P.lqb, q0, tile);
      else if (lpl <= 2) colsolve_group_half<T, 2, 2>(sp, fac, nt, nx, P.lqb, q0, tile);
      else if (lpl <= 4) colsolve_group_half<T, 2, 4>(sp, fac, nt, nx, P.lqb, q0, tile);
      else if (lpl <= 8) colsolve_group_half<T, 2, 8>(sp, fac, nt, nx, P.lqb, q0, tile);
      else colsolve_group_half<T, 2, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
    } else {
      if (lpl <= 1) colsolve_group_half<T, 1, 1>(sp, fac, nt, nx, P.lqb, q0, tile);
      else if (lpl <= 2) colsolve_group_half<T, 1, 2>(sp, fac, nt, nx, P.lqb, q0, tile);
      else if (lpl <= 4) colsolve_group_half<T, 1, 4>(sp, fac, nt, nx, P.lqb, q0, tile);
      else if (lpl <= 8) colsolve_group_half<T, 1, 8>(sp, fac, nt, nx, P.lqb, q0, tile);
      else colsolve_group_half<T, 1, 16>(sp, fac, nt, nx, P.lqb, q0, tile);
    }
  }
}

// ------------------------------------------------------------------ work lists
// One block of kCompactThreads threads.  Problems are visited in the order
// given by `order` (row tiles; the problems of 4 points per thread first) and
// `corder` (column tiles); converged problems contribute no tiles.  counts =
// {row tiles, column tiles, active problems, row tiles of 4 points per thread}.
constexpr int kCompactThreads = 1024;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int& total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int d = 1; d < kCompactThreads; d <<= 1) {
    const int x = tid >= d ? sh[tid - d] : 0;
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  total = sh[kCompactThreads - 1];
  const int incl = sh[tid];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kCompactThreads)
kb_compact(const BatchProb* __restrict__ probs, const Ctrl* __restrict__ ctrls, int nprob,
           const int* __restrict__ order, const int* __restrict__ corder, int2* __restrict__ row_tiles,
           int2* __restrict__ col_tiles, int* __restrict__ counts) {
  __shared__ int sh[kCompactThreads];
  int rbase = 0, cbase = 0, nact = 0, r4base = 0;
  for (int c0 = 0; c0 < nprob; c0 += kCompactThreads) {
    const int i = c0 + threadIdx.x;
    // row tiles
    int p = i < nprob ? order[i] : -1;
    bool act = p >= 0 && ctrls[p].status == 0;
    const int rn = act ? probs[p].rtiles : 0;
    int rtot;
    const int roff = rbase + block_exclusive_scan(rn, sh, rtot);
    const int S = act ? probs[p].pairs_per_tile : 1;
    for (int k = 0; k < rn; ++k) row_tiles[roff + k] = make_int2(p, k * S);
    rbase += rtot;
    int r4tot;
    block_exclusive_scan(act && batch_ept(probs[p].s.nx, kBatchRowThreads) == 4 ? rn : 0, sh, r4tot);
    r4base += r4tot;
    // column tiles
    p = i < nprob ? corder[i] : -1;
    act = p >= 0 && ctrls[p].status == 0;
    const int cn = act ? probs[p].ncolg : 0;
    int ctot;
    const int coff = cbase + block_exclusive_scan(cn, sh, ctot);
    for (int k = 0; k < cn; ++k) col_tiles[coff + k] = make_int2(p, k);
    cbase += ctot;
    int atot;
    block_exclusive_scan(act ? 1 : 0, sh, atot);
    nact += atot;
  }
  if (threadIdx.x == 0) {
    counts[0] = rbase;
    counts[1] = cbase;
    counts[2] = nact;
    counts[3] = r4base;
  }
}

// ------------------------------------------------------------------ set-up and finish
// max |f'(u0)| per problem (the same expression as the single-problem path).
template <typename T>
__global__ void __launch_bounds__(256)
kb_maxabs_dflux(const BatchProb* __restrict__ probs, const T* __restrict__ u0, double* __restrict__ out) {
  __shared__ double red[256];
  const BatchProb& P = probs[blockIdx.x];
  const double a2 = 2.0 * P.s.alpha, b = P.s.beta;
  double m = 0.0;
  for (int i = threadIdx.x; i < P.s.nx; i += 256) m = fmax(m, fabs(a2 * (double)u0[P.u0_off + i] + b));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Initial guess (Section 3.3) of every problem: u^l = u0 on all levels (only
// level 0 with warm start), u_alt = u, phi = 0 (kept with warm start), spectrum
// = 0, control block reset.  Grid (nprob, Y).
template <typename T>
__global__ void __launch_bounds__(256)
kb_init(const BatchProb* __restrict__ probs, const T* __restrict__ u0, T* __restrict__ u, T* __restrict__ u_alt,
        T* __restrict__ phi, T* __restrict__ spec, Ctrl* __restrict__ ctrls, int warm, long long max_iter,
        double eps, double div_factor) {
  const int p = blockIdx.x;
  const BatchProb& P = probs[p];
  const int nx = P.s.nx, nt = P.s.nt;
  const T* a = u0 + P.u0_off;
  T* up = u + P.u_off;
  T* ua = u_alt + P.u_off;
  const size_t nu = (size_t)(nt + 1) * nx, nf = (size_t)nt * nx;
  for (size_t i = (size_t)blockIdx.y * 256 + threadIdx.x; i < nu; i += (size_t)gridDim.y * 256) {
    T v;
    if (warm && i >= (size_t)nx) v = up[i];
    else v = a[i & (nx - 1)];
    up[i] = v;
    ua[i] = v;
    if (i < nf) {
      if (!warm) phi[P.f_off + i] = T(0);
      spec[P.f_off + i] = T(0);
    }
  }
  if (blockIdx.y == 0 && threadIdx.x == 0) {
    Ctrl* c = ctrls + p;
    c->n_done = 0;
    c->max_iter = max_iter;
    c->n_star = 0;
    c->status = 0;
    c->rd_lazy = 1;
    c->eps = eps;
    c->div_factor = div_factor;
    c->rp_prev = __builtin_nan("");
    c->best = __builtin_inf();
    c->rp_star = __builtin_nan("");
    c->rd_star = __builtin_nan("");
    c->best_at = 0;
    c->stall = 0;
    c->ck_iter = -1;
  }
}

// Last-good checkpoint of every problem still running (the single-problem
// k_checkpoint per problem slice): u_alt holds u^{N-1} and phi holds phi^{N-1}
// after a chunk ending with body N; a problem that has stopped keeps its
// previous checkpoint.  Grid: x strides over the slices, y = problem.
template <typename T>
__global__ void __launch_bounds__(256)
kb_checkpoint(const BatchProb* __restrict__ probs, Ctrl* ctrls, const T* __restrict__ u_alt,
              const T* __restrict__ phi, T* __restrict__ ck_u, T* __restrict__ ck_phi) {
  const int p = blockIdx.y;
  Ctrl* c = ctrls + p;
  if (c->status != 0) return;
  const BatchProb& P = probs[p];
  const size_t nx = (size_t)P.s.nx, nu = (size_t)(P.s.nt + 1) * nx, nf = (size_t)P.s.nt * nx;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nu; i += stride)
    ck_u[P.u_off + i] = u_alt[P.u_off + i];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += stride)
    ck_phi[P.f_off + i] = phi[P.f_off + i];
  if (blockIdx.x == 0 && threadIdx.x == 0) c->ck_iter = c->n_done > 0 ? c->n_done - 1 : 0;
}

// After the loop: the returned iterate n* of problem p sits in u_alt when n*
// is odd; copy it to u, and report max_l |m^l - m^0| h_x (discrete mass drift).
template <typename T>
__global__ void __launch_bounds__(256)
kb_finish(const BatchProb* __restrict__ probs, const Ctrl* __restrict__ ctrls, T* __restrict__ u,
          const T* __restrict__ u_alt, double* __restrict__ drift) {
  __shared__ double red[4];
  const int p = blockIdx.x;
  const BatchProb& P = probs[p];
  const int nx = P.s.nx, nt = P.s.nt;
  const bool odd = (ctrls[p].n_star & 1) != 0;
  const T* src = (odd ? u_alt : u) + P.u_off;
  T* dst = u + P.u_off;
  double m0 = 0.0, worst = 0.0;
  for (int l = 0; l <= nt; ++l) {
    double acc = 0.0;
    for (int j = threadIdx.x; j < nx; j += 256) {
      const T v = src[(size_t)l * nx + j];
      acc += (double)v;
      if (odd) dst[(size_t)l * nx + j] = v;
    }
    const double s = block_sum_waves(acc, red);
    if (threadIdx.x == 0) {
      if (l == 0) m0 = s;
      else worst = fmax(worst, fabs(s - m0) * P.s.hx);
    }
  }
  if (threadIdx.x == 0) drift[p] = worst;
}

// ------------------------------------------------------------------ launchers
template <typename T, int TB>
static size_t row_lds_bytes(int max_nx) {
  return sizeof(C2<T>) * batch_row_lds_points(max_nx, 256, TB) + sizeof(T) * 4 * (TB / 64);
}

// Threads per row block: 512 (EPT = 4 up to nx = 2048, 8 at nx = 4096).  In
// FP32 the primal pass runs the streaming body (a sliding window of rows in
// registers, at most 122 VGPRs), so that two of its persistent blocks share a
// CU and hide each other's loads; in FP64 the load-first body (register budget).
template <typename T>
constexpr int batch_row_threads() { return kBatchRowThreads; }


template <typename T>
int batch_row_block_threads() { return batch_row_threads<T>(); }

// Threads per row pair (W) for rows of length nx.
template <typename T>
int batch_row_width(int nx) { return nx / batch_ept(nx, batch_row_threads<T>()); }

template <typename T>
size_t batch_row_lds(int max_nx) { return row_lds_bytes<T, batch_row_threads<T>()>(max_nx); }

template <typename T>
size_t batch_col_lds() {   // the larger of the 8-column (32 lanes) and 16-column (16 lanes) tiles
  return sizeof(T) * std::max((size_t)kColCols * 16 * 33, (size_t)16 * 16 * 17);
}

template <typename T>
hipError_t batch_occupancy(int which, int max_nx, int* blocks_per_cu) {
  constexpr int TB = batch_row_threads<T>();
  hipError_t e;
  if (which == 0) {
    const size_t lds = batch_row_lds<T>(max_nx);
    if ((e = allow_lds(kb_dual_fft<T, TB>, lds)) != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kb_dual_fft<T, TB>, TB, lds);
  }
  if (which == 1) {
    const size_t lds = batch_row_lds<T>(max_nx);
    constexpr int E = batch_needs_e8<TB>() ? 8 : 4;   // the grid of the larger register budget
    if ((e = allow_lds(kb_primal_res<T, TB, E>, lds)) != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kb_primal_res<T, TB, E>, TB, lds);
  }
  const size_t lds = batch_col_lds<T>();
  if ((e = allow_lds(kb_colsolve<T>, lds)) != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kb_colsolve<T>, kColHalfThreads, lds);
}

template <typename T>
hipError_t launch_batch_dual_fft(const BatchLaunch& L, int grid, T* spec, T* phi, T* phibar, hipStream_t st) {
  constexpr int TB = batch_row_threads<T>();
  const size_t lds = batch_row_lds<T>(L.max_nx);
  hipError_t e = allow_lds(kb_dual_fft<T, TB>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((kb_dual_fft<T, TB>), dim3(grid), dim3(TB), lds, st, L.probs, L.ctrls, L.row_tiles, L.counts,
                     L.max_nx, spec, phi, phibar);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_primal_res(const BatchLaunch& L, int grid, const T* u_in, T* u_out, const T* phibar,
                                   const T* phi, T* spec, double* part, int rd_base, hipStream_t st) {
  constexpr int TB = batch_row_threads<T>();
  const size_t lds = batch_row_lds<T>(L.max_nx);
  hipError_t e = allow_lds(kb_primal_res<T, TB, 4>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((kb_primal_res<T, TB, 4>), dim3(grid), dim3(TB), lds, st, L.probs, L.ctrls, L.row_tiles,
                     L.counts, L.max_nx, u_in, u_out, phibar, phi, spec, part, rd_base);
  if constexpr (batch_needs_e8<TB>()) {   // the tiles of 8 points per thread, after those of 4
    if ((e = allow_lds(kb_primal_res<T, TB, 8>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((kb_primal_res<T, TB, 8>), dim3(grid), dim3(TB), lds, st, L.probs, L.ctrls, L.row_tiles,
                       L.counts, L.max_nx, u_in, u_out, phibar, phi, spec, part, rd_base);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_colsolve(const BatchLaunch& L, int grid, T* spec, const double* part, int rd_base,
                                 hipStream_t st) {
  const size_t lds = batch_col_lds<T>();
  hipError_t e = allow_lds(kb_colsolve<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kb_colsolve<T>, dim3(grid), dim3(kColHalfThreads), lds, st, L.probs, L.ctrls, L.col_tiles,
                     L.counts, spec, part, rd_base);
  return hipGetLastError();
}

hipError_t launch_batch_compact(const BatchLaunch& L, hipStream_t st) {
  hipLaunchKernelGGL(kb_compact, dim3(1), dim3(kCompactThreads), 0, st, L.probs, L.ctrls, L.nprob, L.order,
                     L.corder, L.row_tiles, L.col_tiles, L.counts);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_maxabs_dflux(const BatchLaunch& L, const T* u0, double* out, hipStream_t st) {
  hipLaunchKernelGGL(kb_maxabs_dflux<T>, dim3(L.nprob), dim3(256), 0, st, L.probs, u0, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_init(const BatchLaunch& L, const T* u0, T* u, T* u_alt, T* phi, T* spec, int warm,
                             long long max_iter, double eps, double div_factor, hipStream_t st) {
  hipLaunchKernelGGL(kb_init<T>, dim3(L.nprob, 32), dim3(256), 0, st, L.probs, u0, u, u_alt, phi, spec, L.ctrls,
                     warm, max_iter, eps, div_factor);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_checkpoint(const BatchLaunch& L, const T* u_alt, const T* phi, T* ck_u, T* ck_phi,
                                   hipStream_t st) {
  hipLaunchKernelGGL(kb_checkpoint<T>, dim3(64, L.nprob), dim3(256), 0, st, L.probs, L.ctrls, u_alt, phi, ck_u,
                     ck_phi);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_finish(const BatchLaunch& L, T* u, const T* u_alt, double* drift, hipStream_t st) {
  hipLaunchKernelGGL(kb_finish<T>, dim3(L.nprob), dim3(256), 0, st, L.probs, L.ctrls, u, u_alt, drift);
  return hipGetLastError();
}

#define PDHG_BATCH_INSTANTIATE(T)                                                                               \
  template int batch_row_block_threads<T>();                                                                   \
  template int batch_row_width<T>(int);                                                                        \
  template size_t batch_row_lds<T>(int);                                                                       \
  template size_t batch_col_lds<T>();                                                                          \
  template hipError_t batch_occupancy<T>(int, int, int*);                                                      \
  template hipError_t launch_batch_dual_fft<T>(const BatchLaunch&, int, T*, T*, T*, hipStream_t);              \
  template hipError_t launch_batch_primal_res<T>(const BatchLaunch&, int, const T*, T*, const T*, const T*, T*, \
                                                 double*, int, hipStream_t);                                   \
  template hipError_t launch_batch_colsolve<T>(const BatchLaunch&, int, T*, const double*, int, hipStream_t);  \
  template hipError_t launch_batch_maxabs_dflux<T>(const BatchLaunch&, const T*, double*, hipStream_t);       \
  template hipError_t launch_batch_init<T>(const BatchLaunch&, const T*, T*, T*, T*, T*, int, long long, double, \
                                           double, hipStream_t);                                               \
  template hipError_t launch_batch_finish<T>(const BatchLaunch&, T*, const T*, double*, hipStream_t);         \
  template hipError_t launch_batch_checkpoint<T>(const BatchLaunch&, const T*, const T*, T*, T*, hipStream_t);

PDHG_BATCH_INSTANTIATE(float)
PDHG_BATCH_INSTANTIATE(double)

}  // namespace pdhg
