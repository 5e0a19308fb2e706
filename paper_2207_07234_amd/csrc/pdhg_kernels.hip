// HIP kernels of the space-time primal-dual solver (gfx950).
//
// Unfused reference kernels (one pass per step of Algorithm 1, Section 3.3)
// and the building blocks of the preconditioner K_d^{-1} (Section 2.2):
// row FFTs in x and banded Cholesky solves in t per Fourier mode.
#include "pdhg_internal.hpp"

namespace pdhg {

constexpr int kFftThreads = 256;   // threads per row-FFT block (N <= 16 * 256)
constexpr int kEwThreads = 256;    // threads per element-wise block

// ------------------------------------------------------------------ row FFTs
// Forward: real rows [nrows][nx] (row stride nx) -> halfcomplex spectrum rows,
// two rows per block packed as z = a + i b.
template <typename T>
__global__ void __launch_bounds__(kFftThreads)
k_rows_fwd(const T* __restrict__ rows, int nrows, T* __restrict__ spec, int nt_spec, int lqb, int nx,
           const C2<T>* __restrict__ tw, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  extern __shared__ char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(nx);
  const int tid = threadIdx.x;
  const int a = 2 * blockIdx.x, b = a + 1;
  const bool hasb = b < nrows;
  const T* ra = rows + (size_t)a * nx;
  const T* rb = rows + (size_t)b * nx;
  load_twiddles_lds(twl, tw, nx, tid, kFftThreads);
  for (int x = tid; x < nx; x += kFftThreads) buf[lpad(x)] = {ra[x], hasb ? rb[x] : T(0)};
  fft_lds<false, 16>(buf, nx, twl, tid, kFftThreads);
  store_halfcomplex_pair(buf, nx, spec, nt_spec, lqb, a, hasb, tid, kFftThreads);
}

// Inverse: halfcomplex spectrum rows -> real rows (normalised by 1/nx).
template <typename T>
__global__ void __launch_bounds__(kFftThreads)
k_rows_inv(const T* __restrict__ spec, int nt_spec, int lqb, T* __restrict__ rows, int nrows, int nx,
           const C2<T>* __restrict__ tw, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  extern __shared__ char smem[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(nx);
  const int tid = threadIdx.x;
  const int a = 2 * blockIdx.x, b = a + 1;
  const bool hasb = b < nrows;
  load_twiddles_lds(twl, tw, nx, tid, kFftThreads);
  load_halfcomplex_pair(buf, nx, spec, nt_spec, lqb, a, hasb, tid, kFftThreads);
  fft_lds<true, 16>(buf, nx, twl, tid, kFftThreads);
  const T sc = T(1) / T(nx);
  T* ra = rows + (size_t)a * nx;
  T* rb = rows + (size_t)b * nx;
  for (int x = tid; x < nx; x += kFftThreads) {
    const C2<T> z = buf[lpad(x)];
    ra[x] = z.x * sc;
    if (hasb) rb[x] = z.y * sc;
  }
}

// ------------------------------------------------------------------ stencil kernels
// A(u): r^l_k for l = 0..nt-1 (u has nt+1 levels).  Optional partial sums of r^2.
template <typename T>
__global__ void __launch_bounds__(kEwThreads)
k_residual(Scheme s, const T* __restrict__ u, T* __restrict__ r, double* part, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  __shared__ double red[kEwThreads / 64];
  const Consts<T> C(s);
  const int nx = s.nx;
  const size_t idx = (size_t)blockIdx.x * kEwThreads + threadIdx.x;
  double acc = 0.0;
  if (idx < (size_t)s.nt * nx) {
    const int l = (int)(idx / nx), k = (int)(idx % nx);
    const int km = (k - 1) & (nx - 1), kp = (k + 1) & (nx - 1);
    const T* up1 = u + (size_t)(l + 1) * nx;
    const T* u0 = u + (size_t)l * nx;
    T t = C.c0(l) * up1[k] + C.c1(l) * u0[k];
    if (l >= 1 && C.time == kTimeBDF2) t += C.c2(l) * u[(size_t)(l - 1) * nx + k];
    const T v = t * C.inv_ht + C.F(up1[km], up1[k], up1[kp]);
    if (r) r[idx] = v;
    acc = (double)v * (double)v;
  }
  if (part) {
    const double sum = block_sum<kEwThreads>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

// Value of J(u)^T psi at unknown level m (1..nt), point k.
template <typename T>
__device__ __forceinline__ T jt_point(const Consts<T>& C, const T* __restrict__ u, const T* __restrict__ psi,
                                      int m, int k) {
  const int nx = C.nx, nt = C.nt;
  const int km = (k - 1) & (nx - 1), kp = (k + 1) & (nx - 1);
  const T* pm1 = psi + (size_t)(m - 1) * nx;
  const T p0 = (m <= nt - 1) ? psi[(size_t)m * nx + k] : T(0);
  const T pp1 = (m + 1 <= nt - 1) ? psi[(size_t)(m + 1) * nx + k] : T(0);
  return C.JtTime(m, pm1[k], p0, pp1) + C.JtF(u[(size_t)m * nx + k], pm1[km], pm1[k], pm1[kp]);
}

// out[m-1][k] = (J(u)^T psi)^m_k.  Optional partial sums of out^2.
template <typename T>
__global__ void __launch_bounds__(kEwThreads)
k_apply_jt(Scheme s, const T* __restrict__ u, const T* __restrict__ psi, T* __restrict__ out, double* part) {
  __shared__ double red[kEwThreads / 64];
  const Consts<T> C(s);
  const size_t idx = (size_t)blockIdx.x * kEwThreads + threadIdx.x;
  double acc = 0.0;
  if (idx < (size_t)s.nt * s.nx) {
    const int m = (int)(idx / s.nx) + 1, k = (int)(idx % s.nx);
    const T v = jt_point(C, u, psi, m, k);
    if (out) out[idx] = v;
    acc = (double)v * (double)v;
  }
  if (part) {
    const double sum = block_sum<kEwThreads>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

// out[l][k] = (J(u) v)^l_k, v indexed by unknown level (row m-1 = level m).
template <typename T>
__global__ void __launch_bounds__(kEwThreads)
k_apply_j(Scheme s, const T* __restrict__ u, const T* __restrict__ v, T* __restrict__ out) {
  const Consts<T> C(s);
  const int nx = s.nx;
  const size_t idx = (size_t)blockIdx.x * kEwThreads + threadIdx.x;
  if (idx >= (size_t)s.nt * nx) return;
  const int l = (int)(idx / nx), k = (int)(idx % nx);
  const int km = (k - 1) & (nx - 1), kp = (k + 1) & (nx - 1);
  const T* vl = v + (size_t)l * nx;         // level l+1
  const T* ul = u + (size_t)(l + 1) * nx;
  T t = C.c0(l) * vl[k];
  if (l >= 1) t += C.c1(l) * v[(size_t)(l - 1) * nx + k];
  if (l >= 2 && C.time == kTimeBDF2) t += C.c2(l) * v[(size_t)(l - 2) * nx + k];
  out[idx] = t * C.inv_ht + C.JF(ul[km], ul[k], ul[kp], vl[km], vl[k], vl[kp]);
}

// Unfused primal step: u_out^m = u_in^m - tau_u (J(u_in)^T phibar)^m for m = 1..nt,
// and partial sums of ((J(u_in)^T phi)^m)^2 for the dual residual of u_in.
template <typename T>
__global__ void __launch_bounds__(kEwThreads)
k_primal(Scheme s, const T* __restrict__ u_in, T* __restrict__ u_out, const T* __restrict__ phibar,
         const T* __restrict__ phi, T tau_u, double* part, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  __shared__ double red[kEwThreads / 64];
  const Consts<T> C(s);
  const size_t idx = (size_t)blockIdx.x * kEwThreads + threadIdx.x;
  const bool want_rd = !ctrl || rd_needed(ctrl);   // the dual residual only where it can decide
  double acc = 0.0;
  if (idx < (size_t)s.nt * s.nx) {
    const int m = (int)(idx / s.nx) + 1, k = (int)(idx % s.nx);
    const T gbar = jt_point(C, u_in, phibar, m, k);
    const T g = want_rd ? jt_point(C, u_in, phi, m, k) : T(0);
    const size_t o = (size_t)m * s.nx + k;
    u_out[o] = u_in[o] - tau_u * gbar;
    acc = (double)g * (double)g;
  }
  const double sum = block_sum<kEwThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

// Unfused dual step: phi <- phi + tau s ; phibar = phi + tau s.
template <typename T>
__global__ void __launch_bounds__(kEwThreads)
k_dual(T* __restrict__ phi, T* __restrict__ phibar, const T* __restrict__ srow, size_t n, T tau,
       const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  const size_t i = (size_t)blockIdx.x * kEwThreads + threadIdx.x;
  if (i >= n) return;
  const T ts = tau * srow[i];
  const T p = phi[i] + ts;
  phi[i] = p;
  phibar[i] = p + ts;
}

// ------------------------------------------------------------------ small utilities
template <typename T>
__global__ void k_fill(T* __restrict__ p, size_t n, T v) {
  const size_t i = (size_t)blockIdx.x * kEwThreads + threadIdx.x;
  if (i < n) p[i] = v;
}

// u^l = u0 for l = 0..nt (copy the initial data into every level).
template <typename T>
__global__ void k_broadcast_levels(T* __restrict__ u, const T* __restrict__ u0, int nx, int levels) {
  const size_t i = (size_t)blockIdx.x * kEwThreads + threadIdx.x;
  if (i < (size_t)nx * levels) u[i] = u0[i % nx];
}

template <typename T>
__global__ void k_copy(T* __restrict__ dst, const T* __restrict__ src, size_t n) {
  const size_t i = (size_t)blockIdx.x * kEwThreads + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Partial sums over a vector: mode 0: sum x^2; 1: sum x*y; 2: max |f'(x)| (as max, not sum).
template <typename T>
__global__ void __launch_bounds__(kEwThreads)
k_partial_dot(const T* __restrict__ x, const T* __restrict__ y, size_t n, double* part) {
  __shared__ double red[kEwThreads / 64];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * kEwThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kEwThreads)
    acc += (double)x[i] * (double)(y ? y[i] : x[i]);
  const double sum = block_sum<kEwThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

template <typename T>
__global__ void __launch_bounds__(kEwThreads)
k_partial_maxabs_dflux(const T* __restrict__ x, size_t n, double a2, double b, double* part) {
  __shared__ double red[kEwThreads];
  double m = 0.0;
  for (size_t i = (size_t)blockIdx.x * kEwThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kEwThreads)
    m = fmax(m, fabs(a2 * (double)x[i] + b));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = kEwThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Discrete mass of every level: out[l] = sum_j u^l_j (one block per level).
template <typename T>
__global__ void __launch_bounds__(kEwThreads) k_level_sums(const T* __restrict__ u, int nx, size_t stride,
                                                           double* out) {
  __shared__ double red[kEwThreads / 64];
  const T* row = u + (size_t)blockIdx.x * stride;
  double acc = 0.0;
  for (int j = threadIdx.x; j < nx; j += kEwThreads) acc += (double)row[j];
  const double s = block_sum<kEwThreads>(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// Sums of the first nx entries of `levels` rows spaced `stride` elements apart.
template <typename T>
hipError_t launch_level_sums(const T* u, int nx, size_t stride, int levels, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_level_sums<T>, dim3(levels), dim3(kEwThreads), 0, st, u, nx, stride, out);
  return hipGetLastError();
}
template hipError_t launch_level_sums<float>(const float*, int, size_t, int, double*, hipStream_t);
template hipError_t launch_level_sums<double>(const double*, int, size_t, int, double*, hipStream_t);

// Sum `n` partials in a fixed order into out[0] (single block).
__global__ void __launch_bounds__(kEwThreads) k_reduce_parts(const double* __restrict__ part, int n, double* out) {
  __shared__ double red[kEwThreads / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kEwThreads) acc += part[i];
  const double s = block_sum<kEwThreads>(acc, red);
  if (threadIdx.x == 0) out[0] = s;
}

// x <- x * scale (scale read from device: 1/sqrt(*nrm2))
template <typename T>
__global__ void k_normalize(T* __restrict__ x, size_t n, const double* nrm2) {
  const size_t i = (size_t)blockIdx.x * kEwThreads + threadIdx.x;
  if (i < n) x[i] = T((double)x[i] / sqrt(nrm2[0]));
}

// ------------------------------------------------------------------ control
__global__ void k_ctrl_init(Ctrl* c, long long max_iter, double eps, double div_factor, int rd_lazy,
                            long long stall) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->n_done = 0;
    c->max_iter = max_iter;
    c->n_star = 0;
    c->status = 0;
    c->rd_lazy = rd_lazy;
    c->eps = eps;
    c->div_factor = div_factor;
    c->rp_prev = __builtin_nan("");
    c->best = __builtin_inf();
    c->rp_star = __builtin_nan("");
    c->rd_star = __builtin_nan("");
    c->best_at = 0;
    c->stall = stall;
    c->ck_iter = -1;
  }
}

// Last-good checkpoint of a solve: while the solve is running, after a chunk of
// loop bodies ending with body N, u_alt holds u^{N-1} and phi holds phi^{N-1}
// (each body first takes the dual step of the previous iterate), an iterate
// that has passed the stopping and divergence tests.  Copied with its index; a
// solve that has stopped keeps its previous checkpoint.  Before the first body
// u_alt = u and phi are the start, iterate 0.
template <typename T>
__global__ void k_checkpoint(Ctrl* ctrl, const T* __restrict__ su, const T* __restrict__ sp, T* __restrict__ du,
                             T* __restrict__ dp, size_t nu, size_t np) {
  if (ctrl->status != 0) return;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nu; i += stride) du[i] = su[i];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) dp[i] = sp[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->ck_iter = ctrl->n_done > 0 ? ctrl->n_done - 1 : 0;
}

__global__ void __launch_bounds__(kEwThreads)
k_finalize(Ctrl* c, const double* __restrict__ part_rp, int n_rp, const double* __restrict__ part_rd, int n_rd,
           double wscale, double* hist) {
  if (c->status != 0) return;
  __shared__ double red[kEwThreads / 64];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n_rp; i += kEwThreads) a += part_rp[i];
  for (int i = threadIdx.x; i < n_rd; i += kEwThreads) b += part_rd[i];
  const double srp = block_sum<kEwThreads>(a, red);
  const double srd = block_sum<kEwThreads>(b, red);
  if (threadIdx.x == 0) finalize_body(c, srp, srd, wscale, hist);
}

// Refinement in time (Algorithm 2): u on ntc + 1 levels -> 2 ntc + 1 levels (fine
// level 2l = coarse level l, fine level 2l+1 = mean of coarse levels l, l+1);
// phi on ntc rows -> 2 ntc rows (both fine rows of a coarse interval take its
// value).  row = elements per level.
template <typename T>
__global__ void __launch_bounds__(kEwThreads)
k_refine_time(const T* __restrict__ uc, const T* __restrict__ pc, int ntc, size_t row, T* __restrict__ uf,
              T* __restrict__ pf) {
  const size_t i = (size_t)blockIdx.x * kEwThreads + threadIdx.x;
  if (i >= (size_t)(2 * ntc + 1) * row) return;
  const size_t lf = i / row, x = i % row;
  if ((lf & 1) == 0) {
    uf[i] = uc[(lf / 2) * row + x];
  } else {
    const size_t lc = lf / 2;
    uf[i] = T(0.5) * (uc[lc * row + x] + uc[(lc + 1) * row + x]);
  }
  if (lf < (size_t)(2 * ntc)) pf[i] = pc[(lf / 2) * row + x];
}

// ------------------------------------------------------------------ launchers
static inline unsigned grid_for(size_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// Dynamic LDS above 64 KiB needs an explicit opt-in per kernel.
template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <typename T>
hipError_t launch_rows_fwd(const T* rows, int nrows, T* spec, int nt_spec, int lqb, int nx, const void* tw,
                           const Ctrl* ctrl, hipStream_t st) {
  const size_t lds = sizeof(C2<T>) * 2 * (size_t)lds_fft_points(nx);
  hipError_t e = allow_lds(k_rows_fwd<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rows_fwd<T>, dim3((nrows + 1) / 2), dim3(kFftThreads), lds, st, rows, nrows, spec,
                     nt_spec, lqb, nx, (const C2<T>*)tw, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rows_inv(const T* spec, int nt_spec, int lqb, T* rows, int nrows, int nx, const void* tw,
                           const Ctrl* ctrl, hipStream_t st) {
  const size_t lds = sizeof(C2<T>) * 2 * (size_t)lds_fft_points(nx);
  hipError_t e = allow_lds(k_rows_inv<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rows_inv<T>, dim3((nrows + 1) / 2), dim3(kFftThreads), lds, st, spec, nt_spec, lqb,
                     rows, nrows, nx, (const C2<T>*)tw, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_residual(const Scheme& s, const T* u, T* r, double* part, const Ctrl* ctrl, hipStream_t st,
                           int* nblocks) {
  const unsigned g = grid_for((size_t)s.nt * s.nx, kEwThreads);
  if (nblocks) *nblocks = (int)g;
  hipLaunchKernelGGL(k_residual<T>, dim3(g), dim3(kEwThreads), 0, st, s, u, r, part, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_jt(const Scheme& s, const T* u, const T* psi, T* out, double* part, hipStream_t st,
                           int* nblocks) {
  const unsigned g = grid_for((size_t)s.nt * s.nx, kEwThreads);
  if (nblocks) *nblocks = (int)g;
  hipLaunchKernelGGL(k_apply_jt<T>, dim3(g), dim3(kEwThreads), 0, st, s, u, psi, out, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_j(const Scheme& s, const T* u, const T* v, T* out, hipStream_t st) {
  hipLaunchKernelGGL(k_apply_j<T>, dim3(grid_for((size_t)s.nt * s.nx, kEwThreads)), dim3(kEwThreads), 0, st, s,
                     u, v, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_primal(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                         double* part, const Ctrl* ctrl, hipStream_t st, int* nblocks) {
  const unsigned g = grid_for((size_t)s.nt * s.nx, kEwThreads);
  if (nblocks) *nblocks = (int)g;
  hipLaunchKernelGGL(k_primal<T>, dim3(g), dim3(kEwThreads), 0, st, s, u_in, u_out, phibar, phi, tau_u, part,
                     ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dual(T* phi, T* phibar, const T* srow, size_t n, T tau, const Ctrl* ctrl, hipStream_t st) {
  hipLaunchKernelGGL(k_dual<T>, dim3(grid_for(n, kEwThreads)), dim3(kEwThreads), 0, st, phi, phibar, srow, n,
                     tau, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* p, size_t n, T v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n, kEwThreads)), dim3(kEwThreads), 0, st, p, n, v);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_broadcast_levels(T* u, const T* u0, int nx, int levels, hipStream_t st) {
  hipLaunchKernelGGL(k_broadcast_levels<T>, dim3(grid_for((size_t)nx * levels, kEwThreads)), dim3(kEwThreads), 0,
                     st, u, u0, nx, levels);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(T* dst, const T* src, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy<T>, dim3(grid_for(n, kEwThreads)), dim3(kEwThreads), 0, st, dst, src, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_checkpoint(Ctrl* ctrl, const T* su, const T* sp, T* du, T* dp, size_t nu, size_t np,
                             hipStream_t st) {
  const unsigned g0 = grid_for(nu, kEwThreads), g = g0 < 2048u ? g0 : 2048u;
  hipLaunchKernelGGL(k_checkpoint<T>, dim3(g), dim3(kEwThreads), 0, st, ctrl, su, sp, du, dp, nu, np);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dot(const T* x, const T* y, size_t n, double* part, double* out, hipStream_t st) {
  const int g = 256;
  hipLaunchKernelGGL(k_partial_dot<T>, dim3(g), dim3(kEwThreads), 0, st, x, y, n, part);
  hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(kEwThreads), 0, st, part, g, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_maxabs_dflux(const T* x, size_t n, double a2, double b, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_partial_maxabs_dflux<T>, dim3(64), dim3(kEwThreads), 0, st, x, n, a2, b, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_normalize(T* x, size_t n, const double* nrm2, hipStream_t st) {
  hipLaunchKernelGGL(k_normalize<T>, dim3(grid_for(n, kEwThreads)), dim3(kEwThreads), 0, st, x, n, nrm2);
  return hipGetLastError();
}

hipError_t launch_ctrl_init(Ctrl* c, long long max_iter, double eps, double div_factor, hipStream_t st,
                            int rd_lazy, long long stall) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(64), 0, st, c, max_iter, eps, div_factor, rd_lazy, stall);
  return hipGetLastError();
}

hipError_t launch_finalize(Ctrl* c, const double* part_rp, int n_rp, const double* part_rd, int n_rd,
                           double wscale, double* hist, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kEwThreads), 0, st, c, part_rp, n_rp, part_rd, n_rd, wscale, hist);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_refine_time(const T* uc, const T* pc, int ntc, size_t row, T* uf, T* pf, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_time<T>, dim3(grid_for((size_t)(2 * ntc + 1) * row, kEwThreads)), dim3(kEwThreads), 0,
                     st, uc, pc, ntc, row, uf, pf);
  return hipGetLastError();
}
template hipError_t launch_refine_time<float>(const float*, const float*, int, size_t, float*, float*, hipStream_t);
template hipError_t launch_refine_time<double>(const double*, const double*, int, size_t, double*, double*,
                                               hipStream_t);

#define PDHG_INSTANTIATE(T)                                                                                    \
  template hipError_t launch_rows_fwd<T>(const T*, int, T*, int, int, int, const void*, const Ctrl*,          \
                                         hipStream_t);                                                        \
  template hipError_t launch_rows_inv<T>(const T*, int, int, T*, int, int, const void*, const Ctrl*,          \
                                         hipStream_t);                                                        \
  template hipError_t launch_residual<T>(const Scheme&, const T*, T*, double*, const Ctrl*, hipStream_t,      \
                                         int*);                                                               \
  template hipError_t launch_apply_jt<T>(const Scheme&, const T*, const T*, T*, double*, hipStream_t, int*);  \
  template hipError_t launch_apply_j<T>(const Scheme&, const T*, const T*, T*, hipStream_t);                  \
  template hipError_t launch_primal<T>(const Scheme&, const T*, T*, const T*, const T*, T, double*,           \
                                       const Ctrl*, hipStream_t, int*);                                       \
  template hipError_t launch_dual<T>(T*, T*, const T*, size_t, T, const Ctrl*, hipStream_t);                  \
  template hipError_t launch_fill<T>(T*, size_t, T, hipStream_t);                                             \
  template hipError_t launch_broadcast_levels<T>(T*, const T*, int, int, hipStream_t);                        \
  template hipError_t launch_copy<T>(T*, const T*, size_t, hipStream_t);                                      \
  template hipError_t launch_dot<T>(const T*, const T*, size_t, double*, double*, hipStream_t);               \
  template hipError_t launch_checkpoint<T>(Ctrl*, const T*, const T*, T*, T*, size_t, size_t, hipStream_t);  \
  template hipError_t launch_maxabs_dflux<T>(const T*, size_t, double, double, double*, hipStream_t);         \
  template hipError_t launch_normalize<T>(T*, size_t, const double*, hipStream_t);

PDHG_INSTANTIATE(float)
PDHG_INSTANTIATE(double)

}  // namespace pdhg
