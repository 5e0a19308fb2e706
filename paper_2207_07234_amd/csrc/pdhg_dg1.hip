// DG P1 nodal, upwind flux (the paper's DG example, Sections 3.2.2-3.2.3): the
// residual, the dual-equation operator J^T, J, and the step-size speed.
//
// Cell j stores u_h by its values v_j1, v_j2 at xi = -1/2 and +1/2 (basis
// phi_1 = 1/2 - xi, phi_2 = 1/2 + xi, xi = 2 (x - x_c) / h); planes
// u [nt+1][2][nx].  With the right trace a_j = -v_j1/2 + 3 v_j2/2, the upwind
// flux fhat_{j+1/2} = f(a_j), S_j = f(u_q0) + f(u_q1) the 2-point Gauss sum
// of f(u_h) (exact for quadratic f) and M = h [7 -1; -1 7] / 12,
//     F_j = -M^{-1} ( (-S_j, S_j) - f(a_j) (-1/2, 3/2) + f(a_{j-1}) (3/2, -1/2) ).
// With mu = M^{-1} psi and the Gauss values g1 = 1/2 + 1/sqrt(3), g2 = 1/2 - 1/sqrt(3)
// of the basis, the exact transpose of dF is
//     (dF^T psi)_j = -(mu_j2 - mu_j1) (sum_q f'(u_q) phi_m(x_q))_m
//                    + f'(a_j) (-1/2, 3/2) ((-mu_j1 + 3 mu_j2)/2 - (3 mu_{j+1,1} - mu_{j+1,2})/2)
// and dF v = -M^{-1} ( (-s, s) - f'(a_j) A_j (-1/2, 3/2) + f'(a_{j-1}) A_{j-1} (3/2, -1/2) ),
// s = sum_q f'(u_q) v_h(x_q), A = -v_1/2 + 3 v_2/2.  The time difference is that
// of the finite-difference scheme, per nodal plane.
#include "pdhg_internal.hpp"
#include "pdhg_passes.hpp"
#include "pdhg_dg1.hpp"

namespace pdhg {

constexpr int kDg1Threads = 256;

// r^l (2 planes) = time difference + F(u^{l+1}); optional partial sums of r^2.
template <typename T>
__global__ void __launch_bounds__(kDg1Threads)
k_dg1_residual(Scheme s, const T* __restrict__ u, T* __restrict__ r, double* part, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  __shared__ double red[kDg1Threads / 64];
  const Consts<T> C(s);
  const int nx = s.nx;
  const size_t idx = (size_t)blockIdx.x * kDg1Threads + threadIdx.x;
  double acc = 0.0;
  if (idx < (size_t)s.nt * nx) {
    const int l = (int)(idx / nx), j = (int)(idx % nx);
    const int jm = (j - 1) & (nx - 1);
    const size_t L2 = (size_t)2 * nx;
    const T* up1 = u + (size_t)(l + 1) * L2;
    T v[2], vm[2], F[2];
    load_cell2(up1, nx, j, v);
    load_cell2(up1, nx, jm, vm);
    dg1_spatial(C, v, P1Cell<T>::trace(vm), F);
    const T c0 = C.c0(l), c1 = C.c1(l), c2 = C.c2(l);
    const bool use2 = l >= 1 && C.time == kTimeBDF2;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      T t = c0 * v[k] + c1 * u[(size_t)l * L2 + (size_t)k * nx + j];
      if (use2) t += c2 * u[(size_t)(l - 1) * L2 + (size_t)k * nx + j];
      const T val = t * C.inv_ht + F[k];
      if (r) r[(size_t)l * L2 + (size_t)k * nx + j] = val;
      acc += (double)val * (double)val;
    }
  }
  if (part) {
    const double sum = block_sum<kDg1Threads>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

// (J(u)^T psi) at unknown level m (1..nt), cell j, both planes.
template <typename T>
__device__ __forceinline__ void dg1_jt_point(const Consts<T>& C, const T* __restrict__ u, const T* __restrict__ psi,
                                             int m, int j, T* out) {
  const int nx = C.nx, nt = C.nt;
  const int jp = (j + 1) & (nx - 1);
  const size_t L2 = (size_t)2 * nx;
  const T* pr = psi + (size_t)(m - 1) * L2;
  T v[2], p0[2], pp[2];
  load_cell2(u + (size_t)m * L2, nx, j, v);
  load_cell2(pr, nx, j, p0);
  load_cell2(pr, nx, jp, pp);
  dg1_jt_cell(C, v, p0, pp, out);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const T q0 = (m <= nt - 1) ? psi[(size_t)m * L2 + (size_t)k * nx + j] : T(0);
    const T q1 = (m + 1 <= nt - 1) ? psi[(size_t)(m + 1) * L2 + (size_t)k * nx + j] : T(0);
    out[k] += C.JtTime(m, p0[k], q0, q1);
  }
}

template <typename T>
__global__ void __launch_bounds__(kDg1Threads)
k_dg1_apply_jt(Scheme s, const T* __restrict__ u, const T* __restrict__ psi, T* __restrict__ out, double* part) {
  __shared__ double red[kDg1Threads / 64];
  const Consts<T> C(s);
  const int nx = s.nx;
  const size_t idx = (size_t)blockIdx.x * kDg1Threads + threadIdx.x;
  double acc = 0.0;
  if (idx < (size_t)s.nt * nx) {
    const int m = (int)(idx / nx) + 1, j = (int)(idx % nx);
    T g[2];
    dg1_jt_point(C, u, psi, m, j, g);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (out) out[(size_t)(m - 1) * 2 * nx + (size_t)k * nx + j] = g[k];
      acc += (double)g[k] * (double)g[k];
    }
  }
  if (part) {
    const double sum = block_sum<kDg1Threads>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

// Primal step u_out^m = u_in^m - tau (J(u_in)^T phibar)^m and partial sums of
// ((J(u_in)^T phi)^m)^2.
template <typename T>
__global__ void __launch_bounds__(kDg1Threads)
k_dg1_primal(Scheme s, const T* __restrict__ u_in, T* __restrict__ u_out, const T* __restrict__ phibar,
             const T* __restrict__ phi, T tau_u, double* part, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  __shared__ double red[kDg1Threads / 64];
  const Consts<T> C(s);
  const int nx = s.nx;
  const size_t idx = (size_t)blockIdx.x * kDg1Threads + threadIdx.x;
  const bool want_rd = !ctrl || rd_needed(ctrl);   // the dual residual only where it can decide
  double acc = 0.0;
  if (idx < (size_t)s.nt * nx) {
    const int m = (int)(idx / nx) + 1, j = (int)(idx % nx);
    T gb[2], g[2] = {T(0), T(0)};
    dg1_jt_point(C, u_in, phibar, m, j, gb);
    if (want_rd) dg1_jt_point(C, u_in, phi, m, j, g);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const size_t o = (size_t)m * 2 * nx + (size_t)k * nx + j;
      u_out[o] = u_in[o] - tau_u * gb[k];
      acc += (double)g[k] * (double)g[k];
    }
  }
  const double sum = block_sum<kDg1Threads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

// out[l] = (J(u) v)^l, v indexed by unknown level (row m-1 = level m).
template <typename T>
__global__ void __launch_bounds__(kDg1Threads)
k_dg1_apply_j(Scheme s, const T* __restrict__ u, const T* __restrict__ v, T* __restrict__ out) {
  const Consts<T> C(s);
  const int nx = s.nx;
  const size_t idx = (size_t)blockIdx.x * kDg1Threads + threadIdx.x;
  if (idx >= (size_t)s.nt * nx) return;
  const int l = (int)(idx / nx), j = (int)(idx % nx);
  const int jm = (j - 1) & (nx - 1);
  const size_t L2 = (size_t)2 * nx;
  const T* ul = u + (size_t)(l + 1) * L2;
  const T* vl = v + (size_t)l * L2;
  T uc[2], um[2], vm[2], v0[2], o[2];
  load_cell2(ul, nx, j, uc);
  load_cell2(ul, nx, jm, um);
  load_cell2(vl, nx, jm, vm);
  load_cell2(vl, nx, j, v0);
  dg1_j_cell(C, um, uc, vm, v0, o);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    T t = C.c0(l) * v0[k];
    if (l >= 1) t += C.c1(l) * v[(size_t)(l - 1) * L2 + (size_t)k * nx + j];
    if (l >= 2 && C.time == kTimeBDF2) t += C.c2(l) * v[(size_t)(l - 2) * L2 + (size_t)k * nx + j];
    out[(size_t)l * L2 + (size_t)k * nx + j] = t * C.inv_ht + o[k];
  }
}

// max of |f'| over the nodal values and both edge traces of u0 (per-block maxima).
template <typename T>
__global__ void __launch_bounds__(kDg1Threads)
k_dg1_maxabs(const T* __restrict__ u0, int nx, double a2, double b, double* part) {
  __shared__ double red[kDg1Threads];
  double m = 0.0;
  for (int j = blockIdx.x * kDg1Threads + threadIdx.x; j < nx; j += gridDim.x * kDg1Threads) {
    const double v0 = (double)u0[j], v1 = (double)u0[nx + j];
    const double ta = -0.5 * v0 + 1.5 * v1, tb = 1.5 * v0 - 0.5 * v1;
    m = fmax(m, fmax(fmax(fabs(a2 * v0 + b), fabs(a2 * v1 + b)), fmax(fabs(a2 * ta + b), fabs(a2 * tb + b))));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = kDg1Threads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------ launchers
static inline unsigned dg1_grid(size_t n) { return (unsigned)((n + kDg1Threads - 1) / kDg1Threads); }

template <typename T>
hipError_t launch_dg1_residual(const Scheme& s, const T* u, T* r, double* part, const Ctrl* ctrl, hipStream_t st,
                               int* nblocks) {
  const unsigned g = dg1_grid((size_t)s.nt * s.nx);
  if (nblocks) *nblocks = (int)g;
  hipLaunchKernelGGL(k_dg1_residual<T>, dim3(g), dim3(kDg1Threads), 0, st, s, u, r, part, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dg1_apply_jt(const Scheme& s, const T* u, const T* psi, T* out, double* part, hipStream_t st,
                               int* nblocks) {
  const unsigned g = dg1_grid((size_t)s.nt * s.nx);
  if (nblocks) *nblocks = (int)g;
  hipLaunchKernelGGL(k_dg1_apply_jt<T>, dim3(g), dim3(kDg1Threads), 0, st, s, u, psi, out, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dg1_apply_j(const Scheme& s, const T* u, const T* v, T* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dg1_apply_j<T>, dim3(dg1_grid((size_t)s.nt * s.nx)), dim3(kDg1Threads), 0, st, s, u, v, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dg1_primal(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                             double* part, const Ctrl* ctrl, hipStream_t st, int* nblocks) {
  const unsigned g = dg1_grid((size_t)s.nt * s.nx);
  if (nblocks) *nblocks = (int)g;
  hipLaunchKernelGGL(k_dg1_primal<T>, dim3(g), dim3(kDg1Threads), 0, st, s, u_in, u_out, phibar, phi, tau_u, part,
                     ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dg1_maxabs(const T* u0, int nx, double a2, double b, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_dg1_maxabs<T>, dim3(64), dim3(kDg1Threads), 0, st, u0, nx, a2, b, part);
  return hipGetLastError();
}

#define PDHG_DG1_INSTANTIATE(T)                                                                                    \
  template hipError_t launch_dg1_residual<T>(const Scheme&, const T*, T*, double*, const Ctrl*, hipStream_t, int*); \
  template hipError_t launch_dg1_apply_jt<T>(const Scheme&, const T*, const T*, T*, double*, hipStream_t, int*);    \
  template hipError_t launch_dg1_apply_j<T>(const Scheme&, const T*, const T*, T*, hipStream_t);                   \
  template hipError_t launch_dg1_primal<T>(const Scheme&, const T*, T*, const T*, const T*, T, double*,           \
                                           const Ctrl*, hipStream_t, int*);                                       \
  template hipError_t launch_dg1_maxabs<T>(const T*, int, double, double, double*, hipStream_t);

PDHG_DG1_INSTANTIATE(float)
PDHG_DG1_INSTANTIATE(double)

}  // namespace pdhg
