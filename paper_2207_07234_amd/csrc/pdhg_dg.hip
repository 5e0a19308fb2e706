// DG P2 (Legendre, local Lax-Friedrichs flux) in space: the residual, the
// dual-equation operator J^T, J, and the preconditioner's column solve.
//
// Cell j carries three Legendre coefficients v_j0, v_j1, v_j2 (coefficient
// planes: u [nt+1][3][nx], phi [nt][3][nx]).  With s_k = -(2k+1)/h_x, traces
// a_j = v_j0 + v_j1 + v_j2 (right edge), b_j = v_j0 - v_j1 + v_j2 (left edge),
// the LLF flux fhat(a, b) = (f(a) + f(b))/2 - max(|f'(a)|, |f'(b)|) (b - a)/2
// at x_{j+1/2} between a_j and b_{j+1}, and the volume term
// V_jk = int_{-1}^{1} f(u_h) P_k' dxi by 3-point Gauss (exact for quadratic f):
//     F_jk = s_k (V_jk - fhat_{j+1/2} + (-1)^k fhat_{j-1/2}).
// The time difference is that of the finite-difference scheme, per coefficient.
//
// Exact transpose of the Jacobian (generalised derivative of the max, a's
// branch on ties), with Psi+_j = sum_k s_k psi_jk, Psi-_j = sum_k s_k (-1)^k psi_jk:
//     (dF^T psi)_jm = sum_q w_q f'(u_q) P_m(xi_q) (s_1 psi_j1 + 3 xi_q s_2 psi_j2)
//                     + da_{j+1/2} (Psi-_{j+1} - Psi+_j) + (-1)^m db_{j-1/2} (Psi-_j - Psi+_{j-1})
// and of the Jacobian itself, with A_j = sum_m v_jm, B_j = sum_m (-1)^m v_jm:
//     (dF v)_jk = s_k ( sum_q w_q f'(u_q) P_k'(xi_q) v_h(xi_q)
//                       - da_{j+1/2} A_j - db_{j+1/2} B_{j+1} + (-1)^k (da_{j-1/2} A_{j-1} + db_{j-1/2} B_j) ).
//
// Preconditioner column solve: per Fourier mode over the cells, the three
// coefficient planes couple through c^2 G(theta) G(theta)^* (G the unit-speed
// upwind DG symbol).  Its real 6x6 form acts on (Re, Im) of the three planes;
// the host diagonalises it (V Lambda V^T) and the kernel rotates each level's
// 6-vector by V^T, runs one banded Cholesky solve along t per eigenvalue, and
// rotates back by V.
#include "pdhg_internal.hpp"
#include "pdhg_passes.hpp"
#include "pdhg_dg1.hpp"

namespace pdhg {

constexpr int kDgThreads = 256;

template <typename T>
struct DgCell {
  // Gauss nodes xi = -sqrt(3/5), 0, +sqrt(3/5); weights 5/9, 8/9, 5/9
  static __device__ __forceinline__ T xq(int q) { return q == 1 ? T(0) : (q == 0 ? T(-0.7745966692414833770358531) : T(0.7745966692414833770358531)); }
  static __device__ __forceinline__ T wq(int q) { return q == 1 ? T(8.0 / 9.0) : T(5.0 / 9.0); }
  static __device__ __forceinline__ T p2q(int q) { return q == 1 ? T(-0.5) : T(0.4); }   // P_2 at the nodes
};

template <typename T>
__device__ __forceinline__ T llf(const Consts<T>& C, T a, T b) {
  const T s = fmax(fabs(C.dflux(a)), fabs(C.dflux(b)));
  return T(0.5) * (C.flux(a) + C.flux(b)) - T(0.5) * s * (b - a);
}

template <typename T>
__device__ __forceinline__ void llf_partials(const Consts<T>& C, T a, T b, T& da, T& db) {
  const T fa = C.dflux(a), fb = C.dflux(b);
  const bool a_branch = fabs(fa) >= fabs(fb);
  const T s = a_branch ? fabs(fa) : fabs(fb);
  const T sgn_a = fa > T(0) ? T(1) : (fa < T(0) ? T(-1) : T(0));
  const T sgn_b = fb > T(0) ? T(1) : (fb < T(0) ? T(-1) : T(0));
  const T sa = a_branch ? sgn_a * C.alpha2 : T(0);
  const T sb = a_branch ? T(0) : sgn_b * C.alpha2;
  da = T(0.5) * fa + T(0.5) * s - T(0.5) * (b - a) * sa;
  db = T(0.5) * fb - T(0.5) * s - T(0.5) * (b - a) * sb;
}

template <typename T>
__device__ __forceinline__ void load_cell(const T* __restrict__ row3, int nx, int j, T* v) {
  v[0] = row3[j];
  v[1] = row3[nx + j];
  v[2] = row3[2 * nx + j];
}

// F_j (3 values) from the cell's coefficients and the neighbours' traces.
template <typename T>
__device__ __forceinline__ void dg_spatial(const Consts<T>& C, const T* v, T a_left, T b_right, T* F) {
  const T a = v[0] + v[1] + v[2], b = v[0] - v[1] + v[2];
  const T fr = llf(C, a, b_right), fl = llf(C, a_left, b);
  T V1 = T(0), V2 = T(0);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const T x = DgCell<T>::xq(q);
    const T fu = C.flux(v[0] + v[1] * x + v[2] * DgCell<T>::p2q(q));
    V1 += DgCell<T>::wq(q) * fu;
    V2 += DgCell<T>::wq(q) * fu * (T(3) * x);
  }
  const T h1 = C.inv_hx;
  F[0] = -h1 * (T(0) - fr + fl);
  F[1] = -T(3) * h1 * (V1 - fr - fl);
  F[2] = -T(5) * h1 * (V2 - fr + fl);
}

// (dF^T psi)_j for the cell with coefficients v (u at this level), neighbours'
// traces, and psi at cells j-1, j, j+1.
template <typename T>
__device__ __forceinline__ void dg_jt_cell(const Consts<T>& C, const T* v, T a_left, T b_right, const T* pm,
                                           const T* p0, const T* pp, T* out) {
  const T h1 = C.inv_hx;
  const T s0 = -h1, s1 = -T(3) * h1, s2 = -T(5) * h1;
  const T a = v[0] + v[1] + v[2], b = v[0] - v[1] + v[2];
  T da_r, db_r, da_l, db_l;
  llf_partials(C, a, b_right, da_r, db_r);   // interface j+1/2
  llf_partials(C, a_left, b, da_l, db_l);    // interface j-1/2
  const T Pp_m = s0 * pm[0] + s1 * pm[1] + s2 * pm[2];            // Psi+_{j-1}
  const T Pp_0 = s0 * p0[0] + s1 * p0[1] + s2 * p0[2];            // Psi+_j
  const T Pm_0 = s0 * p0[0] - s1 * p0[1] + s2 * p0[2];            // Psi-_j
  const T Pm_p = s0 * pp[0] - s1 * pp[1] + s2 * pp[2];            // Psi-_{j+1}
  T o0 = T(0), o1 = T(0), o2 = T(0);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const T x = DgCell<T>::xq(q), p2 = DgCell<T>::p2q(q);
    const T g = DgCell<T>::wq(q) * C.dflux(v[0] + v[1] * x + v[2] * p2) * (s1 * p0[1] + T(3) * x * s2 * p0[2]);
    o0 += g;
    o1 += g * x;
    o2 += g * p2;
  }
  const T tr = da_r * (Pm_p - Pp_0), tl = db_l * (Pm_0 - Pp_m);
  out[0] = o0 + tr + tl;
  out[1] = o1 + tr - tl;
  out[2] = o2 + tr + tl;
}

// (dF v)_j for the cell (u coefficients uc, neighbours' u traces) and v at cells j-1, j, j+1.
template <typename T>
__device__ __forceinline__ void dg_j_cell(const Consts<T>& C, const T* uc, T ua_left, T ub_right, const T* vm,
                                          const T* v0, const T* vp, T* out) {
  const T h1 = C.inv_hx;
  const T a = uc[0] + uc[1] + uc[2], b = uc[0] - uc[1] + uc[2];
  T da_r, db_r, da_l, db_l;
  llf_partials(C, a, ub_right, da_r, db_r);
  llf_partials(C, ua_left, b, da_l, db_l);
  const T A0 = v0[0] + v0[1] + v0[2], B0 = v0[0] - v0[1] + v0[2];
  const T Am = vm[0] + vm[1] + vm[2], Bp = vp[0] - vp[1] + vp[2];
  T I1 = T(0), I2 = T(0);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const T x = DgCell<T>::xq(q), p2 = DgCell<T>::p2q(q);
    const T g = DgCell<T>::wq(q) * C.dflux(uc[0] + uc[1] * x + uc[2] * p2) * (v0[0] + v0[1] * x + v0[2] * p2);
    I1 += g;
    I2 += g * (T(3) * x);
  }
  const T R = da_r * A0 + db_r * Bp, L = da_l * Am + db_l * B0;
  out[0] = -h1 * (T(0) - R + L);
  out[1] = -T(3) * h1 * (I1 - R - L);
  out[2] = -T(5) * h1 * (I2 - R + L);
}

// ------------------------------------------------------------------ kernels
// r^l (3 planes) = time difference + F(u^{l+1}); optional partial sums of r^2.
template <typename T>
__global__ void __launch_bounds__(kDgThreads)
k_dg_residual(Scheme s, const T* __restrict__ u, T* __restrict__ r, double* part, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  __shared__ double red[kDgThreads / 64];
  const Consts<T> C(s);
  const int nx = s.nx;
  const size_t idx = (size_t)blockIdx.x * kDgThreads + threadIdx.x;
  double acc = 0.0;
  if (idx < (size_t)s.nt * nx) {
    const int l = (int)(idx / nx), j = (int)(idx % nx);
    const int jm = (j - 1) & (nx - 1), jp = (j + 1) & (nx - 1);
    const size_t L3 = (size_t)3 * nx;
    const T* up1 = u + (size_t)(l + 1) * L3;
    T v[3], vm[3], vp[3], F[3];
    load_cell(up1, nx, j, v);
    load_cell(up1, nx, jm, vm);
    load_cell(up1, nx, jp, vp);
    dg_spatial(C, v, vm[0] + vm[1] + vm[2], vp[0] - vp[1] + vp[2], F);
    const T c0 = C.c0(l), c1 = C.c1(l), c2 = C.c2(l);
    const bool use2 = l >= 1 && C.time == kTimeBDF2;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T t = c0 * v[k] + c1 * u[(size_t)l * L3 + (size_t)k * nx + j];
      if (use2) t += c2 * u[(size_t)(l - 1) * L3 + (size_t)k * nx + j];
      const T val = t * C.inv_ht + F[k];
      if (r) r[(size_t)l * L3 + (size_t)k * nx + j] = val;
      acc += (double)val * (double)val;
    }
  }
  if (part) {
    const double sum = block_sum<kDgThreads>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

// The same residual with the per-cell products on the matrix cores (FP32,
// v_mfma_f32_16x16x4f32; a measured alternative, loop-body variant 6).  A
// wavefront takes 64 cells of one level, as four groups of 16.  Per group two
// 16x16x4 products:
//   (1) E v: rows q = 0..2 evaluate u_h at the Gauss nodes (P_m(xi_q)), row 3
//       the right trace (1, 1, 1), row 4 the left trace (1, -1, 1); K = the
//       three coefficients (fourth zero); N = the 16 cells of the group;
//   (2) W f(u_q): rows k = 1, 2 hold w_q P_k'(xi_q) (P_1' = 1, P_2' = 3 xi);
//       K = the three nodes; the volume terms V_1, V_2 of the 16 cells.
// Operand layouts of the 16x16x4 f32 product: lane i + 16 k supplies A[i][k],
// lane j + 16 k supplies B[k][j]; lane j + 16 g receives D[4 g + r][j] in its
// r-th result.  The products' results are then moved (lane permutes) so that
// lane L works on cell j0 + L: LLF fluxes, time difference, norm, one cell
// per lane as in the VALU kernel.
typedef float pdhg_fx4 __attribute__((ext_vector_type(4)));
constexpr int kDgMfmaThreads = 256;

__global__ void __launch_bounds__(kDgMfmaThreads)
k_dg_residual_mfma(Scheme s, const float* __restrict__ u, float* __restrict__ r, double* part, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  __shared__ double red[kDgMfmaThreads / 64];
  const Consts<float> C(s);
  const int nx = s.nx, nt = s.nt;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, kk = lane >> 4;
  const size_t first = ((size_t)blockIdx.x * (kDgMfmaThreads / 64) + wv) * 64;   // flattened l nx + j
  double acc = 0.0;
  if (first < (size_t)nt * nx) {   // uniform per wavefront: 64 | nx
    const int l = (int)(first / nx), j0 = (int)(first % nx);
    const size_t L3 = (size_t)3 * nx;
    const float* up1 = u + (size_t)(l + 1) * L3;
    float ea = 0.f, wa = 0.f;
    if (kk < 3) {
      if (col < 3) ea = kk == 0 ? 1.f : (kk == 1 ? DgCell<float>::xq(col) : DgCell<float>::p2q(col));
      else if (col == 3) ea = 1.f;
      else if (col == 4) ea = (kk & 1) ? -1.f : 1.f;
      if (col == 1 || col == 2) wa = DgCell<float>::wq(kk) * (col == 1 ? 1.f : 3.f * DgCell<float>::xq(kk));
    }
    const pdhg_fx4 zero = {0.f, 0.f, 0.f, 0.f};
    // per group g: right trace a, left trace b, V_1, V_2 of cell j0 + 16 g + col, held by lane col
    float ag[4], bg[4], v1g[4], v2g[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float bv = kk < 3 ? up1[(size_t)kk * nx + j0 + 16 * g + col] : 0.f;
      const pdhg_fx4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(ea, bv, zero, 0, 0, 0);
      const float f0 = C.flux(d[0]), f1 = C.flux(d[1]), f2 = C.flux(d[2]);
      const float g0 = __shfl(f0, col), g1 = __shfl(f1, col), g2 = __shfl(f2, col);
      const float bf = kk == 0 ? g0 : (kk == 1 ? g1 : (kk == 2 ? g2 : 0.f));
      const pdhg_fx4 V = __builtin_amdgcn_mfma_f32_16x16x4f32(wa, bf, zero, 0, 0, 0);
      ag[g] = d[3];
      bg[g] = __shfl(d[0], col + 16);   // row 4 of the first product
      v1g[g] = V[1];
      v2g[g] = V[2];
    }
    // lane L = 16 kk + col takes cell j0 + L: its values sit in group kk of lane col
    float aj = 0.f, bj = 0.f, V1 = 0.f, V2 = 0.f;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float ta = __shfl(ag[g], col), tb = __shfl(bg[g], col);
      const float t1 = __shfl(v1g[g], col), t2 = __shfl(v2g[g], col);
      if (kk == g) {
        aj = ta;
        bj = tb;
        V1 = t1;
        V2 = t2;
      }
    }
    const int j = j0 + lane;
    float am = __shfl(aj, (lane + 63) & 63);   // right trace of cell j - 1
    float bp = __shfl(bj, (lane + 1) & 63);    // left trace of cell j + 1
    if (lane == 0) {
      float vm[3];
      load_cell(up1, nx, (j - 1) & (nx - 1), vm);
      am = vm[0] + vm[1] + vm[2];
    }
    if (lane == 63) {
      float vp[3];
      load_cell(up1, nx, (j + 1) & (nx - 1), vp);
      bp = vp[0] - vp[1] + vp[2];
    }
    const float fr = llf(C, aj, bp), fl = llf(C, am, bj);
    const float h1 = C.inv_hx;
    float F[3];
    F[0] = -h1 * (0.f - fr + fl);
    F[1] = -3.f * h1 * (V1 - fr - fl);
    F[2] = -5.f * h1 * (V2 - fr + fl);
    const float c0 = C.c0(l), c1 = C.c1(l), c2 = C.c2(l);
    const bool use2 = l >= 1 && C.time == kTimeBDF2;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float t = c0 * up1[(size_t)k * nx + j] + c1 * u[(size_t)l * L3 + (size_t)k * nx + j];
      if (use2) t += c2 * u[(size_t)(l - 1) * L3 + (size_t)k * nx + j];
      const float val = t * C.inv_ht + F[k];
      if (r) r[(size_t)l * L3 + (size_t)k * nx + j] = val;
      acc += (double)val * (double)val;
    }
  }
  if (part) {
    const double sum = block_sum<kDgMfmaThreads>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

hipError_t launch_dg_residual_mfma(const Scheme& s, const float* u, float* r, double* part, const Ctrl* ctrl,
                                   hipStream_t st, int* nblocks) {
  if (s.nx < 64 || s.space != kSpaceDgP2) return hipErrorInvalidValue;
  const size_t waves = (size_t)s.nt * s.nx / 64;
  const unsigned g = (unsigned)((waves + kDgMfmaThreads / 64 - 1) / (kDgMfmaThreads / 64));
  if (nblocks) *nblocks = (int)g;
  hipLaunchKernelGGL(k_dg_residual_mfma, dim3(g), dim3(kDgMfmaThreads), 0, st, s, u, r, part, ctrl);
  return hipGetLastError();
}

// (J(u)^T psi) at unknown level m (1..nt), cell j, all three coefficients.
template <typename T>
__device__ __forceinline__ void dg_jt_point(const Consts<T>& C, const T* __restrict__ u, const T* __restrict__ psi,
                                            int m, int j, T* out) {
  const int nx = C.nx, nt = C.nt;
  const int jm = (j - 1) & (nx - 1), jp = (j + 1) & (nx - 1);
  const size_t L3 = (size_t)3 * nx;
  const T* um = u + (size_t)m * L3;
  const T* pr = psi + (size_t)(m - 1) * L3;
  T v[3], vm[3], vp[3], pm[3], p0[3], pp[3];
  load_cell(um, nx, j, v);
  load_cell(um, nx, jm, vm);
  load_cell(um, nx, jp, vp);
  load_cell(pr, nx, jm, pm);
  load_cell(pr, nx, j, p0);
  load_cell(pr, nx, jp, pp);
  dg_jt_cell(C, v, vm[0] + vm[1] + vm[2], vp[0] - vp[1] + vp[2], pm, p0, pp, out);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T q0 = (m <= nt - 1) ? psi[(size_t)m * L3 + (size_t)k * nx + j] : T(0);
    const T q1 = (m + 1 <= nt - 1) ? psi[(size_t)(m + 1) * L3 + (size_t)k * nx + j] : T(0);
    out[k] += C.JtTime(m, p0[k], q0, q1);
  }
}

template <typename T>
__global__ void __launch_bounds__(kDgThreads)
k_dg_apply_jt(Scheme s, const T* __restrict__ u, const T* __restrict__ psi, T* __restrict__ out, double* part) {
  __shared__ double red[kDgThreads / 64];
  const Consts<T> C(s);
  const int nx = s.nx;
  const size_t idx = (size_t)blockIdx.x * kDgThreads + threadIdx.x;
  double acc = 0.0;
  if (idx < (size_t)s.nt * nx) {
    const int m = (int)(idx / nx) + 1, j = (int)(idx % nx);
    T g[3];
    dg_jt_point(C, u, psi, m, j, g);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (out) out[(size_t)(m - 1) * 3 * nx + (size_t)k * nx + j] = g[k];
      acc += (double)g[k] * (double)g[k];
    }
  }
  if (part) {
    const double sum = block_sum<kDgThreads>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
  }
}

// Primal step u_out^m = u_in^m - tau (J(u_in)^T phibar)^m, m = 1..nt, and partial
// sums of ((J(u_in)^T phi)^m)^2 (dual residual of the incoming iterate).
template <typename T>
__global__ void __launch_bounds__(kDgThreads)
k_dg_primal(Scheme s, const T* __restrict__ u_in, T* __restrict__ u_out, const T* __restrict__ phibar,
            const T* __restrict__ phi, T tau_u, double* part, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  __shared__ double red[kDgThreads / 64];
  const Consts<T> C(s);
  const int nx = s.nx;
  const size_t idx = (size_t)blockIdx.x * kDgThreads + threadIdx.x;
  const bool want_rd = !ctrl || rd_needed(ctrl);   // the dual residual only where it can decide
  double acc = 0.0;
  if (idx < (size_t)s.nt * nx) {
    const int m = (int)(idx / nx) + 1, j = (int)(idx % nx);
    T gb[3], g[3] = {T(0), T(0), T(0)};
    dg_jt_point(C, u_in, phibar, m, j, gb);
    if (want_rd) dg_jt_point(C, u_in, phi, m, j, g);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const size_t o = (size_t)m * 3 * nx + (size_t)k * nx + j;
      u_out[o] = u_in[o] - tau_u * gb[k];
      acc += (double)g[k] * (double)g[k];
    }
  }
  const double sum = block_sum<kDgThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

// out[l] = (J(u) v)^l, v indexed by unknown level (row m-1 = level m).
template <typename T>
__global__ void __launch_bounds__(kDgThreads)
k_dg_apply_j(Scheme s, const T* __restrict__ u, const T* __restrict__ v, T* __restrict__ out) {
  const Consts<T> C(s);
  const int nx = s.nx;
  const size_t idx = (size_t)blockIdx.x * kDgThreads + threadIdx.x;
  if (idx >= (size_t)s.nt * nx) return;
  const int l = (int)(idx / nx), j = (int)(idx % nx);
  const int jm = (j - 1) & (nx - 1), jp = (j + 1) & (nx - 1);
  const size_t L3 = (size_t)3 * nx;
  const T* ul = u + (size_t)(l + 1) * L3;
  const T* vl = v + (size_t)l * L3;
  T uc[3], um[3], upp[3], vm[3], v0[3], vp[3], o[3];
  load_cell(ul, nx, j, uc);
  load_cell(ul, nx, jm, um);
  load_cell(ul, nx, jp, upp);
  load_cell(vl, nx, jm, vm);
  load_cell(vl, nx, j, v0);
  load_cell(vl, nx, jp, vp);
  dg_j_cell(C, uc, um[0] + um[1] + um[2], upp[0] - upp[1] + upp[2], vm, v0, vp, o);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T t = C.c0(l) * v0[k];
    if (l >= 1) t += C.c1(l) * v[(size_t)(l - 1) * L3 + (size_t)k * nx + j];
    if (l >= 2 && C.time == kTimeBDF2) t += C.c2(l) * v[(size_t)(l - 2) * L3 + (size_t)k * nx + j];
    out[(size_t)l * L3 + (size_t)k * nx + j] = t * C.inv_ht + o[k];
  }
}

// max over cells of |f'| at both edge traces of u0_h (per-block maxima).
template <typename T>
__global__ void __launch_bounds__(kDgThreads)
k_dg_maxabs_trace(const T* __restrict__ u0, int nx, double a2, double b, double* part) {
  __shared__ double red[kDgThreads];
  double m = 0.0;
  for (int j = blockIdx.x * kDgThreads + threadIdx.x; j < nx; j += gridDim.x * kDgThreads) {
    const double v0 = (double)u0[j], v1 = (double)u0[nx + j], v2 = (double)u0[2 * nx + j];
    m = fmax(m, fmax(fabs(a2 * (v0 + v1 + v2) + b), fabs(a2 * (v0 - v1 + v2) + b)));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = kDgThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// The three FFTs of k_dg_residual_fft alternate between two LDS arrays (one
// barrier per stage instead of two) where a third N-point array fits in 96 KiB:
// up to nx = 4096 in FP32 and 2048 in FP64.  Kernel and launcher decide alike.
template <typename T>
__host__ __device__ constexpr bool dg_fft_pingpong(int nx) { return 3 * (size_t)nx * sizeof(C2<T>) <= 98304; }

// Residual of levels l = 2w and 2w + 1 (3 planes each) and the forward FFT of
// those 6 coefficient rows of the 3 nt-row spectrum, as the three complex
// FFTs of row pairs (6w, 6w+1), (6w+2, 6w+3), (6w+4, 6w+5).  W = nx / E
// threads; thread owns cells j = tid + e W.  Per-block partial sums of r^2.
template <typename T, int E>
__global__ void __launch_bounds__(512)
k_dg_residual_fft(Scheme s, const T* __restrict__ u, T* __restrict__ spec, int lqb, const C2<T>* __restrict__ tw,
                  double* __restrict__ part, const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  extern __shared__ char smem[];
  __shared__ double red[512 / 64];
  const Consts<T> C(s);
  const int nx = s.nx, nt = s.nt, nr = 3 * nt, W = blockDim.x, tid = threadIdx.x;
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(nx);
  C2<T>* alt = dg_fft_pingpong<T>(nx) ? twl + lds_fft_points(nx) : nullptr;
  const int w = xcd_block(blockIdx.x, gridDim.x);
  const size_t L3 = (size_t)3 * nx;
  C2<T> twv[E];
#pragma unroll
  for (int e = 0; e < E; ++e) twv[e] = tw[tid + e * W];
  // residual rows: R[lv][p][e] for level 2w + lv
  T R[2][3][E];
  double rp = 0.0;
#pragma unroll
  for (int lv = 0; lv < 2; ++lv) {
    const int l = 2 * w + lv;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      R[lv][0][e] = R[lv][1][e] = R[lv][2][e] = T(0);
      if (l < nt) {
        const int j = tid + e * W;
        const int jm = (j - 1) & (nx - 1), jp = (j + 1) & (nx - 1);
        const T* up1 = u + (size_t)(l + 1) * L3;
        T v[3], vm[3], vp[3], F[3];
        load_cell(up1, nx, j, v);
        load_cell(up1, nx, jm, vm);
        load_cell(up1, nx, jp, vp);
        dg_spatial(C, v, vm[0] + vm[1] + vm[2], vp[0] - vp[1] + vp[2], F);
        const T c0 = C.c0(l), c1 = C.c1(l), c2 = C.c2(l);
        const bool use2 = l >= 1 && C.time == kTimeBDF2;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          T t = c0 * v[k] + c1 * u[(size_t)l * L3 + (size_t)k * nx + j];
          if (use2) t += c2 * u[(size_t)(l - 1) * L3 + (size_t)k * nx + j];
          const T val = t * C.inv_ht + F[k];
          R[lv][k][e] = val;
          rp += (double)val * (double)val;
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) twl[lpad(tid + e * W)] = twv[e];
  // three complex FFTs: row 6w + 2i + h is (level 2w + (2i + h) / 3, plane (2i + h) % 3)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int ra = 6 * w + 2 * i;
    if (i > 0) __syncthreads();   // the previous round's spectrum reads of buf are done
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int qa = 2 * i, qb = 2 * i + 1;
      buf[lpad(tid + e * W)] = {R[qa / 3][qa % 3][e], R[qb / 3][qb % 3][e]};
    }
    const C2<T>* res = fft_lds<false, E>(buf, nx, twl, tid, W, alt);
    if (ra < nr) store_halfcomplex_pair(res, nx, spec, nr, lqb, ra, ra + 1 < nr, tid, W);
  }
  const double srp = block_sum_waves(rp, red);
  if (tid == 0) part[blockIdx.x] = srp;
}

// ------------------------------------------------------------------ column solve
// Block of 4 waves = 8 spectrum columns = 4 Fourier modes (the first wave of
// block 0 holds the real columns of modes 0 and nx/2).  With NP coefficient
// planes (3 for P2, 2 for P1) the spectrum has NP nt rows, row NP l + p for
// level l and plane p.  The [NP nt][8] tile is staged in LDS; slot (c, p) of
// level l is column c, plane p.  Wave w owns columns 2w (Re) and 2w+1 (Im):
// the 2 NP components r = NP ri + p of its mode.
//   1. rotate every level's 2NP-vector by V^T in LDS (one level per lane at a time)
//   2. per eigen-branch b: banded Cholesky solve along t (lane owns LPL levels)
//   3. rotate back by V
// vtab: 36 values per mode (V row-major with row stride 6, columns = eigenvectors
// of the real 2NP x 2NP form); the factor table of branch b of mode m has index
// 6 m + b.  For the real modes 0 and nx/2 the real form is block-diagonal
// (Im H = 0): branches 0..NP-1 act on the real parts, the only nonzero ones.
template <int LPL, int NP>
__device__ __forceinline__ int dg_slot(int c, int p, int l) {
  return ((c * NP + p) * LPL + l % LPL) * 65 + l / LPL;
}

template <typename T, int LPL, int NP>
__device__ __forceinline__ void dg_rotate(T* tile, const T* __restrict__ V, const int* cs, const int* ps, int ncomp,
                                          bool transpose, int lane, int nt) {
  for (int l = lane; l < nt; l += 64) {
    T x[6], y[6];
    for (int r = 0; r < ncomp; ++r) x[r] = tile[dg_slot<LPL, NP>(cs[r], ps[r], l)];
    for (int b = 0; b < ncomp; ++b) {
      T acc = T(0);
      for (int r = 0; r < ncomp; ++r) acc += (transpose ? V[r * 6 + b] : V[b * 6 + r]) * x[r];
      y[b] = acc;
    }
    for (int b = 0; b < ncomp; ++b) tile[dg_slot<LPL, NP>(cs[b], ps[b], l)] = y[b];
  }
}

template <typename T, int BW, int LPL, int NP>
__device__ __forceinline__ void dg_solve_mode(T* tile, const FacTab<T>& fac, const T* __restrict__ vtab, int mode,
                                              const int* cs, const int* ps, int ncomp, int lane, int nt) {
  const T* V = vtab + (size_t)mode * 36;
  const int l0 = lane * LPL;
  dg_rotate<T, LPL, NP>(tile, V, cs, ps, ncomp, true, lane, nt);        // y = V^T x
  for (int b = 0; b < ncomp; ++b) {
    T invd[LPL], e1[LPL + 1], e2[LPL + 2];
    load_factor_rows<T, LPL>(fac, mode * 6 + b, l0, invd, e1, e2);
    T z[1][LPL];
#pragma unroll
    for (int i = 0; i < LPL; ++i) z[0][i] = tile[dg_slot<LPL, NP>(cs[b], ps[b], l0 + i)];
    cholesky_solve_wave<T, BW, LPL, 1>(z, invd, e1, e2, lane, l0, nt);
#pragma unroll
    for (int i = 0; i < LPL; ++i) tile[dg_slot<LPL, NP>(cs[b], ps[b], l0 + i)] = z[0][i];
  }
  dg_rotate<T, LPL, NP>(tile, V, cs, ps, ncomp, false, lane, nt);       // x = V y
}

template <typename T, int BW, int LPL, int NP>
__global__ void __launch_bounds__(64 * kColWaves)
k_dg_colsolve(T* __restrict__ spec, FacTab<T> fac, const T* __restrict__ vtab, int nt, int nx, int lqb,
              const Ctrl* ctrl) {
  if (ctrl && ctrl->status != 0) return;
  extern __shared__ char smem[];
  T* tile = reinterpret_cast<T*>(smem);   // [8 cols][NP planes][LPL][65]
  const int QB = 1 << lqb, nr = NP * nt;
  const int q0 = xcd_block(blockIdx.x, gridDim.x) * kColCols;
  T* base = spec + (size_t)(q0 >> lqb) * nr * QB + (q0 & (QB - 1));
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  constexpr int kPer = 64 * LPL * kColCols / (64 * kColWaves);   // per plane
  // stage the [NP nt][8] tile through registers, one plane at a time
  for (int p = 0; p < NP; ++p) {
    T stage[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int idx = tid + r * 64 * kColWaves;
      const int l = idx / kColCols, c = idx % kColCols;
      stage[r] = (l < nt) ? base[(size_t)(NP * l + p) * QB + c] : T(0);
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int idx = tid + r * 64 * kColWaves;
      const int l = idx / kColCols, c = idx % kColCols;
      tile[dg_slot<LPL, NP>(c, p, l)] = stage[r];
    }
  }
  __syncthreads();
  const int qa = q0 + 2 * wv;
  if (qa != 0) {   // one complex mode: components (Re, planes 0..NP-1), (Im, planes 0..NP-1)
    int cs[6], ps[6];
#pragma unroll
    for (int r = 0; r < 2 * NP; ++r) {
      cs[r] = 2 * wv + r / NP;
      ps[r] = r % NP;
    }
    dg_solve_mode<T, BW, LPL, NP>(tile, fac, vtab, spec_mode(qa, nx), cs, ps, 2 * NP, lane, nt);
  } else {         // real columns 0 (mode 0) and 1 (mode nx/2)
    int cs0[3], cs1[3], ps[3];
#pragma unroll
    for (int r = 0; r < NP; ++r) {
      cs0[r] = 0;
      cs1[r] = 1;
      ps[r] = r;
    }
    dg_solve_mode<T, BW, LPL, NP>(tile, fac, vtab, 0, cs0, ps, NP, lane, nt);
    dg_solve_mode<T, BW, LPL, NP>(tile, fac, vtab, nx / 2, cs1, ps, NP, lane, nt);
  }
  __syncthreads();
  for (int p = 0; p < NP; ++p) {
    T stage[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int idx = tid + r * 64 * kColWaves;
      const int l = idx / kColCols, c = idx % kColCols;
      stage[r] = tile[dg_slot<LPL, NP>(c, p, l)];
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int idx = tid + r * 64 * kColWaves;
      const int l = idx / kColCols, c = idx % kColCols;
      if (l < nt) base[(size_t)(NP * l + p) * QB + c] = stage[r];
    }
  }
}

// ------------------------------------------------------------------ launchers
static inline unsigned dg_grid(size_t n) { return (unsigned)((n + kDgThreads - 1) / kDgThreads); }

template <typename T>
hipError_t launch_dg_residual(const Scheme& s, const T* u, T* r, double* part, const Ctrl* ctrl, hipStream_t st,
                              int* nblocks) {
  const unsigned g = dg_grid((size_t)s.nt * s.nx);
  if (nblocks) *nblocks = (int)g;
  hipLaunchKernelGGL(k_dg_residual<T>, dim3(g), dim3(kDgThreads), 0, st, s, u, r, part, ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dg_apply_jt(const Scheme& s, const T* u, const T* psi, T* out, double* part, hipStream_t st,
                              int* nblocks) {
  const unsigned g = dg_grid((size_t)s.nt * s.nx);
  if (nblocks) *nblocks = (int)g;
  hipLaunchKernelGGL(k_dg_apply_jt<T>, dim3(g), dim3(kDgThreads), 0, st, s, u, psi, out, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dg_apply_j(const Scheme& s, const T* u, const T* v, T* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dg_apply_j<T>, dim3(dg_grid((size_t)s.nt * s.nx)), dim3(kDgThreads), 0, st, s, u, v, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dg_primal(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                            double* part, const Ctrl* ctrl, hipStream_t st, int* nblocks) {
  const unsigned g = dg_grid((size_t)s.nt * s.nx);
  if (nblocks) *nblocks = (int)g;
  hipLaunchKernelGGL(k_dg_primal<T>, dim3(g), dim3(kDgThreads), 0, st, s, u_in, u_out, phibar, phi, tau_u, part,
                     ctrl);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dg_maxabs_trace(const T* u0, int nx, double a2, double b, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_dg_maxabs_trace<T>, dim3(64), dim3(kDgThreads), 0, st, u0, nx, a2, b, part);
  return hipGetLastError();
}

template <typename T, int E>
static hipError_t launch_dg_residual_fft_e(const Scheme& s, const T* u, T* spec, int lqb, const void* tw,
                                           double* part, const Ctrl* ctrl, hipStream_t st, int* nblocks) {
  const int W = s.nx / E;
  const size_t lds = sizeof(C2<T>) * (dg_fft_pingpong<T>(s.nx) ? 3 : 2) * (size_t)lds_fft_points(s.nx);
  hipError_t e = allow_lds(k_dg_residual_fft<T, E>, lds);
  if (e != hipSuccess) return e;
  const int g = (s.nt + 1) / 2;
  if (nblocks) *nblocks = g;
  hipLaunchKernelGGL((k_dg_residual_fft<T, E>), dim3(g), dim3(W), lds, st, s, u, spec, lqb, (const C2<T>*)tw, part,
                     ctrl);
  return hipGetLastError();
}

// Residual + forward FFT for DG: W = min(512, nx) threads, E = nx / W (nx >= 64).
template <typename T>
hipError_t launch_dg_residual_fft(const Scheme& s, const T* u, T* spec, int lqb, const void* tw, double* part,
                                  const Ctrl* ctrl, hipStream_t st, int* nblocks) {
  const int W = s.nx < 512 ? s.nx : 512;
  switch (s.nx / W) {
    case 1: return launch_dg_residual_fft_e<T, 1>(s, u, spec, lqb, tw, part, ctrl, st, nblocks);
    case 2: return launch_dg_residual_fft_e<T, 2>(s, u, spec, lqb, tw, part, ctrl, st, nblocks);
    case 4: return launch_dg_residual_fft_e<T, 4>(s, u, spec, lqb, tw, part, ctrl, st, nblocks);
    case 8: return launch_dg_residual_fft_e<T, 8>(s, u, spec, lqb, tw, part, ctrl, st, nblocks);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int BW, int LPL, int NP>
static hipError_t launch_dg_colsolve_l(T* spec, const FacTab<T>& fac, const T* vtab, int nt, int nx, int lqb,
                                       const Ctrl* ctrl, hipStream_t st) {
  const size_t lds = sizeof(T) * (size_t)kColCols * NP * LPL * 65;
  hipError_t e = allow_lds(k_dg_colsolve<T, BW, LPL, NP>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_dg_colsolve<T, BW, LPL, NP>), dim3(nx / kColCols), dim3(64 * kColWaves), lds, st, spec, fac,
                     vtab, nt, nx, lqb, ctrl);
  return hipGetLastError();
}

template <typename T, int NP>
static hipError_t launch_dg_colsolve_np(T* spec, const FacTab<T>& fac, const T* vtab, int bw, int nt, int nx, int lqb,
                                        const Ctrl* ctrl, hipStream_t st) {
  const int lpl = (nt + 63) / 64;
#define PDHG_DGC(B, L) return launch_dg_colsolve_l<T, B, L, NP>(spec, fac, vtab, nt, nx, lqb, ctrl, st)
  if (bw == 2) {
    if (lpl <= 1) PDHG_DGC(2, 1);
    if (lpl <= 2) PDHG_DGC(2, 2);
    if (lpl <= 4) PDHG_DGC(2, 4);
    if (lpl <= 8) PDHG_DGC(2, 8);
  } else {
    if (lpl <= 1) PDHG_DGC(1, 1);
    if (lpl <= 2) PDHG_DGC(1, 2);
    if (lpl <= 4) PDHG_DGC(1, 4);
    if (lpl <= 8) PDHG_DGC(1, 8);
  }
#undef PDHG_DGC
  return hipErrorInvalidValue;
}

// np coefficient planes (3: P2, 2: P1); nt <= 512 (LPL <= 8), nx >= 16.
template <typename T>
hipError_t launch_dg_colsolve(T* spec, const FacTab<T>& fac, const T* vtab, int bw, int nt, int nx, int lqb,
                              const Ctrl* ctrl, hipStream_t st, int np) {
  if (np == 2) return launch_dg_colsolve_np<T, 2>(spec, fac, vtab, bw, nt, nx, lqb, ctrl, st);
  if (np == 3) return launch_dg_colsolve_np<T, 3>(spec, fac, vtab, bw, nt, nx, lqb, ctrl, st);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ implicit adjoint (DG)
// The backward march of the dual equation with a source term (Section 3.1), as
// for finite differences: for m = N_t .. 1,
//   (c0(m-1)/h_t I + dF(u^m)^T) mu^{m-1} = g^m - c1(m)/h_t mu^m - c2(m+1)/h_t mu^{m+1},
// then dl/du0 = g^0 - c1(0)/h_t mu^0 - c2(1)/h_t mu^1, per coefficient.  Per
// level the system is periodic block tridiagonal over the cells, NP x NP
// blocks: row j reads  A_j mu_{j-1} + B_j mu_j + C_j mu_{j+1} = d_j  with
//   A_j = U_{j-1}^T, B_j = (c0/h_t I + D_j)^T, C_j = L_{j+1}^T,
// D_j, L_j, U_j the blocks of dF coupling cell j to cells j, j-1, j+1.
//   P2 (LLF; s_k = -(2k+1)/h_x, P_m at the Gauss nodes):
//     D_j[k][m] = s_k (Vol_km - da_{j+1/2} + (-1)^{k+m} db_{j-1/2}),
//     Vol_1m = sum_q w_q f'(u_q) P_m(xi_q), Vol_2m = sum_q w_q f'(u_q) 3 xi_q P_m(xi_q), Vol_0m = 0,
//     U_j[k][m] = -s_k db_{j+1/2} (-1)^m,  L_j[k][m] = s_k (-1)^k da_{j-1/2};
//   P1 (nodal upwind, trace t(v) = -v_1/2 + 3 v_2/2, M^{-1} = [7 1; 1 7] / (4 h_x)):
//     D_j = -M^{-1} [dr1/dv; dr2/dv], dr1/dv_m = -S_m + da_j t_m / 2, dr2/dv_m = S_m - 3 da_j t_m / 2,
//     L_j = -M^{-1} [3 da_{j-1} t / 2; -da_{j-1} t / 2], U_j = 0,
//   with the generalised LLF derivatives of the residual kernels (a's branch on ties).
// The system is solved by block cyclic reduction, in place: at stride s the
// rows i = -1 mod 2s eliminate their neighbours i -+ s (rows = s - 1 mod 2s,
// which keep their coefficients for the back substitution); the last row is
// coupled to itself only (periodic), (A + B + C) x = d; then back substitution
// from stride N_x/2 down to 1.  One workgroup; the block rows live in a
// workspace array (L2-resident: 240 bytes per cell for P2), the multipliers of
// three consecutive levels in another.  Arithmetic in double for both storage
// types, as for finite differences.
constexpr int kDgAdjThreads = 512;

template <int NP>
struct AdjRow {
  static constexpr int kA = 0, kB = NP * NP, kC = 2 * NP * NP, kD = 3 * NP * NP, kLen = 3 * NP * NP + NP;
};

template <int NP>
__device__ __forceinline__ void mat_inv(const double* M, double* R) {
  if (NP == 2) {
    const double id = 1.0 / (M[0] * M[3] - M[1] * M[2]);
    R[0] = M[3] * id;
    R[1] = -M[1] * id;
    R[2] = -M[2] * id;
    R[3] = M[0] * id;
  } else {
    const double c00 = M[4] * M[8] - M[5] * M[7], c01 = M[5] * M[6] - M[3] * M[8], c02 = M[3] * M[7] - M[4] * M[6];
    const double id = 1.0 / (M[0] * c00 + M[1] * c01 + M[2] * c02);
    R[0] = c00 * id;
    R[1] = (M[2] * M[7] - M[1] * M[8]) * id;
    R[2] = (M[1] * M[5] - M[2] * M[4]) * id;
    R[3] = c01 * id;
    R[4] = (M[0] * M[8] - M[2] * M[6]) * id;
    R[5] = (M[2] * M[3] - M[0] * M[5]) * id;
    R[6] = c02 * id;
    R[7] = (M[1] * M[6] - M[0] * M[7]) * id;
    R[8] = (M[0] * M[4] - M[1] * M[3]) * id;
  }
}

// R = X Y (NP x NP, row-major)
template <int NP>
__device__ __forceinline__ void mat_mul(const double* X, const double* Y, double* R) {
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      double a = 0.0;
#pragma unroll
      for (int k = 0; k < NP; ++k) a += X[i * NP + k] * Y[k * NP + j];
      R[i * NP + j] = a;
    }
}

// Block row j of level m (transposed system) from u^m and the right-hand side.
template <typename T, int NP>
__device__ __forceinline__ void adj_build_row(const Consts<double>& C, const T* __restrict__ um, int nx, int j,
                                              double d0, const double* rhs, double* row) {
  typedef AdjRow<NP> R;
  double Dm[NP * NP], Lm[NP * NP], Um[NP * NP];   // D_j, L_{j+1}, U_{j-1} as blocks of dF
  const double h1 = C.inv_hx;
  if constexpr (NP == 3) {
    double v[3], vl[3], vr[3];
    const int jl = (j - 1 + nx) & (nx - 1), jr = (j + 1) & (nx - 1);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v[k] = (double)um[k * nx + j];
      vl[k] = (double)um[k * nx + jl];
      vr[k] = (double)um[k * nx + jr];
    }
    const double a = v[0] + v[1] + v[2], b = v[0] - v[1] + v[2];
    const double a_left = vl[0] + vl[1] + vl[2], b_right = vr[0] - vr[1] + vr[2];
    double da_r, db_r, da_l, db_l;
    llf_partials(C, a, b_right, da_r, db_r);   // interface j+1/2
    llf_partials(C, a_left, b, da_l, db_l);    // interface j-1/2
    double vol1[3] = {0.0, 0.0, 0.0}, vol2[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double x = DgCell<double>::xq(q), p2 = DgCell<double>::p2q(q);
      const double wf = DgCell<double>::wq(q) * C.dflux(v[0] + v[1] * x + v[2] * p2);
      const double P[3] = {1.0, x, p2};
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        vol1[m] += wf * P[m];
        vol2[m] += wf * 3.0 * x * P[m];
      }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double sk = -(2.0 * k + 1.0) * h1, pk = (k & 1) ? -1.0 : 1.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const double pm = (m & 1) ? -1.0 : 1.0;
        const double vol = k == 0 ? 0.0 : (k == 1 ? vol1[m] : vol2[m]);
        Dm[k * 3 + m] = sk * (vol - da_r + pk * pm * db_l);
        Um[k * 3 + m] = -sk * db_l * pm;   // U_{j-1}: db at interface j-1/2
        Lm[k * 3 + m] = sk * pk * da_r;    // L_{j+1}: da at interface j+1/2
      }
    }
  } else {
    double v[2];
    v[0] = (double)um[j];
    v[1] = (double)um[nx + j];
    const double g1 = P1Cell<double>::g1(), g2 = P1Cell<double>::g2();
    const double d0q = C.dflux(g1 * v[0] + g2 * v[1]), d1q = C.dflux(g2 * v[0] + g1 * v[1]);
    const double da = C.dflux(P1Cell<double>::trace(v));
    const double S[2] = {d0q * g1 + d1q * g2, d0q * g2 + d1q * g1};
    const double t[2] = {-0.5, 1.5};
    const double q4 = 0.25 * h1;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const double r1 = -S[m] + 0.5 * da * t[m], r2 = S[m] - 1.5 * da * t[m];
      Dm[m] = -q4 * (7.0 * r1 + r2);
      Dm[2 + m] = -q4 * (r1 + 7.0 * r2);
      // L_{j+1} couples cell j+1 to cell j through cell j's trace
      const double l1 = 1.5 * da * t[m], l2 = -0.5 * da * t[m];
      Lm[m] = -q4 * (7.0 * l1 + l2);
      Lm[2 + m] = -q4 * (l1 + 7.0 * l2);
      Um[m] = 0.0;
      Um[2 + m] = 0.0;
    }
  }
#pragma unroll
  for (int k = 0; k < NP; ++k)
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      // transposed blocks: row m, column k
      row[R::kA + m * NP + k] = Um[k * NP + m];
      row[R::kB + m * NP + k] = Dm[k * NP + m] + (k == m ? d0 : 0.0);
      row[R::kC + m * NP + k] = Lm[k * NP + m];
    }
#pragma unroll
  for (int k = 0; k < NP; ++k) row[R::kD + k] = rhs[k];
}

template <typename T, int NP>
__global__ void __launch_bounds__(kDgAdjThreads)
k_dg_adjoint_march(Scheme s, const T* __restrict__ u, const T* __restrict__ g, T* __restrict__ mu_out,
                   T* __restrict__ grad, double* __restrict__ rows, double* __restrict__ ring) {
  typedef AdjRow<NP> R;
  const Consts<double> C(s);
  const int nx = s.nx, nt = s.nt, tid = threadIdx.x;
  const size_t lev = (size_t)NP * nx;
  // ring slot of level l: (l mod 3); mu^{nt} and mu^{nt+1} are zero
  for (int i = tid; i < NP * nx; i += kDgAdjThreads) {
    ring[((size_t)(nt % 3)) * lev + i] = 0.0;
    ring[((size_t)((nt + 1) % 3)) * lev + i] = 0.0;
  }
  __syncthreads();
  for (int m = nt; m >= 1; --m) {
    const T* um = u + (size_t)m * lev;
    const T* gm = g + (size_t)m * lev;
    const double* mu1 = ring + (size_t)(m % 3) * lev;
    const double* mu2 = ring + (size_t)((m + 1) % 3) * lev;
    double* x = ring + (size_t)((m - 1) % 3) * lev;
    const double d0 = C.c0(m - 1) * C.inv_ht, k1 = C.c1(m) * C.inv_ht, k2 = C.c2(m + 1) * C.inv_ht;
    for (int j = tid; j < nx; j += kDgAdjThreads) {
      double rhs[NP], row[R::kLen];
#pragma unroll
      for (int k = 0; k < NP; ++k)
        rhs[k] = (double)gm[k * nx + j] - k1 * mu1[k * nx + j] - k2 * mu2[k * nx + j];
      adj_build_row<T, NP>(C, um, nx, j, d0, rhs, row);
      double* dst = rows + (size_t)j * R::kLen;
#pragma unroll
      for (int e = 0; e < R::kLen; ++e) dst[e] = row[e];
    }
    __syncthreads();
    // forward reduction
    for (int st = 1; st < nx; st <<= 1) {
      const int n_act = nx / (2 * st);
      for (int q = tid; q < n_act; q += kDgAdjThreads) {
        const int i = 2 * st * q + 2 * st - 1;
        const int il = (i - st) & (nx - 1), ir = (i + st) & (nx - 1);
        double* ri = rows + (size_t)i * R::kLen;
        const double* rl = rows + (size_t)il * R::kLen;
        const double* rr = rows + (size_t)ir * R::kLen;
        double Ai[NP * NP], Bi[NP * NP], Ci[NP * NP], Di[NP], inv[NP * NP], al[NP * NP], be[NP * NP], t[NP * NP];
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) {
          Ai[e] = ri[R::kA + e];
          Bi[e] = ri[R::kB + e];
          Ci[e] = ri[R::kC + e];
        }
#pragma unroll
        for (int e = 0; e < NP; ++e) Di[e] = ri[R::kD + e];
        // alpha = -A_i B_il^{-1}, beta = -C_i B_ir^{-1}
        double Bl[NP * NP], Br[NP * NP];
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) {
          Bl[e] = rl[R::kB + e];
          Br[e] = rr[R::kB + e];
        }
        mat_inv<NP>(Bl, inv);
        mat_mul<NP>(Ai, inv, al);
        mat_inv<NP>(Br, inv);
        mat_mul<NP>(Ci, inv, be);
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) {
          al[e] = -al[e];
          be[e] = -be[e];
        }
        double X[NP * NP];
        // B_i += alpha C_il + beta A_ir
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) X[e] = rl[R::kC + e];
        mat_mul<NP>(al, X, t);
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) Bi[e] += t[e];
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) X[e] = rr[R::kA + e];
        mat_mul<NP>(be, X, t);
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) Bi[e] += t[e];
        // A_i = alpha A_il, C_i = beta C_ir
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) X[e] = rl[R::kA + e];
        mat_mul<NP>(al, X, Ai);
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) X[e] = rr[R::kC + e];
        mat_mul<NP>(be, X, Ci);
        // d_i += alpha d_il + beta d_ir
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          double acc = Di[a];
#pragma unroll
          for (int k = 0; k < NP; ++k) acc += al[a * NP + k] * rl[R::kD + k] + be[a * NP + k] * rr[R::kD + k];
          Di[a] = acc;
        }
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) {
          ri[R::kA + e] = Ai[e];
          ri[R::kB + e] = Bi[e];
          ri[R::kC + e] = Ci[e];
        }
#pragma unroll
        for (int e = 0; e < NP; ++e) ri[R::kD + e] = Di[e];
      }
      __syncthreads();
    }
    // the last row couples to itself only: (A + B + C) x = d
    if (tid == 0) {
      const int i = nx - 1;
      const double* ri = rows + (size_t)i * R::kLen;
      double Mx[NP * NP], inv[NP * NP];
#pragma unroll
      for (int e = 0; e < NP * NP; ++e) Mx[e] = ri[R::kA + e] + ri[R::kB + e] + ri[R::kC + e];
      mat_inv<NP>(Mx, inv);
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < NP; ++k) acc += inv[a * NP + k] * ri[R::kD + k];
        x[a * nx + i] = acc;
      }
    }
    __syncthreads();
    // back substitution: rows s - 1 mod 2s from the solved rows at distance s
    for (int st = nx >> 1; st >= 1; st >>= 1) {
      const int n_act = nx / (2 * st);
      for (int q = tid; q < n_act; q += kDgAdjThreads) {
        const int i = 2 * st * q + st - 1;
        const int il = (i - st) & (nx - 1), ir = (i + st) & (nx - 1);
        const double* ri = rows + (size_t)i * R::kLen;
        double r[NP], Bi[NP * NP], inv[NP * NP];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          double acc = ri[R::kD + a];
#pragma unroll
          for (int k = 0; k < NP; ++k)
            acc -= ri[R::kA + a * NP + k] * x[k * nx + il] + ri[R::kC + a * NP + k] * x[k * nx + ir];
          r[a] = acc;
        }
#pragma unroll
        for (int e = 0; e < NP * NP; ++e) Bi[e] = ri[R::kB + e];
        mat_inv<NP>(Bi, inv);
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < NP; ++k) acc += inv[a * NP + k] * r[k];
          x[a * nx + i] = acc;
        }
      }
      __syncthreads();
    }
    if (mu_out) {
      T* mo = mu_out + (size_t)(m - 1) * lev;
      for (int i = tid; i < NP * nx; i += kDgAdjThreads) mo[i] = (T)x[i];
    }
    __syncthreads();
  }
  // dl/du0 = g^0 - c1(0)/h_t mu^0 - c2(1)/h_t mu^1
  const double k1 = C.c1(0) * C.inv_ht, k2 = (nt >= 2) ? C.c2(1) * C.inv_ht : 0.0;
  const double* mu0 = ring;                           // slot 0 mod 3
  const double* mu1 = ring + (size_t)(1 % 3) * lev;   // slot 1
  for (int i = tid; i < NP * nx; i += kDgAdjThreads)
    grad[i] = (T)((double)g[i] - k1 * mu0[i] - (nt >= 2 ? k2 * mu1[i] : 0.0));
}

// Workspace of the DG adjoint march: block rows and three levels of multipliers (doubles).
size_t dg_adjoint_scratch_doubles(int nx, int np) {
  const int len = 3 * np * np + np;
  return (size_t)nx * len + 3 * (size_t)np * nx;
}

template <typename T>
hipError_t launch_dg_adjoint_march(const Scheme& s, const T* u, const T* g, T* mu, T* grad, double* scratch,
                                   hipStream_t st) {
  const int np = s.space == kSpaceDgP1 ? 2 : 3;
  const size_t len = (size_t)(3 * np * np + np);
  double* rows = scratch;
  double* ring = scratch + (size_t)s.nx * len;
  if (np == 3)
    hipLaunchKernelGGL((k_dg_adjoint_march<T, 3>), dim3(1), dim3(kDgAdjThreads), 0, st, s, u, g, mu, grad, rows, ring);
  else
    hipLaunchKernelGGL((k_dg_adjoint_march<T, 2>), dim3(1), dim3(kDgAdjThreads), 0, st, s, u, g, mu, grad, rows, ring);
  return hipGetLastError();
}

#define PDHG_DG_INSTANTIATE(T)                                                                                   \
  template hipError_t launch_dg_residual<T>(const Scheme&, const T*, T*, double*, const Ctrl*, hipStream_t, int*); \
  template hipError_t launch_dg_apply_jt<T>(const Scheme&, const T*, const T*, T*, double*, hipStream_t, int*);    \
  template hipError_t launch_dg_apply_j<T>(const Scheme&, const T*, const T*, T*, hipStream_t);                   \
  template hipError_t launch_dg_primal<T>(const Scheme&, const T*, T*, const T*, const T*, T, double*, const Ctrl*, \
                                          hipStream_t, int*);                                                    \
  template hipError_t launch_dg_maxabs_trace<T>(const T*, int, double, double, double*, hipStream_t);             \
  template hipError_t launch_dg_residual_fft<T>(const Scheme&, const T*, T*, int, const void*, double*,           \
                                                const Ctrl*, hipStream_t, int*);                                 \
  template hipError_t launch_dg_colsolve<T>(T*, const FacTab<T>&, const T*, int, int, int, int, const Ctrl*,      \
                                            hipStream_t, int);                                                   \
  template hipError_t launch_dg_adjoint_march<T>(const Scheme&, const T*, const T*, T*, T*, double*, hipStream_t);

PDHG_DG_INSTANTIATE(float)
PDHG_DG_INSTANTIATE(double)

}  // namespace pdhg
