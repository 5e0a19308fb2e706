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
                                            hipStream_t, int);

PDHG_DG_INSTANTIATE(float)
PDHG_DG_INSTANTIATE(double)

}  // namespace pdhg
