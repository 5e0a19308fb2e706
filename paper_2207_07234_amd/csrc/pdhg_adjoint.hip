// Implicit adjoint of the space-time scheme (Section 3.1): a backward march in
// time of the discrete dual equation with a source term.
//
// The converged saddle point solves A(U; u0) = 0.  For a loss l(u^0, U) the
// gradient with respect to u0 is dl/du^0 - (dA/du0)^T mu where J(U)^T mu = dl/dU.
// J^T is block upper triangular in time (the dual equation runs backward from
// phi^{N_t} = 0), so mu is obtained level by level:
//   (c0(m-1)/h_t I + dF(u^m)^T) mu^{m-1} = g^m - c1(m)/h_t mu^m - c2(m+1)/h_t mu^{m+1},
// m = N_t .. 1, one periodic tridiagonal system per level, solved here by
// parallel cyclic reduction in one workgroup.
//
// Arithmetic type A is double for both storage types: a march of N_t solves
// accumulates the rounding of every solve (the backward propagator is a
// contraction, so errors add up rather than decay), about N_t kappa eps in
// total; in float that is ~2e-4 at N_t = 512.  Inputs and outputs keep the
// problem's storage type T.
#include "pdhg_internal.hpp"

namespace pdhg {

constexpr int kAdjThreads = 1024;
constexpr int kAdjMaxE = 4;   // nx <= 4096

template <typename T>
__global__ void __launch_bounds__(kAdjThreads)
k_adjoint_march(Scheme s, const T* __restrict__ u, const T* __restrict__ g, T* __restrict__ mu_out,
                T* __restrict__ grad) {
  typedef double A_t;
  extern __shared__ char smem[];
  const Consts<A_t> C(s);
  const int nx = s.nx, nt = s.nt, tid = threadIdx.x;
  A_t* A = reinterpret_cast<A_t*>(smem);
  A_t* B = A + nx;
  A_t* Cc = B + nx;
  A_t* D = Cc + nx;
  const int E = (nx + kAdjThreads - 1) / kAdjThreads;   // equations per thread: i = tid + e * W
  A_t mu1[kAdjMaxE], mu2[kAdjMaxE];                      // mu^m, mu^{m+1} at my points
#pragma unroll
  for (int e = 0; e < kAdjMaxE; ++e) { mu1[e] = A_t(0); mu2[e] = A_t(0); }

  for (int m = nt; m >= 1; --m) {
    const T* um = u + (size_t)m * nx;
    const T* gm = g + (size_t)m * nx;
    const A_t d0 = C.c0(m - 1) * C.inv_ht;
    const A_t k1 = C.c1(m) * C.inv_ht, k2 = C.c2(m + 1) * C.inv_ht;
#pragma unroll
    for (int e = 0; e < kAdjMaxE; ++e) {
      const int i = tid + e * kAdjThreads;
      if (e < E && i < nx) {
        A_t lo, di, up;
        C.JtF_coeffs((A_t)um[i], lo, di, up);
        A[i] = lo;
        B[i] = di + d0;
        Cc[i] = up;
        D[i] = (A_t)gm[i] - k1 * mu1[e] - k2 * mu2[e];
      }
    }
    __syncthreads();
    // periodic cyclic reduction: distance d doubles until every equation is decoupled
    for (int d = 1; d < nx; d <<= 1) {
      A_t na[kAdjMaxE], nb[kAdjMaxE], nc[kAdjMaxE], nd[kAdjMaxE];
#pragma unroll
      for (int e = 0; e < kAdjMaxE; ++e) {
        const int i = tid + e * kAdjThreads;
        if (e < E && i < nx) {
          const int im = (i - d) & (nx - 1), ip = (i + d) & (nx - 1);
          const A_t al = -A[i] / B[im];
          const A_t be = -Cc[i] / B[ip];
          na[e] = al * A[im];
          nc[e] = be * Cc[ip];
          nb[e] = B[i] + al * Cc[im] + be * A[ip];
          nd[e] = D[i] + al * D[im] + be * D[ip];
        }
      }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < kAdjMaxE; ++e) {
        const int i = tid + e * kAdjThreads;
        if (e < E && i < nx) { A[i] = na[e]; B[i] = nb[e]; Cc[i] = nc[e]; D[i] = nd[e]; }
      }
      __syncthreads();
    }
    T* mo = mu_out ? mu_out + (size_t)(m - 1) * nx : nullptr;
#pragma unroll
    for (int e = 0; e < kAdjMaxE; ++e) {
      const int i = tid + e * kAdjThreads;
      if (e < E && i < nx) {
        const A_t x = D[i] / (A[i] + B[i] + Cc[i]);
        mu2[e] = mu1[e];
        mu1[e] = x;
        if (mo) mo[i] = (T)x;
      }
    }
    __syncthreads();
  }
  // dl/du0 = g^0 - c1(0)/h_t mu^0 - c2(1)/h_t mu^1 ; now mu1 = mu^0, mu2 = mu^1
  const A_t k1 = C.c1(0) * C.inv_ht, k2 = (nt >= 2) ? C.c2(1) * C.inv_ht : A_t(0);
#pragma unroll
  for (int e = 0; e < kAdjMaxE; ++e) {
    const int i = tid + e * kAdjThreads;
    if (e < E && i < nx) grad[i] = (T)((A_t)g[i] - k1 * mu1[e] - k2 * mu2[e]);
  }
}

template <typename T>
hipError_t launch_adjoint_march(const Scheme& s, const T* u, const T* g, T* mu, T* grad, hipStream_t st) {
  const size_t lds = sizeof(double) * 4 * (size_t)s.nx;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adjoint_march<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adjoint_march<T>, dim3(1), dim3(kAdjThreads), lds, st, s, u, g, mu, grad);
  return hipGetLastError();
}

template hipError_t launch_adjoint_march<float>(const Scheme&, const float*, const float*, float*, float*,
                                                hipStream_t);
template hipError_t launch_adjoint_march<double>(const Scheme&, const double*, const double*, double*, double*,
                                                 hipStream_t);

}  // namespace pdhg
