// Implicit adjoint of the space-time scheme (Section 3.1): a backward march in
// time of the discrete dual equation with a source term.
//
// The converged saddle point solves A(U; u0) = 0.  For a loss l(u^0, U) the
// gradient with respect to u0 is dl/du^0 - (dA/du0)^T mu where J(U)^T mu = dl/dU.
// J^T is block upper triangular in time (the dual equation runs backward from
// phi^{N_t} = 0), so mu is obtained level by level:
//   (c0(m-1)/h_t I + dF(u^m)^T) mu^{m-1} = g^m - c1(m)/h_t mu^m - c2(m+1)/h_t mu^{m+1},
// m = N_t .. 1, one periodic tridiagonal system per level, solved here by
// parallel cyclic reduction in one workgroup (stopping once decoupled).
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

// Parallel cyclic reduction per level: each pass doubles the coupling distance
// d and squares the off-diagonals' size relative to the diagonal (about rho^(2^k)
// after k passes, rho the coupling ratio of the level's system), so the passes
// stop once every equation is decoupled to 2^-60 of its diagonal (a block-wide
// vote at the pass's barrier), at the latest when d reaches nx.  Where two sets
// of the four coefficient arrays fit in LDS (nx <= 2048, 128 KiB) the passes alternate
// between them, one barrier per pass; otherwise each pass updates in place
// through registers (two barriers).
template <typename T>
__global__ void __launch_bounds__(kAdjThreads)
k_adjoint_march(Scheme s, const T* __restrict__ u, const T* __restrict__ g, T* __restrict__ mu_out,
                T* __restrict__ grad, int pingpong) {
  typedef double A_t;
  extern __shared__ char smem[];
  const Consts<A_t> C(s);
  const int nx = s.nx, nt = s.nt, tid = threadIdx.x;
  A_t* lds = reinterpret_cast<A_t*>(smem);   // [set][A, B, C, D][nx]; set 1 only with pingpong
  const int E = (nx + kAdjThreads - 1) / kAdjThreads;   // equations per thread: i = tid + e * W
  A_t mu1[kAdjMaxE], mu2[kAdjMaxE];                      // mu^m, mu^{m+1} at my points
#pragma unroll
  for (int e = 0; e < kAdjMaxE; ++e) { mu1[e] = A_t(0); mu2[e] = A_t(0); }
  const A_t tiny = 0x1p-60;
  __shared__ int vote[2][kAdjThreads / 64];   // per-wave "still coupled" flags, alternating by pass
  const int lane = tid & 63, wv = tid >> 6;

  for (int m = nt; m >= 1; --m) {
    const T* um = u + (size_t)m * nx;
    const T* gm = g + (size_t)m * nx;
    const A_t d0 = C.c0(m - 1) * C.inv_ht;
    const A_t k1 = C.c1(m) * C.inv_ht, k2 = C.c2(m + 1) * C.inv_ht;
    {
      A_t* A = lds;
      A_t* B = lds + nx;
      A_t* Cc = lds + 2 * nx;
      A_t* D = lds + 3 * nx;
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
    }
    __syncthreads();
    int cur = 0, pass = 0;
    for (int d = 1; d < nx; d <<= 1, ++pass) {
      const A_t* A = lds + (size_t)cur * 4 * nx;
      const A_t* B = A + nx;
      const A_t* Cc = A + 2 * nx;
      const A_t* D = A + 3 * nx;
      A_t na[kAdjMaxE], nb[kAdjMaxE], nc[kAdjMaxE], nd[kAdjMaxE];
      int coupled = 0;
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
          coupled |= fabs(na[e]) + fabs(nc[e]) > tiny * fabs(nb[e]);
        }
      }
      if (!pingpong) __syncthreads();   // every read of this pass is done before the in-place writes
      const int nxt = pingpong ? cur ^ 1 : cur;
      A_t* W = lds + (size_t)nxt * 4 * nx;
#pragma unroll
      for (int e = 0; e < kAdjMaxE; ++e) {
        const int i = tid + e * kAdjThreads;
        if (e < E && i < nx) {
          W[i] = na[e];
          W[nx + i] = nb[e];
          W[2 * nx + i] = nc[e];
          W[3 * nx + i] = nd[e];
        }
      }
      cur = nxt;
      // this pass's vote: slot pass & 1 was last read two passes ago, before the previous barrier
      const bool wave_coupled = __any(coupled);
      if (lane == 0) vote[pass & 1][wv] = wave_coupled ? 1 : 0;
      __syncthreads();   // publishes this pass's coefficients and votes
      int any = 0;
#pragma unroll
      for (int w = 0; w < kAdjThreads / 64; ++w) any |= vote[pass & 1][w];
      if (!any) break;   // every row decoupled to 2^-60 of its diagonal
    }
    T* mo = mu_out ? mu_out + (size_t)(m - 1) * nx : nullptr;
    {
      const A_t* A = lds + (size_t)cur * 4 * nx;
      const A_t* B = A + nx;
      const A_t* Cc = A + 2 * nx;
      const A_t* D = A + 3 * nx;
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
  const int pingpong = 8 * sizeof(double) * (size_t)s.nx <= 128 * 1024 ? 1 : 0;
  const size_t lds = sizeof(double) * (pingpong ? 8 : 4) * (size_t)s.nx;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_adjoint_march<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adjoint_march<T>, dim3(1), dim3(kAdjThreads), lds, st, s, u, g, mu, grad, pingpong);
  return hipGetLastError();
}

template hipError_t launch_adjoint_march<float>(const Scheme&, const float*, const float*, float*, float*,
                                                hipStream_t);
template hipError_t launch_adjoint_march<double>(const Scheme&, const double*, const double*, double*, double*,
                                                 hipStream_t);

}  // namespace pdhg
