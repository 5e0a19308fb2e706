// One-time-step primal-dual solver (Algorithm 3, Section 3.5) on gfx950.
//
// The implicit scheme is advanced one step per launch.  Step l solves, for
// v = u^{l+1} with u^l (and u^{l-1} for BDF2) known,
//
//     A_l(v) = (c0 v + c1 u^l + c2 u^{l-1}) / h_t + F(v) = 0
//
// by Algorithm 1 on the N_x x 1 space-time mesh: the primal step
// v <- v - tau_u J_l(v)^T phibar with J_l = (c0/h_t) I + dF(v), the dual step
// phi <- phi + tau_phi K_l^{-1} A_l(v) (phibar = phi + 2 tau_phi K_l^{-1} A_l(v)),
// and the stopping rule on the two residuals in the L2 norm of the time slice.
// K_l = (c0/h_t)^2 I + c^2 L_x + ghat^2 L_x^2 is the Gram form of the
// preconditioner with one unknown level; it is diagonal in Fourier space.
//
// One workgroup holds the whole slice for the whole step: N_x <= 4096 points
// are EPT <= 8 values per thread in registers, the FFT runs in LDS, and the
// convergence decision is a block reduction, so an iteration touches no
// global memory.  Wave w owns the contiguous segment [w 64 EPT, (w+1) 64 EPT)
// in lane-cyclic order (element e of lane q is x = seg + q + 64 e): stencil
// neighbours inside a wave come from DPP lane shifts, and only the two
// segment ends of each wave pass through LDS.
#include "pdhg_internal.hpp"
#include "pdhg_passes.hpp"

namespace pdhg {

constexpr int kOneStepThreadsMax = 512;

// Periodic neighbours of a lane-cyclic row segment, with the segment ends of
// the neighbouring waves exchanged through LDS slot `ends` ([2][nw]: first,
// last).  Block-wide: every thread calls it.
template <typename T, int EPT>
__device__ __forceinline__ void slice_neighbours(const T* a, T* am, T* ap, T* ends, int wv, int nw, int lane) {
  if (lane == 0) ends[wv] = a[0];
  if (lane == 63) ends[nw + wv] = a[EPT - 1];
  __syncthreads();
  const T prev_last = ends[nw + (wv + nw - 1) % nw];
  const T next_first = ends[(wv + 1) % nw];
  wave_row_neighbours<T, EPT>(a, prev_last, next_first, am, ap);
}

// One block of W = nx / EPT threads advances the problem by step l.
// sym: [2][nx] eigenvalue reciprocals 1 / (N_x ((c0/h_t)^2 + c^2 mu_k + ghat^2 mu_k^2)) per FFT
// index k, row 0 for c0 = 1, row 1 for c0 = 3/2 (BDF2 rows l >= 1).
template <typename T, int EPT>
__global__ void __launch_bounds__(kOneStepThreadsMax)
k_onestep(Scheme sch, const C2<T>* __restrict__ tw, const T* __restrict__ sym, T* __restrict__ u,
          T* __restrict__ phi, int l, T tau_u, T tau_phi, double eps, long long max_iter, double dfac,
          StepStat* __restrict__ stat, int* __restrict__ flag) {
  if (*flag != 0) return;   // an earlier step diverged: the march has stopped
  extern __shared__ char smem[];
  __shared__ T ends[3][2 * (kOneStepThreadsMax / 64)];
  __shared__ double red[2][kOneStepThreadsMax / 64];
  const Consts<T> C(sch);
  const int nx = sch.nx, W = blockDim.x, tid = threadIdx.x;
  const int nw = W >> 6, wv = tid >> 6, lane = tid & 63;
  const int seg = wv * 64 * EPT;
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(nx);
  load_twiddles_lds(twl, tw, nx, tid, W);

  const T c0 = C.c0(l), c1 = C.c1(l), c2 = C.c2(l);
  const T a0 = c0 * C.inv_ht;
  const T* ul = u + (size_t)l * nx;
  const T* ulm = ul - (l >= 1 ? nx : 0);
  const T* symr = sym + (c0 != T(1) ? nx : 0);
  T v[EPT], known[EPT], ph[EPT], pb[EPT], g[EPT], dk[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int x = seg + lane + 64 * e;
    v[e] = ul[x];
    known[e] = (c1 * ul[x] + c2 * ulm[x]) * C.inv_ht;
    dk[e] = symr[x];
    ph[e] = pb[e] = g[e] = T(0);
  }
  const double hx = sch.hx;
  double rp = 0.0, rd = 0.0, best = INFINITY;
  long long n = 0;
  int status = 1;
  while (n < max_iter) {
    ++n;
    // primal step with J_l(v^{n-1})^T phibar^{n-1} (g, from the previous iteration)
#pragma unroll
    for (int e = 0; e < EPT; ++e) v[e] -= tau_u * g[e];
    // implicit residual A_l(v^n) into the FFT buffer
    T vm[EPT], vp[EPT];
    slice_neighbours<T, EPT>(v, vm, vp, ends[0], wv, nw, lane);
    double srp = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int x = seg + lane + 64 * e;
      const T r = a0 * v[e] + known[e] + C.F(vm[e], v[e], vp[e]);
      srp += (double)r * (double)r;
      buf[lpad(x)] = C2<T>{r, T(0)};
    }
    // s = K_l^{-1} r: forward FFT, per-mode scaling (each thread scales the indices it wrote), inverse FFT
    fft_lds<false, EPT>(buf, nx, twl, tid, W);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int k = seg + lane + 64 * e;
      C2<T> z = buf[lpad(k)];
      z.x *= dk[e];
      z.y *= dk[e];
      buf[lpad(k)] = z;
    }
    fft_lds<true, EPT>(buf, nx, twl, tid, W);
    // dual step and extrapolation
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int x = seg + lane + 64 * e;
      const T s = buf[lpad(x)].x;
      pb[e] = ph[e] + T(2) * tau_phi * s;
      ph[e] = ph[e] + tau_phi * s;
    }
    // J_l(v^n)^T phi^n (dual residual) and J_l(v^n)^T phibar^n (next primal step)
    T pm[EPT], pp[EPT], qm[EPT], qp[EPT];
    slice_neighbours<T, EPT>(ph, pm, pp, ends[1], wv, nw, lane);
    slice_neighbours<T, EPT>(pb, qm, qp, ends[2], wv, nw, lane);
    double srd = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const T h = a0 * ph[e] + C.JtF(v[e], pm[e], ph[e], pp[e]);
      srd += (double)h * (double)h;
      g[e] = a0 * pb[e] + C.JtF(v[e], qm[e], pb[e], qp[e]);
    }
    // block sums in a fixed order, read by every thread: a uniform decision
    srp = wave_sum(srp);
    srd = wave_sum(srd);
    if (lane == 0) {
      red[0][wv] = srp;
      red[1][wv] = srd;
    }
    __syncthreads();
    double sp = 0.0, sd = 0.0;
    for (int i = 0; i < nw; ++i) {
      sp += red[0][i];
      sd += red[1][i];
    }
    rp = sqrt(hx * sp);
    rd = sqrt(hx * sd);
    const double m = fmax(rp, rd);
    if (!(isfinite(rp) && isfinite(rd)) || (m > dfac * best)) {
      status = 2;
      break;
    }
    best = fmin(best, m);
    if (m <= eps) {
      status = 0;
      break;
    }
  }
  T* un = u + (size_t)(l + 1) * nx;
  T* pl = phi + (size_t)l * nx;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int x = seg + lane + 64 * e;
    un[x] = v[e];
    pl[x] = ph[e];
  }
  if (tid == 0) {
    stat[l].iters = n;
    stat[l].rp = rp;
    stat[l].rd = rd;
    stat[l].status = status;
    if (status == 2) *flag = 2;
  }
}

template <typename T, int EPT>
static hipError_t launch_onestep_e(const Scheme& s, const void* tw, const T* sym, T* u, T* phi, int l, T tau_u,
                                   T tau_phi, double eps, long long max_iter, double dfac, StepStat* stat, int* flag,
                                   hipStream_t st) {
  const int W = s.nx / EPT;
  const size_t lds = sizeof(C2<T>) * 2 * (size_t)lds_fft_points(s.nx);
  hipError_t e = allow_lds(k_onestep<T, EPT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_onestep<T, EPT>), dim3(1), dim3(W), lds, st, s, (const C2<T>*)tw, sym, u, phi, l, tau_u,
                     tau_phi, eps, max_iter, dfac, stat, flag);
  return hipGetLastError();
}

// W = max(64, nx / 8) threads (one radix-8 butterfly per thread and FFT stage), EPT = nx / W.
template <typename T>
hipError_t launch_onestep(const Scheme& s, const void* tw, const T* sym, T* u, T* phi, int l, T tau_u, T tau_phi,
                          double eps, long long max_iter, double dfac, StepStat* stat, int* flag, hipStream_t st) {
  if (s.nx < 64 || s.nx > 4096 || (s.nx & (s.nx - 1))) return hipErrorInvalidValue;
  const int W = s.nx / 8 < 64 ? 64 : s.nx / 8;
  switch (s.nx / W) {
    case 1: return launch_onestep_e<T, 1>(s, tw, sym, u, phi, l, tau_u, tau_phi, eps, max_iter, dfac, stat, flag, st);
    case 2: return launch_onestep_e<T, 2>(s, tw, sym, u, phi, l, tau_u, tau_phi, eps, max_iter, dfac, stat, flag, st);
    case 4: return launch_onestep_e<T, 4>(s, tw, sym, u, phi, l, tau_u, tau_phi, eps, max_iter, dfac, stat, flag, st);
    case 8: return launch_onestep_e<T, 8>(s, tw, sym, u, phi, l, tau_u, tau_phi, eps, max_iter, dfac, stat, flag, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_onestep<float>(const Scheme&, const void*, const float*, float*, float*, int, float, float,
                                          double, long long, double, StepStat*, int*, hipStream_t);
template hipError_t launch_onestep<double>(const Scheme&, const void*, const double*, double*, double*, int, double,
                                           double, double, long long, double, StepStat*, int*, hipStream_t);

}  // namespace pdhg
