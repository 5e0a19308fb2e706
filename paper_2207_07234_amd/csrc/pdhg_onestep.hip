// One-time-step primal-dual solver (Algorithm 3, Section 3.5) on gfx950.
//
// The implicit scheme is advanced one step at a time.  Step l solves, for
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
// One workgroup holds one problem for a whole range of steps: N_x <= 4096
// points are EPT <= 8 values per thread in registers, u^l and the known part
// of the time difference stay in registers from one step to the next, the
// FFT runs in LDS, and the convergence decision is a block reduction, so an
// iteration touches no global memory; a step reads nothing and writes its
// level, its dual row and its record.  Wave w owns the contiguous segment
// [w 64 EPT, (w+1) 64 EPT) in lane-cyclic order (element e of lane q is
// x = seg + q + 64 e): stencil neighbours inside a wave come from DPP lane
// shifts, and only the two segment ends of each wave pass through LDS.  A
// launch takes a table of problems, one block each (a batch, or a single
// problem); threads beyond a problem's W = max(64, N_x/8) take part in the
// barriers only.
//
// K_l^{-1} of a real row through a half-length complex FFT: the row r, read
// as M = N_x/2 complex values z_m = r_{2m} + i r_{2m+1}, is exactly the LDS
// buffer viewed as reals.  After Z = FFT_M(z), the N-point spectrum is
// R_k = E_k + w^k O_k and R_{k+M} = E_k - w^k O_k (w = e^{-2 pi i/N}) with
// E_k = (Z_k + conj Z_{M-k})/2, O_k = (Z_k - conj Z_{M-k})/(2i) the spectra of
// the even and odd samples.  Scaling by the real, even symbol d and packing
// back, Y_k = (S_k + S_{k+M})/2 + i (S_k - S_{k+M}) conj(w^k)/2, makes
// IFFT_M(Y) = M (s_{2m} + i s_{2m+1}); d carries the 1/M.  The pair (k, M-k)
// is handled by one thread, which writes both Y_k and Y_{M-k}.
#include "pdhg_internal.hpp"
#include "pdhg_passes.hpp"

namespace pdhg {

constexpr int kOneStepThreadsMax = 512;
constexpr int kOneStepWavesMax = kOneStepThreadsMax / 64;

// Periodic neighbours of lane-cyclic row segments: the segment ends of each
// active wave go through LDS ([2][nw]: first, last), one barrier for all NR
// rows.  Block-wide: every thread calls it.
template <typename T, int EPT, int NR>
__device__ __forceinline__ void slice_neighbours(T (*rows)[EPT], T (*rm)[EPT], T (*rp)[EPT],
                                                 T (*ends)[2 * kOneStepWavesMax], bool act, int wv, int nw,
                                                 int lane) {
  if (act) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      if (lane == 0) ends[i][wv] = rows[i][0];
      if (lane == 63) ends[i][nw + wv] = rows[i][EPT - 1];
    }
  }
  __syncthreads();
  const int wp = nw + (wv + nw - 1) % nw, wn = (wv + 1) % nw;
#pragma unroll
  for (int i = 0; i < NR; ++i) wave_row_neighbours<T, EPT>(rows[i], ends[i][wp], ends[i][wn], rm[i], rp[i]);
}

// Spectral pair (k, q = M - k mod M) of the real-row preconditioner: Z_k, Z_q -> Y_k, Y_q.
// a = d_k, b = d_{k+M}, w = e^{-2 pi i k / N}.
template <typename T>
__device__ __forceinline__ void precond_pair(C2<T>* buf, int k, int q, T a, T b, C2<T> w) {
  const C2<T> zk = buf[lpad(k)], zq = buf[lpad(q)];
  const T ex = T(0.5) * (zk.x + zq.x), ey = T(0.5) * (zk.y - zq.y);   // E = (Z_k + conj Z_q) / 2
  const T ox = T(0.5) * (zk.y + zq.y), oy = T(-0.5) * (zk.x - zq.x);  // O = (Z_k - conj Z_q) / (2i)
  const T wox = w.x * ox - w.y * oy, woy = w.x * oy + w.y * ox;      // w O
  const T skx = a * (ex + wox), sky = a * (ey + woy);                 // S_k = d_k R_k
  const T smx = b * (ex - wox), smy = b * (ey - woy);                 // S_{k+M} = d_{k+M} R_{k+M}
  const T sex = T(0.5) * (skx + smx), sey = T(0.5) * (sky + smy);     // (S_k + S_{k+M}) / 2
  const T dx = T(0.5) * (skx - smx), dy = T(0.5) * (sky - smy);
  const T sox = dx * w.x + dy * w.y, soy = dy * w.x - dx * w.y;       // (S_k - S_{k+M}) conj(w) / 2
  buf[lpad(k)] = C2<T>{sex - soy, sey + sox};                         // Y_k = SE + i SO
  if (q != k) buf[lpad(q)] = C2<T>{sex + soy, sox - sey};            // Y_q = conj(SE) + i conj(SO)
}

// Steps [l_begin, l_end) of problem P on a block whose first W = nx / EPT threads are active.
template <typename T, int EPT>
__device__ __forceinline__ void onestep_march(const OneStepProb<T>& P, int W, int l_begin, int l_end, double eps,
                                              long long max_iter, double dfac, C2<T>* buf, C2<T>* twl,
                                              T (*ends)[2 * kOneStepWavesMax], double (*red)[kOneStepWavesMax]) {
  const Scheme& sch = P.s;
  const Consts<T> C(sch);
  const int nx = sch.nx, M = nx >> 1, tid = threadIdx.x;
  const bool act = tid < W;
  const int nw = W >> 6, wv = tid >> 6, lane = tid & 63;
  const int seg = wv * 64 * EPT;
  const T tau_u = (T)P.tau_u, tau_phi = (T)P.tau_phi;
  for (int i = tid; i < M; i += blockDim.x) twl[lpad(i)] = P.tw[2 * i];   // e^{-2 pi i i' / M}
  T* bufr = reinterpret_cast<T*>(buf);
  // spectral pairs k = tid + j W < M/2 (and k = M/2, self-paired, on thread 0)
  constexpr int KP = EPT >= 4 ? EPT / 4 : 1;
  C2<T> pw[KP];
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const int k = tid + j * W;
    pw[j] = (act && k < (M >> 1)) ? P.tw[k] : C2<T>{T(1), T(0)};
  }
  // cur = u^l, known = (c1 u^l + c2 u^{l-1}) / h_t at the first step
  T cur[EPT], known[EPT];
  {
    const T c1 = C.c1(l_begin), c2 = C.c2(l_begin);
    const T* ul = P.u + (size_t)l_begin * nx;
    const T* ulm = ul - (l_begin >= 1 ? nx : 0);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int x = seg + lane + 64 * e;
      cur[e] = act ? ul[x] : T(0);
      known[e] = act ? (c1 * cur[e] + c2 * ulm[x]) * C.inv_ht : T(0);
    }
  }
  const double hx = sch.hx;
  for (int l = l_begin; l < l_end; ++l) {
    const T c0 = C.c0(l);
    const T a0 = c0 * C.inv_ht;
    const T* symr = P.sym + (c0 != T(1) ? nx : 0);
    T pa[KP], pq[KP];
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      const int k = tid + j * W;
      const bool ok = act && k < (M >> 1);
      pa[j] = ok ? symr[k] : T(0);
      pq[j] = ok ? symr[k + M] : T(0);
    }
    const T dmid = symr[M >> 1];
    // initial guess v = u^l, phi = phibar = 0 (so the first primal step is void)
    T v[1][EPT], ph[2][EPT], g[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      v[0][e] = cur[e];
      ph[0][e] = ph[1][e] = g[e] = T(0);
    }
    double rp = 0.0, rd = 0.0, best = INFINITY;
    long long n = 0;
    int status = 1;
    while (n < max_iter) {
      ++n;
      // primal step with J_l(v^{n-1})^T phibar^{n-1} (g, from the previous iteration)
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[0][e] -= tau_u * g[e];
      // implicit residual A_l(v^n) into the FFT buffer
      T vm[1][EPT], vp[1][EPT];
      slice_neighbours<T, EPT, 1>(v, vm, vp, ends, act, wv, nw, lane);
      double srp = 0.0;
      if (act) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int x = seg + lane + 64 * e;
          const T r = a0 * v[0][e] + known[e] + C.F(vm[0][e], v[0][e], vp[0][e]);
          srp += (double)r * (double)r;
          bufr[2 * lpad(x >> 1) + (x & 1)] = r;   // z_m = r_{2m} + i r_{2m+1}
        }
      }
      // s = K_l^{-1} r: half-length forward FFT, spectral pairs, half-length inverse FFT
      fft_lds<false, (EPT + 1) / 2>(buf, M, twl, tid, W);
      if (act) {
#pragma unroll
        for (int j = 0; j < KP; ++j) {
          const int k = tid + j * W;
          if (k < (M >> 1)) precond_pair(buf, k, (M - k) & (M - 1), pa[j], pq[j], pw[j]);
        }
      }
      if (tid == 0) {   // k = M/2: Y = d_{M/2} Z
        C2<T> z = buf[lpad(M >> 1)];
        z.x *= dmid;
        z.y *= dmid;
        buf[lpad(M >> 1)] = z;
      }
      fft_lds<true, (EPT + 1) / 2>(buf, M, twl, tid, W);
      // dual step and extrapolation: ph[0] = phi, ph[1] = phibar
      if (act) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int x = seg + lane + 64 * e;
          const T s = bufr[2 * lpad(x >> 1) + (x & 1)];
          ph[1][e] = ph[0][e] + T(2) * tau_phi * s;
          ph[0][e] = ph[0][e] + tau_phi * s;
        }
      }
      // J_l(v^n)^T phi^n (dual residual) and J_l(v^n)^T phibar^n (next primal step)
      T pm[2][EPT], pp[2][EPT];
      slice_neighbours<T, EPT, 2>(ph, pm, pp, ends + 1, act, wv, nw, lane);
      double srd = 0.0;
      if (act) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const T h = a0 * ph[0][e] + C.JtF(v[0][e], pm[0][e], ph[0][e], pp[0][e]);
          srd += (double)h * (double)h;
          g[e] = a0 * ph[1][e] + C.JtF(v[0][e], pm[1][e], ph[1][e], pp[1][e]);
        }
      }
      // block sums in a fixed order, read by every thread: a uniform decision
      srp = wave_sum(srp);
      srd = wave_sum(srd);
      if (act && lane == 0) {
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
    if (act) {
      T* un = P.u + (size_t)(l + 1) * nx;
      T* pl = P.phi + (size_t)l * nx;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int x = seg + lane + 64 * e;
        un[x] = v[0][e];
        pl[x] = ph[0][e];
      }
    }
    if (tid == 0) {
      P.stat[l].iters = n;
      P.stat[l].rp = rp;
      P.stat[l].rd = rd;
      P.stat[l].status = status;
      if (status == 2) *P.flag = 2;
    }
    if (status == 2) return;   // uniform: the march of this problem stops
    // next step: known = (c1 u^{l+1} + c2 u^l) / h_t, cur = u^{l+1}
    const T c1n = C.c1(l + 1), c2n = C.c2(l + 1);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      known[e] = (c1n * v[0][e] + c2n * cur[e]) * C.inv_ht;
      cur[e] = v[0][e];
    }
  }
}

// Block b marches problem probs[b] over steps [l_begin, min(l_end, nt)).
template <typename T>
__global__ void __launch_bounds__(kOneStepThreadsMax)
k_onestep(const OneStepProb<T>* __restrict__ probs, int l_begin, int l_end, double eps, long long max_iter,
          double dfac) {
  const OneStepProb<T> P = probs[blockIdx.x];
  if (*P.flag != 0) return;   // this problem's march has stopped (diverged step)
  const int le = l_end < P.s.nt ? l_end : P.s.nt;
  if (l_begin >= le) return;
  extern __shared__ char smem[];
  __shared__ T ends[3][2 * kOneStepWavesMax];
  __shared__ double red[2][kOneStepWavesMax];
  const int M = P.s.nx >> 1;
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(M);
  const int W = onestep_threads(P.s.nx);
  switch (P.s.nx / W) {
    case 8: onestep_march<T, 8>(P, W, l_begin, le, eps, max_iter, dfac, buf, twl, ends, red); break;
    case 4: onestep_march<T, 4>(P, W, l_begin, le, eps, max_iter, dfac, buf, twl, ends, red); break;
    case 2: onestep_march<T, 2>(P, W, l_begin, le, eps, max_iter, dfac, buf, twl, ends, red); break;
    default: onestep_march<T, 1>(P, W, l_begin, le, eps, max_iter, dfac, buf, twl, ends, red); break;
  }
}

// nprob problems (device table), block size = the largest problem's W; LDS for the largest nx.
template <typename T>
hipError_t launch_onestep(const OneStepProb<T>* probs, int nprob, int max_nx, int l_begin, int l_end, double eps,
                          long long max_iter, double dfac, hipStream_t st) {
  if (max_nx < 64 || max_nx > 4096 || (max_nx & (max_nx - 1)) || nprob < 1) return hipErrorInvalidValue;
  const int W = onestep_threads(max_nx);
  const size_t lds = sizeof(C2<T>) * 2 * (size_t)lds_fft_points(max_nx / 2);
  hipError_t e = allow_lds(k_onestep<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_onestep<T>), dim3(nprob), dim3(W), lds, st, probs, l_begin, l_end, eps, max_iter, dfac);
  return hipGetLastError();
}

template hipError_t launch_onestep<float>(const OneStepProb<float>*, int, int, int, int, double, long long, double,
                                          hipStream_t);
template hipError_t launch_onestep<double>(const OneStepProb<double>*, int, int, int, int, double, long long, double,
                                           hipStream_t);

}  // namespace pdhg
