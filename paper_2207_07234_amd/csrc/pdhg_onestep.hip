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
// problem); threads beyond a problem's W (onestep_threads: N_x/4 in FP64,
// N_x/8 in FP32, within [64, 512]) take part in the barriers only.
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
//
// Without the fourth-order term (ghat = 0) K_l is the constant-coefficient
// periodic tridiagonal d x_i - e (x_{i-1} + x_{i+1}) = r_i, d = (c0/h_t)^2 + 2 c^2/h_x^2,
// e = c^2/h_x^2, and cyclic reduction solves it with no FFT: step k replaces
// r_i by r_i + rho_k (r_{i-2^k} + r_{i+2^k}), rho_k = e_k/d_k, with
// d_{k+1} = d_k - 2 e_k^2/d_k, e_{k+1} = e_k^2/d_k; rho_k falls quadratically, and
// once it is below the rounding level x_i = r_i / d_k.  The host computes the
// ratios (long double) and chooses this path only when it ends before the
// wrap-around distance N_x/2 (otherwise the FFT path is used).  Each step is
// one LDS pass over the slice (double-buffered, one barrier).
#include "pdhg_internal.hpp"
#include "pdhg_passes.hpp"
#include "pdhg_dg1.hpp"

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

// Per-thread constants of the spectral pairs k = tid + j W < M/2 for one symbol row.
template <typename T, int KP>
struct PairConsts {
  T a[KP], b[KP];   // d_k, d_{k+M}
  C2<T> w[KP];      // e^{-2 pi i k / N}
  T mid;            // d_{M/2}
  int pcr_k;        // > 0: cyclic reduction with pcr[0..pcr_k-1] and scale pcr[15] instead of the FFT
  const T* pcr;
};

// This block's problem entry, with its pointers re-typed as global (they are
// read from the problem table, so the compiler cannot infer their space).
template <typename T>
__device__ __forceinline__ OneStepProb<T> load_prob(const OneStepProb<T>* __restrict__ probs) {
  OneStepProb<T> P = probs[blockIdx.x];
  P.tw = as_global(P.tw);
  P.sym = as_global(P.sym);
  P.u0 = as_global(P.u0);
  P.u = as_global(P.u);
  P.phi = as_global(P.phi);
  P.stat = as_global(P.stat);
  P.flag = as_global(P.flag);
  P.pcr = as_global(P.pcr);
  return P;
}

// Symbol (or cyclic-reduction coefficients) of row r (0: c0 = 1, 1: c0 = 3/2).
template <typename T, int KP>
__device__ __forceinline__ void load_pair_symbol(PairConsts<T, KP>& pc, const OneStepProb<T>& P, int r, bool act,
                                                 int tid, int W, int M) {
  pc.pcr_k = P.pcr_k[r];
  pc.pcr = as_global(P.pcr + 16 * r);
  if (pc.pcr_k > 0) return;
  const T* symr = as_global(P.sym + (size_t)r * 2 * M);
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const int k = tid + j * W;
    const bool ok = act && k < (M >> 1);
    pc.a[j] = ok ? symr[k] : T(0);
    pc.b[j] = ok ? symr[k + M] : T(0);
  }
  pc.mid = symr[M >> 1];
}

// row <- K_l^{-1} row for the slice held in lane-cyclic order (block-wide; the
// caller separates consecutive calls by at least one barrier).
template <typename T, int EPT, int KP>
__device__ __forceinline__ void kinv_slice(T (&row)[EPT], const PairConsts<T, KP>& pc, bool act, int seg, int lane,
                                           int tid, int W, int M, C2<T>* buf, C2<T>* twl) {
  T* bufr = reinterpret_cast<T*>(buf);
  if (pc.pcr_k > 0) {   // cyclic reduction: LDS arrays buf and twl (N reals each), alternating
    const int nm = 2 * M - 1;
    for (int k = 0; k < pc.pcr_k; ++k) {
      T* A = (k & 1) ? reinterpret_cast<T*>(twl) : bufr;
      const int D = 1 << k;
      const T rho = pc.pcr[k];
      if (act) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) A[seg + lane + 64 * e] = row[e];
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int x = seg + lane + 64 * e;
          row[e] += rho * (A[(x - D) & nm] + A[(x + D) & nm]);
        }
      }
    }
    const T fin = pc.pcr[15];
#pragma unroll
    for (int e = 0; e < EPT; ++e) row[e] *= fin;
    return;
  }
  if (act) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int x = seg + lane + 64 * e;
      bufr[2 * lpad(x >> 1) + (x & 1)] = row[e];   // z_m = r_{2m} + i r_{2m+1}
    }
  }
  fft_lds<false, (EPT + 1) / 2>(buf, M, twl, tid, W);
  if (act) {
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      const int k = tid + j * W;
      if (k < (M >> 1)) precond_pair(buf, k, (M - k) & (M - 1), pc.a[j], pc.b[j], pc.w[j]);
    }
  }
  if (tid == 0) {   // k = M/2: Y = d_{M/2} Z
    C2<T> z = buf[lpad(M >> 1)];
    z.x *= pc.mid;
    z.y *= pc.mid;
    buf[lpad(M >> 1)] = z;
  }
  fft_lds<true, (EPT + 1) / 2>(buf, M, twl, tid, W);
  if (act) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int x = seg + lane + 64 * e;
      row[e] = bufr[2 * lpad(x >> 1) + (x & 1)];
    }
  }
}

// Block sums of two per-thread values in a fixed order, returned to every thread.
__device__ __forceinline__ void block_sum2(double& a, double& b, bool act, int wv, int nw, int lane,
                                           double (*red)[kOneStepWavesMax]) {
  a = wave_sum(a);
  b = wave_sum(b);
  if (act && lane == 0) {
    red[0][wv] = a;
    red[1][wv] = b;
  }
  __syncthreads();
  // all reads issued before the additions (unrolled to the largest wave count)
  double ra[kOneStepWavesMax], rb[kOneStepWavesMax];
#pragma unroll
  for (int i = 0; i < kOneStepWavesMax; ++i) {
    ra[i] = i < nw ? red[0][i] : 0.0;
    rb[i] = i < nw ? red[1][i] : 0.0;
  }
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int i = 0; i < kOneStepWavesMax; ++i) {
    if (i < nw) {
      sa += ra[i];
      sb += rb[i];
    }
  }
  a = sa;
  b = sb;
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
  if (P.pcr_k[0] == 0)   // FFT path: twiddles e^{-2 pi i i' / M} in LDS
    for (int i = tid; i < M; i += blockDim.x) twl[lpad(i)] = P.tw[2 * i];
  // spectral pairs k = tid + j W < M/2 (and k = M/2, self-paired, on thread 0)
  constexpr int KP = EPT >= 4 ? EPT / 4 : 1;
  PairConsts<T, KP> pc;
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const int k = tid + j * W;
    pc.w[j] = (act && k < (M >> 1)) ? P.tw[k] : C2<T>{T(1), T(0)};
  }
  // cur = u^l, known = (c1 u^l + c2 u^{l-1}) / h_t at the first step; from u0 (also written to
  // level 0) when the march starts at step 0 with P.u0 given
  T cur[EPT], known[EPT];
  {
    const T c1 = C.c1(l_begin), c2 = C.c2(l_begin);
    const bool from_u0 = l_begin == 0 && P.u0 != nullptr;
    const T* ul = from_u0 ? P.u0 : P.u + (size_t)l_begin * nx;
    const T* ulm = ul - (l_begin >= 1 ? nx : 0);
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int x = seg + lane + 64 * e;
      cur[e] = act ? ul[x] : T(0);
      known[e] = act ? (c1 * cur[e] + c2 * ulm[x]) * C.inv_ht : T(0);
      if (act && from_u0) P.u[x] = cur[e];
    }
  }
  const double hx = sch.hx;
  for (int l = l_begin; l < l_end; ++l) {
    const T c0 = C.c0(l);
    const T a0 = c0 * C.inv_ht;
    load_pair_symbol(pc, P, c0 != T(1) ? 1 : 0, act, tid, W, M);
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
      // implicit residual A_l(v^n)
      T vm[1][EPT], vp[1][EPT];
      slice_neighbours<T, EPT, 1>(v, vm, vp, ends, act, wv, nw, lane);
      double srp = 0.0;
      T r[EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        r[e] = a0 * v[0][e] + known[e] + C.F(vm[0][e], v[0][e], vp[0][e]);
        if (act) srp += (double)r[e] * (double)r[e];
      }
      // s = K_l^{-1} r (in place), then the dual step and extrapolation: ph[0] = phi, ph[1] = phibar
      kinv_slice<T, EPT, KP>(r, pc, act, seg, lane, tid, W, M, buf, twl);
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        ph[1][e] = ph[0][e] + T(2) * tau_phi * r[e];
        ph[0][e] = ph[0][e] + tau_phi * r[e];
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
      block_sum2(srp, srd, act, wv, nw, lane, red);
      rp = sqrt(hx * srp);
      rd = sqrt(hx * srd);
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

// Largest eigenvalue of J_l(u0)^T K_l^{-1} J_l(u0) over the step operators of
// problem P (c0 = 1, and c0 = 3/2 for BDF2 with nt > 1) by `iters` power
// iterations from a fixed pseudo-random start; u0 is level 0 of P.u (or P.u0).
template <typename T, int EPT>
__device__ __forceinline__ double onestep_power(const OneStepProb<T>& P, int W, int iters, C2<T>* buf, C2<T>* twl,
                                                T (*ends)[2 * kOneStepWavesMax], double (*red)[kOneStepWavesMax]) {
  const Scheme& sch = P.s;
  const Consts<T> C(sch);
  const int nx = sch.nx, M = nx >> 1, tid = threadIdx.x;
  const bool act = tid < W;
  const int nw = W >> 6, wv = tid >> 6, lane = tid & 63;
  const int seg = wv * 64 * EPT;
  if (P.pcr_k[0] == 0)
    for (int i = tid; i < M; i += blockDim.x) twl[lpad(i)] = P.tw[2 * i];
  constexpr int KP = EPT >= 4 ? EPT / 4 : 1;
  PairConsts<T, KP> pc;
#pragma unroll
  for (int j = 0; j < KP; ++j) {
    const int k = tid + j * W;
    pc.w[j] = (act && k < (M >> 1)) ? P.tw[k] : C2<T>{T(1), T(0)};
  }
  const T* u0 = P.u0 ? P.u0 : P.u;
  T uu[1][EPT], um[1][EPT], up[1][EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) uu[0][e] = act ? u0[seg + lane + 64 * e] : T(0);
  slice_neighbours<T, EPT, 1>(uu, um, up, ends, act, wv, nw, lane);
  double nu = 0.0;
  const int nc0 = (sch.time == kTimeBDF2 && sch.nt > 1) ? 2 : 1;
  for (int ci = 0; ci < nc0; ++ci) {
    const T a0 = T(ci ? 1.5 : 1.0) * C.inv_ht;
    load_pair_symbol(pc, P, ci, act, tid, W, M);
    T v[1][EPT];
    double s2 = 0.0, dummy = 0.0;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {   // xorshift-hashed start in [-1/2, 1/2)
      unsigned long long h = 0x9E3779B97F4A7C15ull * (unsigned long long)(seg + lane + 64 * e + 1);
      h ^= h >> 31;
      h *= 0xBF58476D1CE4E5B9ull;
      h ^= h >> 27;
      v[0][e] = act ? T((double)(h >> 11) * (1.0 / 9007199254740992.0) - 0.5) : T(0);
      s2 += (double)v[0][e] * (double)v[0][e];
    }
    block_sum2(s2, dummy, act, wv, nw, lane, red);
    {
      const T sc = T(1.0 / sqrt(s2));
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[0][e] *= sc;
    }
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
      T vm[1][EPT], vp[1][EPT];
      slice_neighbours<T, EPT, 1>(v, vm, vp, ends + 1, act, wv, nw, lane);
      T w[1][EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e)   // J v = a0 v + dF(u0) v
        w[0][e] = a0 * v[0][e] + C.JF(um[0][e], uu[0][e], up[0][e], vm[0][e], v[0][e], vp[0][e]);
      kinv_slice<T, EPT, KP>(w[0], pc, act, seg, lane, tid, W, M, buf, twl);
      T wm[1][EPT], wp[1][EPT];
      slice_neighbours<T, EPT, 1>(w, wm, wp, ends + 2, act, wv, nw, lane);
      double tv = 0.0, tt = 0.0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {   // t = J^T w
        const T t = a0 * w[0][e] + C.JtF(uu[0][e], wm[0][e], w[0][e], wp[0][e]);
        if (act) {
          tv += (double)t * (double)v[0][e];
          tt += (double)t * (double)t;
        }
        w[0][e] = t;
      }
      block_sum2(tv, tt, act, wv, nw, lane, red);
      lam = tv;
      const T sc = T(1.0 / sqrt(tt));
#pragma unroll
      for (int e = 0; e < EPT; ++e) v[0][e] = w[0][e] * sc;
    }
    nu = fmax(nu, lam);
  }
  return nu;
}

// Block b estimates nu_max of problem probs[b] into nu[b]; where the problem's
// step sizes are not positive it sets both to sqrt(0.95 / nu_max) in the table.
template <typename T>
__global__ void __launch_bounds__(kOneStepThreadsMax)
k_onestep_power(OneStepProb<T>* __restrict__ probs, int iters, double* __restrict__ nu) {
  const OneStepProb<T> P = load_prob(probs);
  extern __shared__ char smem[];
  __shared__ T ends[3][2 * kOneStepWavesMax];
  __shared__ double red[2][kOneStepWavesMax];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(P.s.nx >> 1);
  const int W = onestep_threads<T>(P.s.nx);
  double v;
  switch (P.s.nx / W) {
    case 8: v = onestep_power<T, 8>(P, W, iters, buf, twl, ends, red); break;
    case 4: v = onestep_power<T, 4>(P, W, iters, buf, twl, ends, red); break;
    case 2: v = onestep_power<T, 2>(P, W, iters, buf, twl, ends, red); break;
    default: v = onestep_power<T, 1>(P, W, iters, buf, twl, ends, red); break;
  }
  if (threadIdx.x == 0) {
    nu[blockIdx.x] = v;
    if (!(P.tau_u > 0.0) || !(P.tau_phi > 0.0)) {
      const double t = (v > 0.0 && isfinite(v)) ? sqrt(0.95 / v) : 0.0;
      probs[blockIdx.x].tau_u = t;
      probs[blockIdx.x].tau_phi = t;
    }
  }
}

template <typename T>
hipError_t launch_onestep_power(OneStepProb<T>* probs, int nprob, int max_nx, int iters, double* nu, hipStream_t st) {
  if (max_nx < 64 || max_nx > 4096 || (max_nx & (max_nx - 1)) || nprob < 1) return hipErrorInvalidValue;
  const size_t lds = sizeof(C2<T>) * 2 * (size_t)lds_fft_points(max_nx / 2);
  hipError_t e = allow_lds(k_onestep_power<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_onestep_power<T>), dim3(nprob), dim3(onestep_threads<T>(max_nx)), lds, st, probs, iters, nu);
  return hipGetLastError();
}

template hipError_t launch_onestep_power<float>(OneStepProb<float>*, int, int, int, double*, hipStream_t);
template hipError_t launch_onestep_power<double>(OneStepProb<double>*, int, int, int, double*, hipStream_t);

// Block b marches problem probs[b] over steps [l_begin, min(l_end, nt)).
template <typename T>
__global__ void __launch_bounds__(kOneStepThreadsMax)
k_onestep(const OneStepProb<T>* __restrict__ probs, int l_begin, int l_end, double eps, long long max_iter,
          double dfac) {
  const OneStepProb<T> P = load_prob(probs);
  if (*P.flag != 0) return;   // this problem's march has stopped (diverged step)
  const int le = l_end < P.s.nt ? l_end : P.s.nt;
  if (l_begin >= le) return;
  extern __shared__ char smem[];
  __shared__ T ends[3][2 * kOneStepWavesMax];
  __shared__ double red[2][kOneStepWavesMax];
  const int M = P.s.nx >> 1;
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(M);
  const int W = onestep_threads<T>(P.s.nx);
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
  const int W = onestep_threads<T>(max_nx);
  const size_t lds = sizeof(C2<T>) * 2 * (size_t)lds_fft_points(max_nx / 2);
  hipError_t e = allow_lds(k_onestep<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_onestep<T>), dim3(nprob), dim3(W), lds, st, probs, l_begin, l_end, eps, max_iter, dfac);
  return hipGetLastError();
}

// ------------------------------------------------------------------ DG P1
// The one-level problem on the two nodal planes of the DG P1 scheme.  A step's
// preconditioner is (c0/h_t)^2 I + c^2 G G^T with G the unit-speed upwind P1
// operator: per Fourier mode m over the cells a Hermitian 2x2 matrix, whose
// inverse [a b; conj(b) d] (the inverse FFT's 1/N folded in) the host tables
// in P.sym as [2 rows c0 = 1, 3/2][N/2 + 1 modes][a, Re b, Im b, d].  The two
// real planes are one complex row Z = r_1 + i r_2 for the FFT.

// Spectral pair (m, q = N - m mod N): R_1 = (Z_m + conj Z_q)/2 and
// R_2 = (Z_m - conj Z_q)/(2i) are the planes' spectra at m; S = K^{-1} R, and
// Y_m = S_1 + i S_2, Y_q = conj(S_1) + i conj(S_2) (the planes are real).
template <typename T>
__device__ __forceinline__ void dg1_precond_pair(C2<T>* buf, int m, int q, T a, T br, T bi, T d) {
  const C2<T> zm = buf[lpad(m)], zq = buf[lpad(q)];
  const T r0x = T(0.5) * (zm.x + zq.x), r0y = T(0.5) * (zm.y - zq.y);
  const T r1x = T(0.5) * (zm.y + zq.y), r1y = T(-0.5) * (zm.x - zq.x);
  const T s0x = a * r0x + br * r1x - bi * r1y, s0y = a * r0y + br * r1y + bi * r1x;   // a R_1 + b R_2
  const T s1x = br * r0x + bi * r0y + d * r1x, s1y = br * r0y - bi * r0x + d * r1y;   // conj(b) R_1 + d R_2
  buf[lpad(m)] = C2<T>{s0x - s1y, s0y + s1x};
  if (q != m) buf[lpad(q)] = C2<T>{s0x + s1y, s1x - s0y};
}

// Steps [l_begin, l_end) of a DG P1 problem; cell x = seg + lane + 64 e, both planes per thread.
template <typename T, int EPT>
__device__ __forceinline__ void onestep_march_dg1(const OneStepProb<T>& P, int W, int l_begin, int l_end,
                                                  double eps, long long max_iter, double dfac, C2<T>* buf,
                                                  C2<T>* twl, T (*ends)[2 * kOneStepWavesMax],
                                                  double (*red)[kOneStepWavesMax]) {
  const Scheme& sch = P.s;
  const Consts<T> C(sch);
  const int nx = sch.nx, tid = threadIdx.x, half = nx >> 1;
  const bool act = tid < W;
  const int nw = W >> 6, wv = tid >> 6, lane = tid & 63;
  const int seg = wv * 64 * EPT;
  const T tau_u = (T)P.tau_u, tau_phi = (T)P.tau_phi;
  const size_t L2 = 2 * (size_t)nx;   // one level: two planes
  for (int i = tid; i < nx; i += blockDim.x) twl[lpad(i)] = P.tw[i];
  constexpr int KP = EPT / 2 + 1;     // modes m = tid + j W <= N/2
  T cur[2][EPT], known[2][EPT];
  {
    const T c1 = C.c1(l_begin), c2 = C.c2(l_begin);
    const bool from_u0 = l_begin == 0 && P.u0 != nullptr;
    const T* ul = from_u0 ? P.u0 : P.u + (size_t)l_begin * L2;
    const T* ulm = ul - (l_begin >= 1 ? L2 : 0);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int x = seg + lane + 64 * e;
        cur[k][e] = act ? ul[(size_t)k * nx + x] : T(0);
        known[k][e] = act ? (c1 * cur[k][e] + c2 * ulm[(size_t)k * nx + x]) * C.inv_ht : T(0);
        if (act && from_u0) P.u[(size_t)k * nx + x] = cur[k][e];
      }
  }
  const double hx = sch.hx;
  for (int l = l_begin; l < l_end; ++l) {
    const T c0 = C.c0(l);
    const T a0 = c0 * C.inv_ht;
    const T* kt = P.sym + (size_t)(c0 != T(1) ? 1 : 0) * (half + 1) * 4;
    T ka[KP], kbr[KP], kbi[KP], kd[KP];
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      const int m = tid + j * W;
      const bool ok = act && m <= half;
      ka[j] = ok ? kt[4 * m] : T(0);
      kbr[j] = ok ? kt[4 * m + 1] : T(0);
      kbi[j] = ok ? kt[4 * m + 2] : T(0);
      kd[j] = ok ? kt[4 * m + 3] : T(0);
    }
    // initial guess v = u^l, phi = phibar = 0
    T v[2][EPT], ph[2][2][EPT], g[2][EPT];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        v[k][e] = cur[k][e];
        ph[0][k][e] = ph[1][k][e] = g[k][e] = T(0);
      }
    double rp = 0.0, rd = 0.0, best = INFINITY;
    long long n = 0;
    int status = 1;
    while (n < max_iter) {
      ++n;
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int e = 0; e < EPT; ++e) v[k][e] -= tau_u * g[k][e];
      // implicit residual A_l(v): the upwind flux of cell x needs the right trace of cell x - 1
      T tr[1][EPT], trm[1][EPT], trp[1][EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const T vc[2] = {v[0][e], v[1][e]};
        tr[0][e] = P1Cell<T>::trace(vc);
      }
      slice_neighbours<T, EPT, 1>(tr, trm, trp, ends, act, wv, nw, lane);
      double srp = 0.0;
      T r[2][EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const T vc[2] = {v[0][e], v[1][e]};
        T F[2];
        dg1_spatial(C, vc, trm[0][e], F);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          r[k][e] = a0 * v[k][e] + known[k][e] + F[k];
          if (act) srp += (double)r[k][e] * (double)r[k][e];
        }
      }
      // s = K_l^{-1} r over both planes
      if (act) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) buf[lpad(seg + lane + 64 * e)] = C2<T>{r[0][e], r[1][e]};
      }
      fft_lds<false, EPT>(buf, nx, twl, tid, W);
      if (act) {
#pragma unroll
        for (int j = 0; j < KP; ++j) {
          const int m = tid + j * W;
          if (m <= half) dg1_precond_pair(buf, m, (nx - m) & (nx - 1), ka[j], kbr[j], kbi[j], kd[j]);
        }
      }
      fft_lds<true, EPT>(buf, nx, twl, tid, W);
      if (act) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const C2<T> y = buf[lpad(seg + lane + 64 * e)];
          r[0][e] = y.x;
          r[1][e] = y.y;
        }
      }
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          ph[1][k][e] = ph[0][k][e] + T(2) * tau_phi * r[k][e];
          ph[0][k][e] = ph[0][k][e] + tau_phi * r[k][e];
        }
      // J_l(v)^T phi (dual residual) and J_l(v)^T phibar (next primal step): psi of cell x + 1
      T pr[4][EPT], pl4[4][EPT], pn4[4][EPT];
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        pr[0][e] = ph[0][0][e];
        pr[1][e] = ph[0][1][e];
        pr[2][e] = ph[1][0][e];
        pr[3][e] = ph[1][1][e];
      }
      slice_neighbours<T, EPT, 4>(pr, pl4, pn4, ends + 1, act, wv, nw, lane);
      double srd = 0.0;
      if (act) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const T vc[2] = {v[0][e], v[1][e]};
          T o[2];
          const T p0[2] = {pr[0][e], pr[1][e]}, pn[2] = {pn4[0][e], pn4[1][e]};
          dg1_jt_cell(C, vc, p0, pn, o);
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            const T hk = a0 * ph[0][k][e] + o[k];
            srd += (double)hk * (double)hk;
          }
          const T q0[2] = {pr[2][e], pr[3][e]}, qn[2] = {pn4[2][e], pn4[3][e]};
          dg1_jt_cell(C, vc, q0, qn, o);
#pragma unroll
          for (int k = 0; k < 2; ++k) g[k][e] = a0 * ph[1][k][e] + o[k];
        }
      }
      block_sum2(srp, srd, act, wv, nw, lane, red);
      rp = sqrt(hx * srp);
      rd = sqrt(hx * srd);
      const double mm = fmax(rp, rd);
      if (!(isfinite(rp) && isfinite(rd)) || (mm > dfac * best)) {
        status = 2;
        break;
      }
      best = fmin(best, mm);
      if (mm <= eps) {
        status = 0;
        break;
      }
    }
    if (act) {
      T* un = P.u + (size_t)(l + 1) * L2;
      T* pl = P.phi + (size_t)l * L2;
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int x = seg + lane + 64 * e;
          un[(size_t)k * nx + x] = v[k][e];
          pl[(size_t)k * nx + x] = ph[0][k][e];
        }
    }
    if (tid == 0) {
      P.stat[l].iters = n;
      P.stat[l].rp = rp;
      P.stat[l].rd = rd;
      P.stat[l].status = status;
      if (status == 2) *P.flag = 2;
    }
    if (status == 2) return;
    const T c1n = C.c1(l + 1), c2n = C.c2(l + 1);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        known[k][e] = (c1n * v[k][e] + c2n * cur[k][e]) * C.inv_ht;
        cur[k][e] = v[k][e];
      }
  }
}

template <typename T>
__global__ void __launch_bounds__(kOneStepThreadsMax)
k_onestep_dg1(const OneStepProb<T>* __restrict__ probs, int l_begin, int l_end, double eps, long long max_iter,
              double dfac) {
  const OneStepProb<T> P = load_prob(probs);
  if (*P.flag != 0) return;
  const int le = l_end < P.s.nt ? l_end : P.s.nt;
  if (l_begin >= le) return;
  extern __shared__ char smem[];
  __shared__ T ends[5][2 * kOneStepWavesMax];
  __shared__ double red[2][kOneStepWavesMax];
  C2<T>* buf = reinterpret_cast<C2<T>*>(smem);
  C2<T>* twl = buf + lds_fft_points(P.s.nx);
  const int W = onestep_threads_dg1(P.s.nx);
  switch (P.s.nx / W) {
    case 8: onestep_march_dg1<T, 8>(P, W, l_begin, le, eps, max_iter, dfac, buf, twl, ends, red); break;
    case 4: onestep_march_dg1<T, 4>(P, W, l_begin, le, eps, max_iter, dfac, buf, twl, ends, red); break;
    case 2: onestep_march_dg1<T, 2>(P, W, l_begin, le, eps, max_iter, dfac, buf, twl, ends, red); break;
    default: onestep_march_dg1<T, 1>(P, W, l_begin, le, eps, max_iter, dfac, buf, twl, ends, red); break;
  }
}

template <typename T>
hipError_t launch_onestep_dg1(const OneStepProb<T>* probs, int nprob, int max_nx, int l_begin, int l_end,
                              double eps, long long max_iter, double dfac, hipStream_t st) {
  if (max_nx < 64 || max_nx > 4096 || (max_nx & (max_nx - 1)) || nprob < 1) return hipErrorInvalidValue;
  const int W = onestep_threads_dg1(max_nx);
  const size_t lds = sizeof(C2<T>) * 2 * (size_t)lds_fft_points(max_nx);
  hipError_t e = allow_lds(k_onestep_dg1<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_onestep_dg1<T>), dim3(nprob), dim3(W), lds, st, probs, l_begin, l_end, eps, max_iter,
                     dfac);
  return hipGetLastError();
}

template hipError_t launch_onestep_dg1<float>(const OneStepProb<float>*, int, int, int, int, double, long long,
                                              double, hipStream_t);
template hipError_t launch_onestep_dg1<double>(const OneStepProb<double>*, int, int, int, int, double, long long,
                                               double, hipStream_t);

template hipError_t launch_onestep<float>(const OneStepProb<float>*, int, int, int, int, double, long long, double,
                                          hipStream_t);
template hipError_t launch_onestep<double>(const OneStepProb<double>*, int, int, int, int, double, long long, double,
                                           hipStream_t);

}  // namespace pdhg
