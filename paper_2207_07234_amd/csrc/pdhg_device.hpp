// Device building blocks of the space-time primal-dual solver (gfx950).
//
// * Scheme / Consts: grid, flux and time-scheme constants of one problem.
// * Point formulas of the implicit residual A(u) (Section 3.1-3.2), of the
//   dual-equation operator J(u)^T phi obtained by summation by parts
//   (Section 3.1) and of J(u) v (for the step-size power iteration).
// * An in-LDS Stockham FFT (radix 8/4/2) used by the preconditioner
//   K_d^{-1} (Section 2.2: the dual step is solved with the FFT in x).
// * Deterministic block reductions in double precision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdhg {

constexpr int kTimeBE = 0;
constexpr int kTimeBDF2 = 1;
constexpr int kSpaceUpwind = 0;
constexpr int kSpaceLF = 1;

// Host-filled description of one problem (all in double; kernels convert).
struct Scheme {
  int nx, nt;
  int time, space;
  double ht, hx;
  double alpha, beta, gamma, lf;
};

// Per-kernel constants in the compute type T.
template <typename T>
struct Consts {
  T inv_ht, inv_hx, inv_2hx, inv_hx2, alpha2, alpha, beta, gamma, lf;
  int nx, nt, time, space;
  __device__ __forceinline__ explicit Consts(const Scheme& s)
      : inv_ht(T(1.0 / s.ht)), inv_hx(T(1.0 / s.hx)), inv_2hx(T(0.5 / s.hx)),
        inv_hx2(T(1.0 / (s.hx * s.hx))), alpha2(T(2.0 * s.alpha)), alpha(T(s.alpha)),
        beta(T(s.beta)), gamma(T(s.gamma)), lf(T(s.lf)), nx(s.nx), nt(s.nt), time(s.time),
        space(s.space) {}

  __device__ __forceinline__ T flux(T u) const { return (alpha * u + beta) * u; }
  __device__ __forceinline__ T dflux(T u) const { return alpha2 * u + beta; }

  // Coefficients (c0, c1, c2) of row l: (c0 u^{l+1} + c1 u^l + c2 u^{l-1}) / h_t.
  // BDF2 uses backward Euler on row 0.
  __device__ __forceinline__ T c0(int l) const { return (time == kTimeBDF2 && l >= 1) ? T(1.5) : T(1); }
  __device__ __forceinline__ T c1(int l) const { return (time == kTimeBDF2 && l >= 1) ? T(-2) : T(-1); }
  __device__ __forceinline__ T c2(int l) const { return (time == kTimeBDF2 && l >= 1) ? T(0.5) : T(0); }

  // Spatial operator F(v) at a point from v_{k-1}, v_k, v_{k+1}.
  __device__ __forceinline__ T F(T vm, T v0, T vp) const {
    T out;
    if (space == kSpaceUpwind) {
      out = (flux(v0) - flux(vm)) * inv_hx;
    } else {
      out = (T(0.5) * (flux(vp) - flux(vm)) - T(0.5) * lf * (vp - T(2) * v0 + vm)) * inv_hx;
    }
    if (gamma != T(0)) out -= gamma * (vp - T(2) * v0 + vm) * inv_hx2;
    return out;
  }

  // (dF(u)^T psi) at point k from u_k and psi_{k-1}, psi_k, psi_{k+1}.
  __device__ __forceinline__ T JtF(T u0, T pm, T p0, T pp) const {
    const T fp = dflux(u0);
    T out;
    if (space == kSpaceUpwind) {
      out = fp * (p0 - pp) * inv_hx;
    } else {
      out = (fp * (pm - pp) + lf * (T(2) * p0 - pm - pp)) * inv_2hx;
    }
    if (gamma != T(0)) out += gamma * (T(2) * p0 - pm - pp) * inv_hx2;
    return out;
  }

  // Stencil of (dF(u)^T psi)_k = lo psi_{k-1} + di psi_k + up psi_{k+1} at u_k.
  __device__ __forceinline__ void JtF_coeffs(T u0, T& lo, T& di, T& up) const {
    const T fp = dflux(u0);
    if (space == kSpaceUpwind) {
      lo = T(0);
      di = fp * inv_hx;
      up = -fp * inv_hx;
    } else {
      lo = (fp - lf) * inv_2hx;
      di = lf * inv_hx;
      up = (-fp - lf) * inv_2hx;
    }
    if (gamma != T(0)) {
      lo -= gamma * inv_hx2;
      di += T(2) * gamma * inv_hx2;
      up -= gamma * inv_hx2;
    }
  }

  // (dF(u) v) at point k from u_{k-1..k+1}, v_{k-1..k+1}.
  __device__ __forceinline__ T JF(T um, T u0, T up, T vm, T v0, T vp) const {
    T out;
    if (space == kSpaceUpwind) {
      out = (dflux(u0) * v0 - dflux(um) * vm) * inv_hx;
    } else {
      out = (T(0.5) * (dflux(up) * vp - dflux(um) * vm) - T(0.5) * lf * (vp - T(2) * v0 + vm)) * inv_hx;
    }
    if (gamma != T(0)) out -= gamma * (vp - T(2) * v0 + vm) * inv_hx2;
    return out;
  }

  // Time part of (J^T psi) at unknown level m (1..nt) from psi^{m-1}, psi^m, psi^{m+1}
  // (psi rows beyond nt-1 are zero; the caller passes 0 for them).
  __device__ __forceinline__ T JtTime(int m, T pm1, T p0, T pp1) const {
    return (c0(m - 1) * pm1 + c1(m) * p0 + c2(m + 1) * pp1) * inv_ht;
  }
};

// ------------------------------------------------------------------ complex
template <typename T>
struct C2 {
  T x, y;
};
template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <bool INV, typename T>
__device__ __forceinline__ C2<T> cmul_tw(C2<T> a, C2<T> w) {
  // a * w (forward) or a * conj(w) (inverse)
  if (INV) return {a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
  return {a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x};
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename T>
__device__ __forceinline__ C2<T> mul_mi(C2<T> a) {
  if (INV) return {-a.y, a.x};
  return {a.y, -a.x};
}

template <bool INV, typename T>
__device__ __forceinline__ void dft2(C2<T>* v) {
  C2<T> a = v[0];
  v[0] = cadd(a, v[1]);
  v[1] = csub(a, v[1]);
}

template <bool INV, typename T>
__device__ __forceinline__ void dft4(C2<T>* v) {
  C2<T> e0 = cadd(v[0], v[2]), e1 = csub(v[0], v[2]);
  C2<T> o0 = cadd(v[1], v[3]), o1 = mul_mi<INV>(csub(v[1], v[3]));
  v[0] = cadd(e0, o0);
  v[2] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[3] = csub(e1, o1);
}

template <bool INV, typename T>
__device__ __forceinline__ void dft8(C2<T>* v) {
  C2<T> e[4] = {v[0], v[2], v[4], v[6]};
  C2<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  const T h = T(0.70710678118654752440084436210485);
  if (INV) {
    o[1] = {h * (o[1].x - o[1].y), h * (o[1].x + o[1].y)};
    o[3] = {-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)};
  } else {
    o[1] = {h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
    o[3] = {h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
  }
  o[2] = mul_mi<INV>(o[2]);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[q] = cadd(e[q], o[q]);
    v[q + 4] = csub(e[q], o[q]);
  }
}

// One Stockham radix-R stage on an LDS array of N points, in place: every
// thread loads all inputs of its butterflies, the block synchronises, then
// the outputs are stored.  Butterfly j (0 <= j < N/R) reads x[j + r N/R],
// twiddles input r by w_N^{r k N/(Ns R)} with k = j mod Ns, and writes
// output q to x[(j - k) R + k + q Ns].
template <bool INV, int R, int W, typename T>
__device__ __forceinline__ void stockham_stage(C2<T>* buf, int N, int Ns, const C2<T>* __restrict__ tw,
                                               int tid) {
  constexpr int MAXB = 16 / R;  // butterflies per thread (N <= 16 W)
  const int nbf = N / R;
  C2<T> v[MAXB * R];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = tid + b * W;
    if (j < nbf) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b * R + r] = buf[j + r * nbf];
    }
  }
  __syncthreads();
  const int tstride = N / (Ns * R);
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = tid + b * W;
    if (j < nbf) {
      const int k = j & (Ns - 1);
      C2<T>* vb = v + b * R;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) vb[r] = cmul_tw<INV>(vb[r], tw[r * k * tstride]);
      }
      if (R == 8) dft8<INV>(vb);
      else if (R == 4) dft4<INV>(vb);
      else dft2<INV>(vb);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) buf[base + q * Ns] = vb[q];
    }
  }
  __syncthreads();
}

// Unnormalised DFT of the N points in buf (natural order in and out):
// X_k = sum_x z_x e^{-2 pi i x k / N} (forward) or e^{+...} (inverse).
// tw[i] = e^{-2 pi i i / N}.  Requires N = 2^m, 2 <= N <= 16 W, and all W
// threads of the block to call it.
template <bool INV, int W, typename T>
__device__ void fft_lds(C2<T>* buf, int N, const C2<T>* __restrict__ tw, int tid) {
  __syncthreads();
  int Ns = 1;
  while (Ns < N) {
    const int rem = N / Ns;
    if (rem >= 8) {
      stockham_stage<INV, 8, W>(buf, N, Ns, tw, tid);
      Ns *= 8;
    } else if (rem == 4) {
      stockham_stage<INV, 4, W>(buf, N, Ns, tw, tid);
      Ns *= 4;
    } else {
      stockham_stage<INV, 2, W>(buf, N, Ns, tw, tid);
      Ns *= 2;
    }
  }
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over the block (W threads); result valid in thread 0.  Fixed order.
template <int W>
__device__ __forceinline__ double block_sum(double v, double* red /* >= W/64 doubles of LDS */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < W / 64; ++i) s += red[i];
  }
  return s;
}

// Spectrum layout: halfcomplex column q of row l, stored in column blocks of
// QB = 2^lqb columns: element (l, q) at ((q >> lqb) * nt + l) * QB + (q & (QB-1)).
// Column 0 holds Re X_0, column 1 Re X_{N/2}, columns 2k and 2k+1 Re and Im X_k.
__device__ __forceinline__ size_t spec_index(int l, int q, int nt, int lqb) {
  return ((size_t)(q >> lqb) * nt + l) * ((size_t)1 << lqb) + (q & ((1 << lqb) - 1));
}

// Fourier mode of halfcomplex column q.
__device__ __forceinline__ int spec_mode(int q, int nx) { return q == 0 ? 0 : (q == 1 ? nx / 2 : q >> 1); }

// Row of the banded Cholesky factor L of (B_t B_t^T + s_k I): inverse diagonal
// and the two sub-diagonal entries L_{l,l-1}, L_{l,l-2}.
template <typename T>
struct FacRow {
  T invd, e1, e2, pad;
};

// Factor tables of all modes: rows[off[k] + min(l, last[k])].
template <typename T>
struct FacTab {
  const FacRow<T>* rows;
  const int* off;
  const int* last;
};

// Device-side control block of one solve.
struct Ctrl {
  long long n_done;    // loop bodies completed
  long long max_iter;
  long long n_star;    // returned iterate
  int status;          // 0 running, 1 converged, 2 diverged, 3 max_iter reached
  int pad;
  double eps, div_factor;
  double rp_prev;      // ||A(u^{n_done})||
  double best;         // min over checked iterates of max(Rp, Rd)
  double rp_star, rd_star;
};

}  // namespace pdhg
