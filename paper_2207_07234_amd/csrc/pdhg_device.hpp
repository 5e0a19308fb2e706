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
constexpr int kSpaceDgP2 = 2;
constexpr int kSpaceDgP1 = 3;

// A device pointer read from a table in memory (rather than passed as a kernel
// argument) is generic to the compiler, and every access through it becomes a
// flat instruction, which counts against both the vector-memory and the LDS
// wait counters.  Re-typing it through an integer as a global pointer lets the
// address-space inference turn its accesses into global loads and stores.
// Only for pointers into device (HBM) allocations.
template <typename P>
__device__ __forceinline__ P* as_global(P* p) {
  using G = __attribute__((address_space(1))) char*;
  return (P*)(reinterpret_cast<G>(reinterpret_cast<uintptr_t>(p)));
}

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

// LDS layout of an N-point complex FFT buffer: point x is stored at
// x ^ ((x >> 4) & 15), a permutation inside each block of 16 points.  Reads of
// consecutive points stay conflict-free, and the strided Stockham writes and
// twiddle reads of consecutive lanes spread over the banks (fewer conflicts
// than a padded layout, measured on a bank model of the whole FFT, and no
// extra space).  lds_fft_points(N) slots are needed.
__device__ __forceinline__ int lpad(int x) { return x ^ ((x >> 4) & 15); }
__host__ __device__ constexpr int lds_fft_points(int n) { return n; }

// Copy the twiddle table w_N^i, i = 0..N-1, from global memory into LDS (padded).
template <typename T>
__device__ __forceinline__ void load_twiddles_lds(C2<T>* twl, const C2<T>* __restrict__ tw, int N, int tid,
                                                  int W) {
  for (int i = tid; i < N; i += W) twl[lpad(i)] = tw[i];
}

// One Stockham radix-R stage on LDS arrays of N points: every thread loads all
// inputs of its butterflies from src, and stores the outputs to dst.  In place
// (dst == src) the block synchronises between the loads and the stores.
// Butterfly j (0 <= j < N/R) reads x[j + r N/R], twiddles input r by
// w_N^{r k N/(Ns R)} with k = j mod Ns, and writes output q to
// x[(j - k) R + k + q Ns].  EPT bounds N / W (points per thread).
template <bool INV, int R, int EPT, typename T>
__device__ __forceinline__ void stockham_stage(const C2<T>* src, C2<T>* dst, int N, int Ns,
                                               const C2<T>* __restrict__ twl, int tid, int W) {
  constexpr int MAXB = (EPT + R - 1) / R;  // butterflies per thread
  const int nbf = N / R;
  const int tstride = N / (Ns * R);
  // inputs and twiddles of all butterflies are read before any is used, so that
  // their LDS latencies overlap
  C2<T> v[MAXB * R], w[MAXB * R];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = tid + b * W;
    if (tid < W && j < nbf) {
      const int k = j & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) v[b * R + r] = src[lpad(j + r * nbf)];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) w[b * R + r] = twl[lpad(r * k * tstride)];
      }
    }
  }
  if (dst == src) __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = tid + b * W;
    if (tid < W && j < nbf) {
      const int k = j & (Ns - 1);
      C2<T>* vb = v + b * R;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) vb[r] = cmul_tw<INV>(vb[r], w[b * R + r]);
      }
      if (R == 8) dft8<INV>(vb);
      else if (R == 4) dft4<INV>(vb);
      else dft2<INV>(vb);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) dst[lpad(base + q * Ns)] = vb[q];
    }
  }
  __syncthreads();
}

// Unnormalised DFT of the N points in buf (natural order in and out, padded
// layout): X_k = sum_x z_x e^{-2 pi i x k / N} (forward) or e^{+...} (inverse).
// twl: LDS twiddle table from load_twiddles_lds.  Requires N = 2^m, 2 <= N <=
// EPT W, and every thread of the block to call it; threads tid = 0..W-1 do the
// work, any others take part in the barriers only.  With a second LDS array
// alt of N points the stages alternate between buf and alt (one barrier per
// stage instead of two); the returned pointer (buf or alt) holds the result.
template <bool INV, int EPT, typename T>
__device__ __forceinline__ C2<T>* fft_lds(C2<T>* buf, int N, const C2<T>* __restrict__ twl, int tid, int W,
                          C2<T>* alt = nullptr) {
  __syncthreads();
  C2<T>* src = buf;
  C2<T>* dst = alt ? alt : buf;
  int Ns = 1;
  while (Ns < N) {
    const int rem = N / Ns;
    if (rem >= 8) {
      stockham_stage<INV, 8, EPT>(src, dst, N, Ns, twl, tid, W);
      Ns *= 8;
    } else if (rem == 4) {
      stockham_stage<INV, 4, EPT>(src, dst, N, Ns, twl, tid, W);
      Ns *= 4;
    } else {
      stockham_stage<INV, 2, EPT>(src, dst, N, Ns, twl, tid, W);
      Ns *= 2;
    }
    if (alt) {
      C2<T>* t = src;
      src = dst;
      dst = t;
    }
  }
  return src;
}

// ------------------------------------------------------------------ XCD-aware block order
// The dispatcher hands consecutive workgroups to the 8 XCDs of an MI355X in
// turn, and each XCD has its own L2.  Blocks that share halo data (neighbouring
// time rows, the two halves of a spectrum column block) should sit on the same
// XCD: logical block L = (b mod 8) (n / 8) + b / 8 gives XCD x the contiguous
// range [x n/8, (x+1) n/8).  Identity when n is not a multiple of 8.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_block(int b, int n) {
  if (n % kNumXcd != 0) return b;
  return (b % kNumXcd) * (n / kNumXcd) + b / kNumXcd;
}

// ------------------------------------------------------------------ cross-lane moves
// DPP wavefront shifts (all 64 lanes active): from_lane_below(v, fill) gives
// lane l the value of lane l-1 and lane 0 `fill`; from_lane_above gives lane l
// the value of lane l+1 and lane 63 `fill`.
__device__ __forceinline__ int dpp_below_i(int v, int fill) { return __builtin_amdgcn_update_dpp(fill, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_above_i(int v, int fill) { return __builtin_amdgcn_update_dpp(fill, v, 0x130, 0xf, 0xf, false); }

__device__ __forceinline__ float from_lane_below(float v, float fill) {
  return __int_as_float(dpp_below_i(__float_as_int(v), __float_as_int(fill)));
}
__device__ __forceinline__ float from_lane_above(float v, float fill) {
  return __int_as_float(dpp_above_i(__float_as_int(v), __float_as_int(fill)));
}
__device__ __forceinline__ double from_lane_below(double v, double fill) {
  const long long a = __double_as_longlong(v), f = __double_as_longlong(fill);
  const int lo = dpp_below_i((int)(a & 0xffffffffll), (int)(f & 0xffffffffll));
  const int hi = dpp_below_i((int)(a >> 32), (int)(f >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_lane_above(double v, double fill) {
  const long long a = __double_as_longlong(v), f = __double_as_longlong(fill);
  const int lo = dpp_above_i((int)(a & 0xffffffffll), (int)(f & 0xffffffffll));
  const int hi = dpp_above_i((int)(a >> 32), (int)(f >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Generic DPP move with control word CTRL (all rows and banks enabled): lanes
// whose source lane is invalid for CTRL receive `fill`.  Row shifts within rows
// of 16 lanes: row_shr:n = 0x110 + n (from lane l - n), row_shl:n = 0x100 + n
// (from lane l + n).
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v, float fill) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v, double fill) {
  const long long a = __double_as_longlong(v), f = __double_as_longlong(fill);
  const int lo = __builtin_amdgcn_update_dpp((int)(f & 0xffffffffll), (int)(a & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(f >> 32), (int)(a >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Value of v in lane `src` (uniform result).
__device__ __forceinline__ float read_lane(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double read_lane(double v, int src) {
  const long long a = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(a & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(a >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Periodic x-neighbours of a row held by a wavefront in "lane-cyclic" order:
// element e of lane l is x = seg0 + l + 64 e, e = 0..E-1, so x-1 and x+1 are
// the neighbouring lanes, with wrap-around between consecutive e.  prev_last
// and next_first are the row values just before and after the wave's segment.
template <typename T, int E>
__device__ __forceinline__ void wave_row_neighbours(const T* v, T prev_last, T next_first, T* vm, T* vp) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const T lo = (e == 0) ? prev_last : read_lane(v[e - 1], 63);
    const T hi = (e == E - 1) ? next_first : read_lane(v[e + 1], 0);
    vm[e] = from_lane_below(v[e], lo);
    vp[e] = from_lane_above(v[e], hi);
  }
}

// ------------------------------------------------------------------ reductions
// Sum over the 64 lanes of a wavefront (all lanes active), the same value in
// every lane: an inclusive scan inside each row of 16 lanes by DPP row shifts
// (no LDS), then the four row totals (lanes 15, 31, 47, 63) added in a fixed
// order.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0x111>(v, 0.0);   // row_shr:1
  v += dpp_move<0x112>(v, 0.0);   // row_shr:2
  v += dpp_move<0x114>(v, 0.0);   // row_shr:4
  v += dpp_move<0x118>(v, 0.0);   // row_shr:8
  return (read_lane(v, 15) + read_lane(v, 31)) + (read_lane(v, 47) + read_lane(v, 63));
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

// Sum over a block whose size is a multiple of 64: wave reductions, then one
// thread adds the per-wave sums.  Result valid in thread 0.  Fixed order.
__device__ __forceinline__ double block_sum_waves(double v, double* red /* >= blockDim.x/64 doubles */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    // reads issued together (unrolled to 16 waves), added in wave order
    double r[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) r[i] = i < nw ? red[i] : 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i < nw) s += r[i];
  }
  return s;
}

// Sum over a block of any power-of-two size (blockDim.x <= 1024) by a tree in
// LDS; result valid in thread 0.  Fixed order.
__device__ __forceinline__ double block_sum_tree(double v, double* red /* >= blockDim.x doubles */) {
  const int tid = threadIdx.x, n = blockDim.x;
  __syncthreads();
  red[tid] = v;
  __syncthreads();
  for (int s = n >> 1; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  return red[0];
}

// Spectrum layout: halfcomplex column q of row l, stored in column blocks of
// QB = 2^lqb columns: element (l, q) at ((q >> lqb) * nt + l) * QB + (q & (QB-1)).
// Column 0 holds Re X_0, column 1 Re X_{N/2}, columns 2k and 2k+1 Re and Im X_k.
__device__ __forceinline__ size_t spec_index(int l, int q, int nt, int lqb) {
  return ((size_t)(q >> lqb) * nt + l) * ((size_t)1 << lqb) + (q & ((1 << lqb) - 1));
}

// Halfcomplex spectra of two real rows a, b from Z = DFT(a + i b) in buf:
// A_k = (Z_k + conj Z_{N-k})/2, B_k = (Z_k - conj Z_{N-k})/(2i), k = 0..N/2.
// Row b is skipped when !hasb.
template <typename T>
__device__ __forceinline__ void store_halfcomplex_pair(const C2<T>* buf, int nx, T* __restrict__ spec, int nt,
                                                       int lqb, int a, bool hasb, int tid, int W) {
  const int half = nx >> 1;
  const int b = a + 1;
  for (int k = tid; k <= half; k += W) {
    const C2<T> zk = buf[lpad(k)], zm = buf[lpad((nx - k) & (nx - 1))];
    const T ar = T(0.5) * (zk.x + zm.x), ai = T(0.5) * (zk.y - zm.y);
    const T br = T(0.5) * (zk.y + zm.y), bi = T(0.5) * (zm.x - zk.x);
    if (k == 0 || k == half) {
      const int q = (k == 0) ? 0 : 1;
      spec[spec_index(a, q, nt, lqb)] = ar;
      if (hasb) spec[spec_index(b, q, nt, lqb)] = br;
    } else {
      spec[spec_index(a, 2 * k, nt, lqb)] = ar;
      spec[spec_index(a, 2 * k + 1, nt, lqb)] = ai;
      if (hasb) {
        spec[spec_index(b, 2 * k, nt, lqb)] = br;
        spec[spec_index(b, 2 * k + 1, nt, lqb)] = bi;
      }
    }
  }
}

// Z_k = A_k + i B_k for k = 0..N-1 in buf from the halfcomplex spectra of rows
// a and b (B = 0 when !hasb), using A_{N-k} = conj A_k.
template <typename T>
__device__ __forceinline__ void load_halfcomplex_pair(C2<T>* buf, int nx, const T* __restrict__ spec, int nt,
                                                      int lqb, int a, bool hasb, int tid, int W) {
  const int half = nx >> 1;
  const int b = a + 1;
  for (int k = tid; k <= half; k += W) {
    T ar, ai = T(0), br = T(0), bi = T(0);
    if (k == 0 || k == half) {
      const int q = (k == 0) ? 0 : 1;
      ar = spec[spec_index(a, q, nt, lqb)];
      if (hasb) br = spec[spec_index(b, q, nt, lqb)];
    } else {
      ar = spec[spec_index(a, 2 * k, nt, lqb)];
      ai = spec[spec_index(a, 2 * k + 1, nt, lqb)];
      if (hasb) {
        br = spec[spec_index(b, 2 * k, nt, lqb)];
        bi = spec[spec_index(b, 2 * k + 1, nt, lqb)];
      }
    }
    buf[lpad(k)] = {ar - bi, ai + br};
    if (k != 0 && k != half) buf[lpad(nx - k)] = {ar + bi, br - ai};
  }
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

// Chunked column solve: chunks of kChunkLevels levels of kChunkCols spectrum
// columns (one column block), kChunkCw lanes per column, kChunkLpl levels per lane.
constexpr int kChunkLpl = 8;
constexpr int kChunkCw = 32;
constexpr int kChunkLevels = kChunkLpl * kChunkCw;
constexpr int kChunkCols = 16;
constexpr int kChunkThreads = kChunkCw * kChunkCols;
constexpr int kChunkMinNt = 4097;   // N_t from which the fused solve uses the chunked column solve
__host__ __device__ constexpr int chunk_count(int nt) { return (nt + kChunkLevels - 1) / kChunkLevels; }

// Arguments of the chunked column solve of long time axes (N_t > 4096,
// N_x >= 16).  Column blocks g < g64 (and every block where f32.rows is null)
// run their recurrences in FP64 on f64, the others in float on f32; the maps
// and the chunk states are FP64.
// Past a mode's last distinct factor row every lane of a chunk sees the same
// rows, so each lane's homogeneous segment map (kChunkLpl levels, the same
// both ways) is one 2x2 matrix M per mode; the scans of such chunks use the
// powers M^(2^s), s < kChunkPow.
constexpr int kChunkPow = 4;
struct ChunkArgs {
  FacTab<double> f64;
  FacTab<float> f32;
  const double* cmap;   // [N_x/2 + 1][nchunk][12]: H, G, K of every mode and chunk
  const double* cpow;   // [N_x/2 + 1][kChunkPow][4]: M, M^2, M^4, M^8 of every mode (below)
  double* cwork;        // [2][nchunk][N_x][4]: pass-1 records (P, R), entering states (t, h)
  // tiles (g nchunk + c) of the four grids of either pass, in this order: FP64 recurrences with general
  // rows, FP64 with constant rows, float general, float constant (constant: for every column of the tile
  // the chunk is full and lies past the last distinct row of the table it uses); tile[k] starts at
  // tiles + toff[k] and holds ntile[k] entries
  const int* tiles;
  int toff[4];
  int ntile[4];
  int nchunk;
  int g64;
};

// Multiplier form of Algorithm 1 (Section 3.3): the initial level u^0 is an
// unknown, and lambda (nx values) imposes u^0 = u0.  u0 == nullptr: u^0 is held
// fixed.  The pass that holds rows 0 and 1 updates u^0 and lambda (no other
// pair reads u^0): u^0 <- u^0 - tau_u0 (h_t J_0^T phibar + lambdabar) with
// h_t J_0^T phibar = c1(0) phibar^0 + c2(1) phibar^1, then
// lambda <- lambda + tau_lam (u^0 - u0), lambdabar = 2 lambda_new - lambda_old.
template <typename T>
struct LamArgs {
  const T* u0;
  T* lam;
  T* lambar;
  T tau_u0, tau_lam;
};

// Device-side control block of one solve.
struct Ctrl {
  long long n_done;    // loop bodies completed
  long long max_iter;
  long long n_star;    // returned iterate
  int status;          // 0 running, 1 converged, 2 diverged, 3 max_iter reached, 4 stalled
  int rd_lazy;         // 1: the fused row pass evaluates Rd only where rd_needed says so
  double eps, div_factor;
  double rp_prev;      // ||A(u^{n_done})||
  double best;         // min over checked iterates of ||A(u)||
  double rp_star, rd_star;
  long long best_at;   // iterate at which best was reached
  long long stall;     // > 0: stop (status 4) when best is that many iterates old
  long long ck_iter;   // iterate held by the last-good checkpoint (-1: none)
};

// Whether loop body n = n_done + 1 must evaluate Rd(n-1) = ||J(u^{n-1})^T phi^{n-1}||.
// The stopping test needs it only where Rp(n-1) <= eps (both entries must be
// below eps), and the stats report it for the last iterate (n-1 = max_iter);
// divergence is judged on Rp alone.  Without rd_lazy it is always evaluated
// (the residual history records every Rd).
__device__ __forceinline__ bool rd_needed(const Ctrl* c) {
  return !c->rd_lazy || c->rp_prev <= c->eps || c->n_done >= c->max_iter;
}

// End of loop body n = n_done + 1: Rp(n) and Rd(n-1) from the partial sums;
// decide whether iterate n-1 is converged, diverged or the last one.  Where
// Rd(n-1) was not evaluated (rd_needed false) srd is 0 and Rd reads as NaN.
__device__ inline void finalize_body(Ctrl* c, double srp, double srd, double wscale, double* hist) {
  const bool have_rd = rd_needed(c);
  const long long n = c->n_done + 1;
  const double rp = sqrt(wscale * srp);
  const double rd = have_rd ? sqrt(wscale * srd) : __builtin_nan("");
  const long long it = n - 1;
  if (hist) {
    hist[2 * n] = rp;
    hist[2 * it + 1] = rd;
    if (n == 1) hist[0] = __builtin_nan("");
  }
  int st = 0;
  if (it >= 1) {
    const double p = c->rp_prev;
    if (!(p == p) || isinf(p)) st = 2;
    else if (p <= c->eps && rd <= c->eps) st = 1;
    else if (p > c->div_factor * c->best) st = 2;
    if (p < c->best) {
      c->best = p;
      c->best_at = it;
    }
    if (st == 0 && c->stall > 0 && it - c->best_at >= c->stall) st = 4;   // rounding floor reached
    if (st == 0 && it >= c->max_iter) st = 3;
  }
  if (st == 0 && !(rp == rp && !isinf(rp) && (!have_rd || (rd == rd && !isinf(rd))))) st = 2;
  if (st != 0) {
    c->status = st;
    c->n_star = it;
    c->rp_star = (it >= 1) ? c->rp_prev : __builtin_nan("");
    c->rd_star = rd;
  }
  c->rp_prev = rp;
  c->n_done = n;
}

}  // namespace pdhg
