// DG P1 nodal upwind cell operators (Sections 3.2.2-3.2.3), shared by the
// space-time passes and the one-time-step march.  Cell j holds u_h by its
// values at xi = -1/2 and +1/2 (basis phi_1 = 1/2 - xi, phi_2 = 1/2 + xi,
// xi = 2 (x - x_c) / h); the right trace is a_j = -v_j1/2 + 3 v_j2/2.
#pragma once

#include "pdhg_device.hpp"

namespace pdhg {

template <typename T>
struct P1Cell {
  static __device__ __forceinline__ T g1() { return T(0.5 + 0.57735026918962576450914878); }
  static __device__ __forceinline__ T g2() { return T(0.5 - 0.57735026918962576450914878); }
  static __device__ __forceinline__ T trace(const T* v) { return T(-0.5) * v[0] + T(1.5) * v[1]; }
  // M^{-1} r for M = h [7 -1; -1 7] / 12: (7 r1 + r2, r1 + 7 r2) / (4 h)
  static __device__ __forceinline__ void minv(const Consts<T>& C, T r1, T r2, T* out) {
    out[0] = T(0.25) * C.inv_hx * (T(7) * r1 + r2);
    out[1] = T(0.25) * C.inv_hx * (r1 + T(7) * r2);
  }
};

template <typename T>
__device__ __forceinline__ void load_cell2(const T* __restrict__ row2, int nx, int j, T* v) {
  v[0] = row2[j];
  v[1] = row2[nx + j];
}

// F_j from the cell's nodal values and the left neighbour's right trace.
template <typename T>
__device__ __forceinline__ void dg1_spatial(const Consts<T>& C, const T* v, T a_left, T* F) {
  const T g1 = P1Cell<T>::g1(), g2 = P1Cell<T>::g2();
  const T S = C.flux(g1 * v[0] + g2 * v[1]) + C.flux(g2 * v[0] + g1 * v[1]);
  const T fr = C.flux(P1Cell<T>::trace(v)), fl = C.flux(a_left);
  const T r1 = -S + T(0.5) * fr + T(1.5) * fl;
  const T r2 = S - T(1.5) * fr - T(0.5) * fl;
  T m[2];
  P1Cell<T>::minv(C, r1, r2, m);
  F[0] = -m[0];
  F[1] = -m[1];
}

// (dF^T psi)_j from the cell's u values and psi at cells j, j+1.
template <typename T>
__device__ __forceinline__ void dg1_jt_cell(const Consts<T>& C, const T* v, const T* p0, const T* pp, T* out) {
  const T g1 = P1Cell<T>::g1(), g2 = P1Cell<T>::g2();
  const T d0 = C.dflux(g1 * v[0] + g2 * v[1]), d1 = C.dflux(g2 * v[0] + g1 * v[1]);
  const T da = C.dflux(P1Cell<T>::trace(v));
  T m0[2], mp[2];
  P1Cell<T>::minv(C, p0[0], p0[1], m0);
  P1Cell<T>::minv(C, pp[0], pp[1], mp);
  const T dm = m0[1] - m0[0];
  const T X = (T(-0.5) * m0[0] + T(1.5) * m0[1]) - (T(1.5) * mp[0] - T(0.5) * mp[1]);
  out[0] = -dm * (d0 * g1 + d1 * g2) - T(0.5) * da * X;
  out[1] = -dm * (d0 * g2 + d1 * g1) + T(1.5) * da * X;
}

// (dF v)_j from the u values of cells j-1, j and v at cells j-1, j.
template <typename T>
__device__ __forceinline__ void dg1_j_cell(const Consts<T>& C, const T* um, const T* uc, const T* vm, const T* v0,
                                           T* out) {
  const T g1 = P1Cell<T>::g1(), g2 = P1Cell<T>::g2();
  const T d0 = C.dflux(g1 * uc[0] + g2 * uc[1]), d1 = C.dflux(g2 * uc[0] + g1 * uc[1]);
  const T s = d0 * (g1 * v0[0] + g2 * v0[1]) + d1 * (g2 * v0[0] + g1 * v0[1]);
  const T ra = C.dflux(P1Cell<T>::trace(uc)) * P1Cell<T>::trace(v0);
  const T rl = C.dflux(P1Cell<T>::trace(um)) * P1Cell<T>::trace(vm);
  T m[2];
  P1Cell<T>::minv(C, -s + T(0.5) * ra + T(1.5) * rl, s - T(1.5) * ra - T(0.5) * rl, m);
  out[0] = -m[0];
  out[1] = -m[1];
}

}  // namespace pdhg
