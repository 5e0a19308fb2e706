// Declarations shared by the kernel translation units and the host runtime.
#pragma once

#include "pdhg_device.hpp"

namespace pdhg {

template <typename T>
hipError_t launch_rows_fwd(const T* rows, int nrows, T* spec, int nt_spec, int lqb, int nx, const void* tw,
                           const Ctrl* ctrl, hipStream_t st);
template <typename T>
hipError_t launch_rows_inv(const T* spec, int nt_spec, int lqb, T* rows, int nrows, int nx, const void* tw,
                           const Ctrl* ctrl, hipStream_t st);
template <typename T>
hipError_t launch_colsolve(T* spec, const FacTab<T>& fac, int bw, int nt, int nx, int lqb, const Ctrl* ctrl,
                           hipStream_t st);
template <typename T>
hipError_t launch_residual(const Scheme& s, const T* u, T* r, double* part, const Ctrl* ctrl, hipStream_t st,
                           int* nblocks);
template <typename T>
hipError_t launch_apply_jt(const Scheme& s, const T* u, const T* psi, T* out, double* part, hipStream_t st,
                           int* nblocks);
template <typename T>
hipError_t launch_apply_j(const Scheme& s, const T* u, const T* v, T* out, hipStream_t st);
template <typename T>
hipError_t launch_primal(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                         double* part, const Ctrl* ctrl, hipStream_t st, int* nblocks);
template <typename T>
hipError_t launch_dual(T* phi, T* phibar, const T* srow, size_t n, T tau, const Ctrl* ctrl, hipStream_t st);
template <typename T>
hipError_t launch_fill(T* p, size_t n, T v, hipStream_t st);
template <typename T>
hipError_t launch_broadcast_levels(T* u, const T* u0, int nx, int levels, hipStream_t st);
template <typename T>
hipError_t launch_copy(T* dst, const T* src, size_t n, hipStream_t st);
template <typename T>
hipError_t launch_dot(const T* x, const T* y, size_t n, double* part, double* out, hipStream_t st);
template <typename T>
hipError_t launch_maxabs_dflux(const T* x, size_t n, double a2, double b, double* part, hipStream_t st);
template <typename T>
hipError_t launch_normalize(T* x, size_t n, const double* nrm2, hipStream_t st);

hipError_t launch_ctrl_init(Ctrl* c, long long max_iter, double eps, double div_factor, hipStream_t st);
hipError_t launch_finalize(Ctrl* c, const double* part_rp, int n_rp, const double* part_rd, int n_rd,
                           double wscale, double* hist, hipStream_t st);

}  // namespace pdhg

namespace pdhg {
template <typename T>
hipError_t launch_adjoint_march(const Scheme& s, const T* u, const T* g, T* mu, T* grad, hipStream_t st);
}  // namespace pdhg

namespace pdhg {
template <typename T>
hipError_t launch_dual_fft(const T* spec, int nt, int lqb, int nx, const void* tw, T* phi, T* phibar, T tau,
                           const Ctrl* ctrl, hipStream_t st);
template <typename T>
hipError_t launch_primal_res(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                             T* spec, int lqb, const void* tw, double* part, const Ctrl* ctrl, hipStream_t st);
template <typename T>
hipError_t launch_colsolve_wave(T* spec, const FacTab<T>& fac, int bw, int nt, int nx, int lqb, Ctrl* ctrl,
                                const double* part, int nparts, double wscale, double* hist, hipStream_t st);
}  // namespace pdhg

namespace pdhg {
template <typename T>
hipError_t launch_level_sums(const T* u, int nx, int levels, double* out, hipStream_t st);
}  // namespace pdhg
