// Declarations shared by the kernel translation units and the host runtime.
#pragma once

#include <vector>

#include "pdhg.h"
#include "pdhg_device.hpp"

namespace pdhg {

template <typename T>
hipError_t launch_rows_fwd(const T* rows, int nrows, T* spec, int nt_spec, int lqb, int nx, const void* tw,
                           const Ctrl* ctrl, hipStream_t st);
template <typename T>
hipError_t launch_rows_inv(const T* spec, int nt_spec, int lqb, T* rows, int nrows, int nx, const void* tw,
                           const Ctrl* ctrl, hipStream_t st);
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

// rd_lazy = 1: the fused row pass evaluates the dual residual only where the
// stopping test or the stats need it (rd_needed).
// Copy (su, sp) to (du, dp) and record ctrl->ck_iter = max(n_done - 1, 0), unless the solve has stopped.
template <typename T>
hipError_t launch_checkpoint(Ctrl* ctrl, const T* su, const T* sp, T* du, T* dp, size_t nu, size_t np,
                             hipStream_t st);
hipError_t launch_ctrl_init(Ctrl* c, long long max_iter, double eps, double div_factor, hipStream_t st,
                            int rd_lazy = 0, long long stall = 0);
hipError_t launch_finalize(Ctrl* c, const double* part_rp, int n_rp, const double* part_rd, int n_rd,
                           double wscale, double* hist, hipStream_t st);

}  // namespace pdhg

namespace pdhg {
template <typename T>
hipError_t launch_adjoint_march(const Scheme& s, const T* u, const T* g, T* mu, T* grad, hipStream_t st);
}  // namespace pdhg

namespace pdhg {
// S: type of the spectrum, the FFT and the twiddle table tw (T, or float with
// an FP64 state and the single-precision preconditioner).  s0 (optional, nt
// values of type T): mode 0 of each spectrum row, taken from there instead of
// the spectrum.
template <typename T, typename S = T>
hipError_t launch_dual_fft(const S* spec, int nt, int lqb, int nx, const void* tw, T* phi, T* phibar, T tau,
                           const Ctrl* ctrl, hipStream_t st, const T* s0 = nullptr);
template <typename T, typename S = T>
hipError_t launch_primal_res(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                             S* spec, int lqb, const void* tw, double* part, const Ctrl* ctrl, hipStream_t st,
                             const LamArgs<T>* lam = nullptr);
// T: type of the spectrum; A: type of the factor rows and of the recurrences
// (double for a float spectrum under an FP64 state).  s0 (optional, nt values
// of type A): receives the mode-0 column of the solution.
template <typename T, typename A = T>
hipError_t launch_colsolve_wave(T* spec, const FacTab<A>& fac, int bw, int nt, int nx, int lqb, Ctrl* ctrl,
                                const double* part, int nparts, double wscale, double* hist, hipStream_t st,
                                A* s0 = nullptr);
// Maps of the chunked column solve (per mode and chunk, from the factor rows;
// nmodes = N_x/2 + 1): out [nmodes][chunk_count(nt)][12].
template <typename A>
hipError_t launch_colchunk_maps(const FacTab<A>& fac, int bw, int nt, int nmodes, A* out, hipStream_t st);
// The constant-row segment map of every mode and its squares (ChunkArgs::cpow):
// out [nmodes][kChunkPow][4].
hipError_t launch_colchunk_powers(const FacTab<double>& fac, int bw, int nmodes, double* out, hipStream_t st);
// The chunked column solve (N_t >= kChunkMinNt, N_x >= 16); s0 as for
// launch_colsolve_wave, in FP64.
template <typename T>
hipError_t launch_colsolve_chunk(T* spec, const ChunkArgs& ca, int bw, int nt, int nx, int lqb, Ctrl* ctrl,
                                 const double* part, int nparts, double wscale, double* hist, hipStream_t st,
                                 double* s0 = nullptr);
// Full-symbol preconditioner: g_k = (wr + vr)(1 - cos theta_k) + i ci sin theta_k per Fourier mode.
struct FullSym {
  double inv_ht;   // 1 / h_t
  double wr;       // lf_speed / h_x (Lax-Friedrichs) or c / h_x (upwind)
  double vr;       // 2 ghat / h_x^2 (viscosity of the linear-flux operator)
  double ci;       // c / h_x
  int bdf2;
};
template <typename T>
hipError_t launch_colsolve_full(T* spec, const FullSym& F, const void* tw, int nt, int nx, int lqb, Ctrl* ctrl,
                                const double* part, int nparts, double wscale, double* hist, hipStream_t st);
}  // namespace pdhg

namespace pdhg {
template <typename T>
hipError_t launch_level_sums(const T* u, int nx, size_t stride, int levels, double* out, hipStream_t st);
template <typename T>
hipError_t launch_refine_time(const T* uc, const T* pc, int ntc, size_t row, T* uf, T* pf, hipStream_t st);

// One-time-step solver (Algorithm 3): record of step l, written by its launch.
struct StepStat {
  long long iters;   // n*_l
  double rp, rd;     // residuals of the step at n*_l (L2 norm over the time slice)
  int status;        // 0 converged, 1 max_iter reached, 2 diverged
  int pad;
};
// One problem of a one-step launch (device table entry).
template <typename T>
struct OneStepProb {
  Scheme s;            // grid, scheme and resolved flux constants
  const C2<T>* tw;     // [nx] twiddles e^{-2 pi i j / nx}
  const T* sym;        // [2][nx] preconditioner symbol reciprocals (c0 = 1, c0 = 3/2), 1/M folded in;
                       // DG P1: [2][nx/2 + 1][4] per-mode inverses (onestep_dg1_kinv)
  const T* u0;         // [nx] or null; a march from step 0 reads u0 here and writes it to level 0 of u
  T* u;                // [nt+1][nx]; otherwise the levels before the first step marched are read
  T* phi;              // [nt][nx]  (DG P1: u0 [2][nx], u [nt+1][2][nx], phi [nt][2][nx])
  StepStat* stat;      // [nt]
  int* flag;           // 0 while the march runs, 2 after a step diverged
  double tau_u, tau_phi;
  // K_l^{-1} by cyclic reduction instead of the FFT when pcr_k[r] > 0 (row r as for sym): pcr [2][16]
  // holds the reduction ratios rho_0..rho_{k-1} and, in entry 15, the final scale
  const T* pcr;
  int pcr_k[2];
};
// Cyclic-reduction coefficients of the periodic tridiagonal K_l = (c0/h_t)^2 I + c^2 L_x (ghat = 0),
// rows c0 = 1 and c0 = 3/2, into out [2][16]; returns false (FFT path) when ghat != 0 or when a row
// would need the wrap-around step (the coupling ratio does not fall below tol within log2(nx) - 1 steps).
bool onestep_pcr(const pdhg_problem& p, double c, double tol, double* out, int* k);
template <typename T>
void onestep_symbol(const pdhg_problem& p, double c, double lf, T* out);   // host: [2][nx]
struct OneStepSummary {
  long long total;   // sum of the steps' n*
  double rp, rd;     // largest final step residuals
  int status;        // PDHG_OK / PDHG_NOT_CONVERGED / PDHG_DIVERGED
  int done;          // steps marched (the march stops after a diverged step)
};
OneStepSummary summarize_steps(const StepStat* rec, int nt, int64_t* step_iters, double* step_res);
// Threads per problem of the one-step march.
template <typename T>
__host__ __device__ inline int onestep_threads(int nx) {
  // FP64: 4 points per thread up to nx = 2048 (8 at 4096, the 512-thread limit), which keeps the
  // march's registers within the file; FP32: 8 points per thread
  const int w = nx / (sizeof(T) == 8 ? 4 : 8);
  return w < 64 ? 64 : (w > 512 ? 512 : w);
}
// Threads per problem of the DG P1 one-step march: two cells (four nodal values) per thread.
__host__ __device__ inline int onestep_threads_dg1(int nx) {
  const int w = nx / 2;
  return w < 64 ? 64 : (w > 512 ? 512 : w);
}
// DG P1: per-mode inverse of the one-level preconditioner, [2 rows c0 = 1, 3/2][nx/2 + 1][a, Re b, Im b, d]
template <typename T>
void onestep_dg1_kinv(const pdhg_problem& p, double c, T* out);
template <typename T>
hipError_t launch_onestep_dg1(const OneStepProb<T>* probs, int nprob, int max_nx, int l_begin, int l_end,
                              double eps, long long max_iter, double dfac, hipStream_t st);
template <typename T>
hipError_t launch_onestep_power(OneStepProb<T>* probs, int nprob, int max_nx, int iters, double* nu, hipStream_t st);
template <typename T>
hipError_t launch_onestep(const OneStepProb<T>* probs, int nprob, int max_nx, int l_begin, int l_end, double eps,
                          long long max_iter, double dfac, hipStream_t st);
}  // namespace pdhg

namespace pdhg {

// One problem of a batch (device table entry; filled on the host).
struct BatchProb {
  Scheme s;                  // grid, scheme and resolved flux constants
  long long u_off;           // element offset of u ([nt+1][nx]) in the packed u and u_alt
  long long f_off;           // element offset of phi, phibar and the spectrum ([nt][nx])
  long long u0_off;          // element offset of u0 ([nx])
  const void* tw;            // twiddles w_nx^i, i < nx (C2<T>)
  const void* fac_rows;      // preconditioner factor table of this problem (FacRow<T>)
  const int* fac_off;
  const int* fac_last;
  double tau_u, tau_phi, wscale;
  int lqb;                   // log2 of the spectrum column-block width
  int part_off;              // first partial-sum slot (one per row pair)
  int npairs;                // (nt + 1) / 2 row pairs
  int pairs_per_tile;        // S: row pairs per row tile
  int rtiles;                // ceil(npairs / S)
  int ncolg;                 // nx / 8 column groups
};

// Device pointers shared by the batched launches.
struct BatchLaunch {
  const BatchProb* probs;
  Ctrl* ctrls;
  int2* row_tiles;
  int2* col_tiles;
  int* counts;               // {row tiles, column tiles, active problems}
  const int* order;          // problem order of the row tiles
  const int* corder;         // problem order of the column tiles (decreasing nt)
  int nprob, max_nx;
};

template <typename T>
int batch_row_block_threads();
template <typename T>
int batch_row_width(int nx);
template <typename T>
size_t batch_row_lds(int max_nx);
template <typename T>
size_t batch_col_lds();
template <typename T>
hipError_t batch_occupancy(int which, int max_nx, int* blocks_per_cu);
template <typename T>
hipError_t launch_batch_dual_fft(const BatchLaunch& L, int grid, T* spec, T* phi, T* phibar, hipStream_t st);
template <typename T>
hipError_t launch_batch_primal_res(const BatchLaunch& L, int grid, const T* u_in, T* u_out, const T* phibar,
                                   const T* phi, T* spec, double* part, int rd_base, hipStream_t st);
template <typename T>
hipError_t launch_batch_colsolve(const BatchLaunch& L, int grid, T* spec, const double* part, int rd_base,
                                 hipStream_t st);
hipError_t launch_batch_compact(const BatchLaunch& L, hipStream_t st);
template <typename T>
hipError_t launch_batch_maxabs_dflux(const BatchLaunch& L, const T* u0, double* out, hipStream_t st);
template <typename T>
hipError_t launch_batch_init(const BatchLaunch& L, const T* u0, T* u, T* u_alt, T* phi, T* spec, int warm,
                             long long max_iter, double eps, double div_factor, hipStream_t st);
template <typename T>
hipError_t launch_batch_checkpoint(const BatchLaunch& L, const T* u_alt, const T* phi, T* ck_u, T* ck_phi,
                                   hipStream_t st);
template <typename T>
hipError_t launch_batch_finish(const BatchLaunch& L, T* u, const T* u_alt, double* drift, hipStream_t st);

}  // namespace pdhg

namespace pdhg {
// Host: banded Cholesky factor table of the time Gram plus the mode shifts
// (compressed per mode; rows[off[k] + min(l, last[k])]).
template <typename T>
void build_factor_rows(const pdhg_problem& p, double c, double ghat, std::vector<FacRow<T>>& rows,
                       std::vector<int>& off, std::vector<int>& last);
// The same for an explicit list of shifts (one table per entry).
template <typename T>
void build_factor_rows_shifts(const pdhg_problem& p, const std::vector<long double>& shifts,
                              std::vector<FacRow<T>>& rows, std::vector<int>& off, std::vector<int>& last);
}  // namespace pdhg

namespace pdhg {
// DG P2 space discretisation (pdhg_dg.hip).
template <typename T>
hipError_t launch_dg_residual(const Scheme& s, const T* u, T* r, double* part, const Ctrl* ctrl, hipStream_t st,
                              int* nblocks);
template <typename T>
hipError_t launch_dg_apply_jt(const Scheme& s, const T* u, const T* psi, T* out, double* part, hipStream_t st,
                              int* nblocks);
template <typename T>
hipError_t launch_dg_apply_j(const Scheme& s, const T* u, const T* v, T* out, hipStream_t st);
template <typename T>
hipError_t launch_dg_primal(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                            double* part, const Ctrl* ctrl, hipStream_t st, int* nblocks);
template <typename T>
hipError_t launch_dg_maxabs_trace(const T* u0, int nx, double a2, double b, double* part, hipStream_t st);
template <typename T>
hipError_t launch_dg_residual_fft(const Scheme& s, const T* u, T* spec, int lqb, const void* tw, double* part,
                                  const Ctrl* ctrl, hipStream_t st, int* nblocks);
// np coefficient planes: 3 (P2) or 2 (P1).
template <typename T>
hipError_t launch_dg_colsolve(T* spec, const FacTab<T>& fac, const T* vtab, int bw, int nt, int nx, int lqb,
                              const Ctrl* ctrl, hipStream_t st, int np);

// DG P2 residual with its per-cell products on the matrix cores (FP32; nx >= 64).
hipError_t launch_dg_residual_mfma(const Scheme& s, const float* u, float* r, double* part, const Ctrl* ctrl,
                                   hipStream_t st, int* nblocks);

// Implicit adjoint march of the DG schemes (pdhg_dg.hip): P2 or P1 by s.space; scratch of
// dg_adjoint_scratch_doubles(nx, planes) doubles of device memory.
size_t dg_adjoint_scratch_doubles(int nx, int np);
template <typename T>
hipError_t launch_dg_adjoint_march(const Scheme& s, const T* u, const T* g, T* mu, T* grad, double* scratch,
                                   hipStream_t st);

// DG P1 nodal upwind space discretisation (pdhg_dg1.hip).
template <typename T>
hipError_t launch_dg1_residual(const Scheme& s, const T* u, T* r, double* part, const Ctrl* ctrl, hipStream_t st,
                               int* nblocks);
template <typename T>
hipError_t launch_dg1_apply_jt(const Scheme& s, const T* u, const T* psi, T* out, double* part, hipStream_t st,
                               int* nblocks);
template <typename T>
hipError_t launch_dg1_apply_j(const Scheme& s, const T* u, const T* v, T* out, hipStream_t st);
template <typename T>
hipError_t launch_dg1_primal(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                             double* part, const Ctrl* ctrl, hipStream_t st, int* nblocks);
template <typename T>
hipError_t launch_dg1_maxabs(const T* u0, int nx, double a2, double b, double* part, hipStream_t st);

// Either DG discretisation, chosen by the scheme's space.
template <typename T>
inline hipError_t dgx_residual(const Scheme& s, const T* u, T* r, double* part, const Ctrl* ctrl, hipStream_t st,
                               int* nblocks) {
  return s.space == kSpaceDgP1 ? launch_dg1_residual<T>(s, u, r, part, ctrl, st, nblocks)
                               : launch_dg_residual<T>(s, u, r, part, ctrl, st, nblocks);
}
template <typename T>
inline hipError_t dgx_apply_jt(const Scheme& s, const T* u, const T* psi, T* out, double* part, hipStream_t st,
                               int* nblocks) {
  return s.space == kSpaceDgP1 ? launch_dg1_apply_jt<T>(s, u, psi, out, part, st, nblocks)
                               : launch_dg_apply_jt<T>(s, u, psi, out, part, st, nblocks);
}
template <typename T>
inline hipError_t dgx_apply_j(const Scheme& s, const T* u, const T* v, T* out, hipStream_t st) {
  return s.space == kSpaceDgP1 ? launch_dg1_apply_j<T>(s, u, v, out, st) : launch_dg_apply_j<T>(s, u, v, out, st);
}
template <typename T>
inline hipError_t dgx_primal(const Scheme& s, const T* u_in, T* u_out, const T* phibar, const T* phi, T tau_u,
                             double* part, const Ctrl* ctrl, hipStream_t st, int* nblocks) {
  return s.space == kSpaceDgP1 ? launch_dg1_primal<T>(s, u_in, u_out, phibar, phi, tau_u, part, ctrl, st, nblocks)
                               : launch_dg_primal<T>(s, u_in, u_out, phibar, phi, tau_u, part, ctrl, st, nblocks);
}
}  // namespace pdhg
