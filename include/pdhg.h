/*
 * pdhg.h -- C ABI of the space-time primal-dual solver for implicit
 * discretisations of 1-D periodic conservation laws.
 *
 * Method: Liu, Osher, Li, Shu, "A primal-dual approach for solving
 * conservation laws with implicit in time approximations".  The initial-value
 * problem u_t + f(u)_x - gamma u_xx = 0, u(x,0) = u0 (Section 2.1) is
 * discretised implicitly in time (backward Euler or BDF2, Section 3.1) and in
 * space (finite differences, Section 3.2), and the whole space-time system
 * A(u) = 0 is solved at once as the saddle point of L(u,phi) = <phi, A(u)>
 * by the preconditioned primal-dual hybrid gradient iteration of Algorithm 1
 * (Section 3.3), with the dual proximal step taken in the H-norm induced by
 * K = -d_tt - c^2 d_xx + ghat^2 d_xxxx (Section 2.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array argument is DEVICE memory on the current HIP device, owned by
 *   the caller (for example a PyTorch tensor).  The library never frees a
 *   caller buffer.  Scalars and structs are host memory.
 * - The element type of every array is the problem's dtype (float or double).
 * - Layouts, row-major, x fastest:
 *     u   [nt+1][nx]   levels l = 0..nt; level 0 is the initial data
 *                      (DG: [nt+1][3][nx], and every [nt][nx] below is [nt][3][nx])
 *     phi [nt][nx]     one dual row per implicit equation l = 0..nt-1
 *     r   [nt][nx]     implicit residual rows A(u)^l
 *     g   [nt][nx]     J(u)^T phi, row m-1 belongs to unknown level m = 1..nt
 * - nx must be a power of two, 8 <= nx <= 4096; 1 <= nt <= 8192.
 * - Calls are asynchronous on the given stream unless stated otherwise.  One
 *   handle must not be used from two streams at the same time.
 * - Functions return a pdhg_status; they never throw.  On PDHG_EHIP the HIP
 *   error text is available from pdhg_last_error(handle).
 */
#ifndef PDHG_H_
#define PDHG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* pdhg_stream_t;   /* a hipStream_t; NULL = default stream */

typedef enum {
  PDHG_OK = 0,
  PDHG_NOT_CONVERGED = 1,   /* max_iter reached; u, phi hold iterate max_iter            */
  PDHG_DIVERGED = 2,        /* non-finite or exploding residual; u, phi hold the last good
                               checkpoint (pdhg_solve) or the last iterate (the other solvers) */
  PDHG_STALLED = 3,         /* stall_iters iterations without a new best ||A(u)|| (rounding
                               floor); u, phi hold the last iterate (pdhg_solve only)      */
  PDHG_EINVAL = -1,         /* invalid argument (sizes, enums, null pointers)            */
  PDHG_EHIP = -2,           /* a HIP runtime call failed                                 */
  PDHG_EUNSUPPORTED = -3,   /* valid but not implemented combination                     */
  PDHG_EWORKSPACE = -4      /* workspace too small                                       */
} pdhg_status;

typedef enum { PDHG_F32 = 0, PDHG_F64 = 1 } pdhg_dtype;

/* Time discretisation (Section 3.1).  BDF2 starts with one backward Euler row,
 * the start-up step being left open by the paper. */
typedef enum { PDHG_BE = 0, PDHG_BDF2 = 1 } pdhg_time;

/* Spatial discretisation (Section 3.2):
 *  PDHG_FD_UPWIND: F_j = (f(u_j) - f(u_{j-1}))/h_x, requires f' >= 0 (as the paper's
 *                  upwind examples assume);
 *  PDHG_FD_LF:     global Lax-Friedrichs flux with constant lf_speed.
 *  Both add centred diffusion -gamma (u_{j+1} - 2u_j + u_{j-1})/h_x^2 when gamma > 0.
 *  PDHG_DG_P2_LLF: discontinuous Galerkin on nx cells, Legendre basis of degree 2
 *                  (3 coefficients per cell), local Lax-Friedrichs flux
 *                  (s = max(|f'(a)|, |f'(b)|) per interface), volume integrals by
 *                  3-point Gauss.  Arrays carry coefficient planes: u [nt+1][3][nx],
 *                  phi [nt][3][nx], u0 [3][nx] (the projected initial data).
 *                  Requires 16 <= nx, nt <= 512, gamma = 0; lf_speed and
 *                  precond_gamma_hat are not used; the default precond_c is
 *                  max |f'| over the cell-edge traces of u0.  The preconditioner
 *                  couples the three planes through the unit-speed upwind DG
 *                  operator G: K_d = (B_t B_t^T) (x) I + I_t (x) c^2 G G^T.
 *  PDHG_DG_P1_UPWIND: the paper's DG example (Sections 3.2.2, 3.2.3): piecewise
 *                  linear on nx cells, stored by the nodal values at x_c - h/4 and
 *                  x_c + h/4 (x_c the cell centre), upwind flux f(u^-) (requires
 *                  f' >= 0), volume integrals by 2-point Gauss.  Arrays: u [nt+1][2][nx],
 *                  phi [nt][2][nx], u0 [2][nx] (nodal values of the initial data).
 *                  Limits as for PDHG_DG_P2_LLF; the default precond_c is max |f'|
 *                  over the nodal values and edge traces of u0; K_d as above with
 *                  the P1 operator G. */
typedef enum { PDHG_FD_UPWIND = 0, PDHG_FD_LF = 1, PDHG_DG_P2_LLF = 2, PDHG_DG_P1_UPWIND = 3 } pdhg_space;

/* Dual-step preconditioner K_d (Sections 2.2, 3.3):
 *  PDHG_PRECOND_GRAM: K_d = (B_t B_t^T) (x) I + I_t (x) (c^2 L_x + ghat^2 L_x^2), the
 *                  discrete form of the paper's K = -d_tt - c^2 d_xx + ghat^2 d_xxxx
 *                  (default precond_c: max |f'(u0)|).
 *  PDHG_PRECOND_FULL: K_d = J_c J_c^T with J_c = B_t (x) I + I (x) G_c the scheme's
 *                  Jacobian for the linear flux f = c u (same Lax-Friedrichs constant,
 *                  ghat as the viscosity): the Gram reading with the cross term of
 *                  A^T A that the paper drops when it forms K.  Per Fourier mode k,
 *                  K_k = L_k L_k^* with L_k = B_t + g_k I lower triangular (g_k the
 *                  symbol of G_c), solved by two substitutions along t.  Default
 *                  precond_c: the mean of f'(u0) (the signed transport speed).
 *                  Finite differences only (PDHG_EUNSUPPORTED for DG and for batches).
 *  PDHG_PRECOND_GRAM_F32: K_d as PDHG_PRECOND_GRAM for an FP64 problem, with the
 *                  spectral pass in single precision inside pdhg_solve: the residual
 *                  rows are rounded to float before the forward FFT, and the FFTs,
 *                  the spectrum in the workspace, the factor tables and the column
 *                  solve are float; u, phi, phibar, the residuals and both norms stay
 *                  FP64.  The rounding is relative to the residual, so the fixed point
 *                  (A(u) = 0) and the stopping test are those of FP64.  Requires
 *                  dtype PDHG_F64, finite differences, nx >= 64 and the fused loop
 *                  body (variant 0 or 2); PDHG_EUNSUPPORTED otherwise, and for
 *                  pdhg_solve_refined, pdhg_solve_onestep and batches.  pdhg_precond
 *                  and the step-size power iteration apply the FP64 operator. */
typedef enum { PDHG_PRECOND_GRAM = 0, PDHG_PRECOND_FULL = 1, PDHG_PRECOND_GRAM_F32 = 2 } pdhg_precond_kind;

typedef struct {
  int32_t nx, nt;
  double length;            /* periodic domain [0, length)                                */
  double t_final;           /* T; h_t = T / nt                                            */
  double alpha, beta;       /* flux f(u) = alpha u^2 + beta u (linear transport: alpha = 0) */
  double gamma;             /* constant viscosity (>= 0)                                  */
  int32_t time;             /* pdhg_time                                                  */
  int32_t space;            /* pdhg_space                                                 */
  int32_t dtype;            /* pdhg_dtype                                                 */
  int32_t precond_kind;     /* pdhg_precond_kind                                          */
  double lf_speed;          /* Lax-Friedrichs constant; < 0: max |f'(u0)| at solve time    */
  double precond_c;         /* c of K (Section 2.2); < 0: max |f'(u0)| at solve time       */
  double precond_gamma_hat; /* ghat of K (>= 0)                                           */
} pdhg_problem;

typedef struct {
  double tau_u, tau_phi;    /* step sizes; <= 0: both sqrt(0.95 / nu_max), nu_max the largest
                               eigenvalue of J(u0)^T K_d^{-1} J(u0) by power iteration
                               (Proposition 2.1 needs tau_u tau_phi nu < 1)               */
  double eps;               /* stop when ||A(u)|| <= eps and ||J(u)^T phi|| <= eps (Section 3.3);
                               eps <= 0 runs exactly max_iter iterations                 */
  int64_t max_iter;
  int32_t check_every;      /* iterations per captured graph launch between host polls   */
  int32_t warm_start;       /* 0: u^l = u0, phi = 0 (Section 3.3);  1: start from u, phi   */
  double diverge_factor;    /* diverged when max(Rp,Rd) > diverge_factor * best so far;
                               <= 0: 1e6                                                 */
  int32_t variant;          /* 0 = auto (2; DG: 4), 1 = unfused reference kernels (7 per
                               iteration), 2 = fused passes (3 kernels per iteration),
                               4 = the DG loop body (5 kernels per iteration),
                               6 = the DG P2 body (FP32, nx >= 64) whose residual runs its
                               per-cell Gauss-node and volume products on the matrix cores
                               (v_mfma_f32_16x16x4f32), then the row FFT: a measured
                               alternative to 4 (PDHG_EUNSUPPORTED for other problems)  */
  int32_t backoff;          /* after a divergence, restart from the last good checkpoint with
                               tau_u and tau_phi times 0.7, at most this many times (0: none) */
  double* history;          /* nullable DEVICE buffer [max_iter+2][2] of doubles: entry n holds
                               (||A(u^n)||, ||J(u^n)^T phi^n||) for n = 0..n*; entry 0 is
                               (NaN, ||J(u^0)^T phi^0||); entries past n* may be written */
  double eps_rel;           /* > 0: the tolerance is max(eps, eps_rel ||u0|| / h_t) with
                               ||u0|| = sqrt(h_x sum u0^2), the scale-free form for single
                               precision, whose residual floor grows like 1/h_t          */
  int32_t stall_iters;      /* > 0: stop with PDHG_STALLED when ||A(u)|| has not improved on its
                               best for this many iterations (the rounding floor)         */
  int32_t init_multiplier;  /* 1: the multiplier form of Algorithm 1 (Section 3.3): u^0 is an
                               unknown and lambda imposes u^0 = u0 through the term
                               h_x sum_j lambda_j (u^0_j - u0_j) of the Lagrangian; standard
                               primal-dual steps u^0 <- u^0 - tau_u0 (h_t J_0^T phibar + lambdabar),
                               lambda <- lambda + tau_lam (u^0 - u0) with extrapolation, where
                               h_t J_0^T phibar = -phibar^0 (+ phibar^1 / 2 for BDF2); u[0] then
                               returns the iterated u^0.  Fused finite-difference passes only
                               (PDHG_EUNSUPPORTED otherwise, and with backoff > 0).       */
  double tau_u0;            /* u^0 step of the multiplier form; <= 0: tau_u / 2            */
  double tau_lam;           /* lambda step of the multiplier form; <= 0: 0.99              */
} pdhg_params;

typedef struct {
  int64_t iters;            /* n*, the index of the returned iterate                      */
  double res_primal;        /* ||A(u^{n*})||   (space-time L2 norm sqrt(h_t h_x sum .^2)) */
  double res_dual;          /* ||J(u^{n*})^T phi^{n*}||; NaN after divergence in the fused   */
                            /* loop body, which evaluates it only where the stopping test  */
                            /* or the last iterate needs it (||A(u)|| <= eps or n = max_iter) */
  double tau_u, tau_phi;    /* step sizes used                                            */
  double nu_max;            /* power-iteration estimate (0 if steps were given)           */
  double lf_speed, precond_c; /* constants used                                           */
  double seconds;           /* wall time of the iteration loop                            */
  double mass_drift;        /* max_l |m^l - m^0| with m^l = h_x sum_j u^l_j (conservation check) */
  int32_t status;
  int32_t variant;          /* kernel variant that ran                                    */
} pdhg_stats;

typedef struct pdhg_handle pdhg_handle;

/* Create a plan for one problem: validates it and builds the FFT twiddle
 * tables on the current device.  The banded Cholesky factors of the
 * preconditioner are built at the first solve, once c is known. */
int pdhg_setup(const pdhg_problem* prob, pdhg_handle** out);

/* Bytes of device workspace pdhg_solve/pdhg_adjoint need for this problem. */
size_t pdhg_workspace_bytes(const pdhg_handle* h);

/* Run Algorithm 1 (u^0 = u0 held fixed, standard PDHG signs; Section 3.3):
 *   u   <- u - tau_u J(u)^T phibar            (primal step)
 *   phi <- phi + tau_phi K_d^{-1} A(u)        (dual step; phibar = phi + tau_phi K_d^{-1} A(u))
 * until both residuals are <= eps or max_iter iterations.  u [nt+1][nx] and
 * phi [nt][nx] receive the iterate n* (u[0] = u0).  workspace: device buffer
 * of pdhg_workspace_bytes() bytes, or NULL to let the handle allocate its own
 * (kept until pdhg_destroy).  stats: host struct, filled on return.
 * Synchronises the stream (it polls the device-side convergence flag).
 * Divergence (a non-finite residual, or ||A(u)|| above diverge_factor times the
 * best so far) returns PDHG_DIVERGED with u, phi = the last good checkpoint:
 * the iterate M = k check_every - 1 (k >= 1), or the start (M = 0), latest
 * before the diverging one; stats then report M and that state's residuals.
 * With params->backoff > 0 the solve instead restarts from that checkpoint
 * with both step sizes times 0.7 (warm start: phibar = phi), up to backoff
 * times; stats.iters counts every iteration run up to the returned iterate,
 * and stats.tau_u, tau_phi are the steps of the last run.
 * Returns PDHG_OK, PDHG_NOT_CONVERGED, PDHG_DIVERGED or an error. */
int pdhg_solve(pdhg_handle* h, const void* u0, void* u, void* phi, void* workspace,
               const pdhg_params* params, pdhg_stats* stats, pdhg_stream_t stream);

/* Mesh refinement in time (Algorithm 2, Section 3.4): Algorithm 1 on the meshes
 * N x nt_start, N x 2 nt_start, ..., N x nt (nt / nt_start a power of two), each
 * level started from the previous level's solution interpolated in time (u
 * linearly: fine level 2l = coarse level l, fine level 2l+1 = their mean; phi
 * piecewise constant: fine rows 2l and 2l+1 take coarse row l), the first level
 * from u^l = u0, phi = 0.  Coarse levels stop at coarse_eps (<= 0: params->eps)
 * or coarse_max_iter; the finest level uses params (its warm_start is implied
 * when there are coarse levels).  Step sizes: params->tau_u/tau_phi for every
 * level when > 0, otherwise the power-iteration default per level.  The coarse
 * levels' plans and buffers are created on first use and kept by the handle. */
typedef struct {
  int32_t nt_start;         /* coarsest mesh N_t0 (>= 1)                                 */
  int32_t reserved;
  int64_t coarse_max_iter;  /* iteration cap on each coarse level                        */
  double coarse_eps;        /* tolerance on the coarse levels; <= 0: params->eps          */
} pdhg_refine_params;

/* As pdhg_solve, on the refined mesh sequence.  stats: the finest level's
 * (or, if a coarse level diverges, that level's, with PDHG_DIVERGED returned).
 * level_iters: nullable HOST array with one entry per level (n* of each). */
int pdhg_solve_refined(pdhg_handle* h, const void* u0, void* u, void* phi, void* workspace,
                       const pdhg_params* params, const pdhg_refine_params* refine, pdhg_stats* stats,
                       int64_t* level_iters, pdhg_stream_t stream);

/* One-time-step solver (Algorithm 3, Section 3.5).  The scheme is marched one
 * implicit step at a time: step l (l = 0..nt-1) runs Algorithm 1 on the N_x x 1
 * problem A_l(v) = (c0 v + c1 u^l + c2 u^{l-1})/h_t + F(v) = 0 for v = u^{l+1},
 * (c0, c1, c2) the coefficients of row l, started from v = u^l, phi = 0.  Its
 * preconditioner is K_l = (c0/h_t)^2 I + c^2 L_x + ghat^2 L_x^2 (the Gram form
 * with one unknown level, inverted by the FFT), and it stops when both
 * residuals, in the L2 norm of the time slice sqrt(h_x sum z^2), are <= eps or
 * after max_iter iterations; the march then goes on from that step's iterate.
 *   params: tau_u, tau_phi (<= 0: sqrt(0.95 / nu_max), nu_max the largest
 *   power-iteration eigenvalue of J^T K^{-1} J at u0 over the step operators,
 *   c0 = 1 and, for BDF2, 3/2), eps and max_iter per step, diverge_factor as
 *   for pdhg_solve; check_every, warm_start, variant and history are ignored.
 *   u [nt+1][nx] receives u^0 = u0 and every step's solution; phi [nt][nx] row l
 *   receives the dual of step l at its n*.  A step that diverges stops the
 *   march: PDHG_DIVERGED, and the rows after it are left unwritten.
 *   stats: iters = sum of the steps' n*, res_primal/res_dual = the largest final
 *   step residuals, variant = 5.  step_iters: nullable HOST [nt] (n* per step);
 *   step_res: nullable HOST [nt][2] (final residuals per step).
 * Finite differences with nx >= 64, and the DG P1 nodal upwind scheme with
 * 64 <= nx <= 4096 cells (PDHG_EUNSUPPORTED otherwise, including DG P2).  For
 * DG P1 the unknowns are the two nodal planes: u0 [2][nx], u [nt+1][2][nx],
 * phi [nt][2][nx]; K_l = (c0/h_t)^2 I + c^2 G G^T with G the unit-speed upwind
 * P1 operator (a 2x2 block per Fourier mode over the cells), the slice norm
 * sums both planes, nu_max comes from Algorithm 1's power iteration on the
 * one-level problems, and stats.mass_drift is -1 (not measured).  One
 * workgroup per step: the call is latency-bound by design and leaves the rest
 * of the GPU to other streams.  Synchronous on `stream`. */
int pdhg_solve_onestep(pdhg_handle* h, const void* u0, void* u, void* phi, const pdhg_params* params,
                       pdhg_stats* stats, int64_t* step_iters, double* step_res, pdhg_stream_t stream);

/* Residual of the saddle-point system (Section 2.3): Au = A(u) [nt][nx] and
 * JTphi = J(u)^T phi [nt][nx] (either may be NULL), and res[2] (host) =
 * { ||A(u)||, ||J(u)^T phi|| } (res may be NULL; then the call is asynchronous).
 * u includes level 0.  Uses the constants of the last solve, or the
 * defaults computed from u[0] when no solve ran yet. */
int pdhg_residual(pdhg_handle* h, const void* u, const void* phi, void* Au, void* JTphi,
                  double* res, pdhg_stream_t stream);

/* pdhg_residual without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, outputs and constants as
 * pdhg_residual; A(u) and J(u)^T phi are bitwise those of pdhg_residual, and
 * the two norms agree to rounding (they are reduced on the device instead of
 * on the host).  Instead of the handle's workspace, the per-block partial sums
 * live in a static device array of 4 MiB that each GPU the library runs on
 * holds until the process ends; nt * nx must not exceed 67,092,480 points
 * (PDHG_EINVAL otherwise, with the reason in pdhg_last_error).  Every call on
 * one GPU shares that array: calls that overlap on one GPU (on different
 * streams, or from different threads) race and must be serialised by the
 * caller.  No hipMalloc, hipFree or other allocating call is made; the
 * constants, when no solve ran yet, are resolved from u[0] without building
 * the preconditioner's factor tables.  Synchronous on `stream` when res is
 * non-NULL. */
int pdhg_residual_static(pdhg_handle* h, const void* u, const void* phi, void* Au, void* JTphi,
                         double* res, pdhg_stream_t stream);

/* Preconditioner: s = K_d^{-1} r for r, s of shape [nt][nx] (may alias).
 * K_d = (B_t B_t^T) (x) I + I (x) (c^2 L_x + ghat^2 L_x^2), solved by FFT in x and
 * banded Cholesky in t (Sections 2.2, 3.3).  c = precond_c (must be resolved:
 * either given >= 0 in the problem or set by a previous solve). */
int pdhg_precond(pdhg_handle* h, const void* r, void* s, pdhg_stream_t stream);

/* Dual-equation operator and the implicit adjoint (Section 3.1).
 *  mode PDHG_ADJ_APPLY: out[nt][nx] = J(u)^T in, in = phi [nt][nx].
 *  mode PDHG_ADJ_SOLVE:
 *     in = dL/du [nt+1][nx] (all levels, level 0 included);
 *     solves J(u)^T mu = dL/du[1:] by a backward march in time and writes
 *     out[nx] = dL/du0 = dL/du^0 - (dA/du0)^T mu.  mu [nt][nx] receives the
 *     multiplier if non-NULL.  Finite differences: one periodic tridiagonal
 *     solve per level (cyclic reduction in one workgroup).  DG (P2 and P1; every
 *     [nx] above is [planes][nx], and the gradient is with respect to the
 *     initial coefficients or nodal values): one periodic block-tridiagonal
 *     solve per level (3x3 or 2x2 blocks of the exact Jacobian, block cyclic
 *     reduction in one workgroup over a block-row array in the workspace).
 *     Arithmetic in double for both storage types.  u must be the converged
 *     implicit solution for this to be the gradient of the solution map.
 *     workspace as for pdhg_solve (NULL allowed). */
typedef enum { PDHG_ADJ_APPLY = 0, PDHG_ADJ_SOLVE = 1 } pdhg_adjoint_mode;
int pdhg_adjoint(pdhg_handle* h, int32_t mode, const void* u, const void* in, void* out,
                 void* mu, void* workspace, pdhg_stream_t stream);

/* Average device time (milliseconds, from HIP events on `stream`) of `reps`
 * back-to-back launches of one kernel of the solve loop, with the buffers and
 * step sizes of the last pdhg_solve on this handle (the buffers' contents are
 * overwritten).  kernel: 0 = fused primal/residual/FFT pass, 1 = column solve,
 * 2 = inverse row FFT, 3 = dual update, 4 = primal update, 5 = residual,
 * 6 = forward row FFT, 7 = fused inverse-FFT/dual pass, 8 = plain device copy
 * (DG: 0 = residual of two levels + forward FFT of their six coefficient rows,
 * 1 = column solve in the per-mode eigenbasis, 4 = primal step with the
 * dual residual, 5 = residual, 6 = forward row FFT of the 3 nt coefficient
 * rows, 7 = inverse FFT + dual step, 8 = copy, 9 = residual with its per-cell
 * products on the matrix cores (P2, FP32); others PDHG_EUNSUPPORTED)
 * of N_t*N_x elements (one read and one write per element; the reference point
 * for bandwidth and for scaling hardware byte counters).
 * Used for roofline measurements.  Returns PDHG_EINVAL without a previous solve. */
int pdhg_time_kernel(pdhg_handle* h, int32_t kernel, int32_t reps, double* ms_per_launch,
                     pdhg_stream_t stream);

void pdhg_destroy(pdhg_handle* h);
const char* pdhg_status_string(int status);
const char* pdhg_last_error(const pdhg_handle* h);

/* ======================================================================
 * Batched solver: many independent problems of Section 2.1 (each its own
 * N_x, N_t, flux, scheme and initial data) advanced together by Algorithm 1,
 * one kernel launch per pass for the whole batch, the iteration loop replayed
 * as a HIP graph, and a convergence decision per problem (Section 3.3 stopping
 * rule) taken on the device; converged problems drop out of the work lists.
 * Each problem's iterates are those of pdhg_solve with the fused passes (the
 * same pass bodies); the residual norms can differ in the last bits where the
 * reduction order differs.
 *
 * Packed layouts: problem i occupies
 *     u0  [u0_off_i, u0_off_i + nx_i)                    its initial data
 *     u   [u_off_i,  u_off_i + (nt_i+1) nx_i)            as [nt_i+1][nx_i]
 *     phi [phi_off_i, phi_off_i + nt_i nx_i)             as [nt_i][nx_i]
 * with offsets (in elements) the exclusive prefix sums in problem order, from
 * pdhg_batch_offsets.  Limits: every problem has the same dtype, nx a power of
 * two with 256 <= nx <= 4096, 1 <= nt <= 512.
 * ==================================================================== */
typedef struct pdhg_batch pdhg_batch;

typedef struct {
  const double* tau_u;      /* HOST array [nprob] or NULL; entries <= 0 (or NULL): automatic
                               per problem, as pdhg_params.tau_u                          */
  const double* tau_phi;    /* HOST array [nprob] or NULL (as tau_u)                      */
  double eps;               /* per-problem stopping tolerance, as pdhg_params.eps         */
  int64_t max_iter;         /* per problem                                                */
  int32_t check_every;      /* iterations per graph launch between host polls (even)      */
  int32_t warm_start;       /* as pdhg_params.warm_start                                  */
  double diverge_factor;    /* as pdhg_params.diverge_factor                              */
} pdhg_batch_params;

/* Plan a batch of nprob >= 1 problems (host array).  Builds twiddle tables
 * and the problem table on the current device.  Returns PDHG_EINVAL for an
 * invalid problem, PDHG_EUNSUPPORTED outside the limits above. */
int pdhg_batch_setup(const pdhg_problem* probs, int32_t nprob, pdhg_batch** out);

/* Element counts of the packed u0, u and phi arrays, and the workspace bytes
 * pdhg_batch_solve needs (any pointer may be NULL). */
int pdhg_batch_sizes(const pdhg_batch* b, int64_t* u0_elems, int64_t* u_elems, int64_t* phi_elems,
                     size_t* workspace_bytes);

/* Offsets (elements) of problem i in the packed u0, u and phi arrays. */
int pdhg_batch_offsets(const pdhg_batch* b, int32_t i, int64_t* u0_off, int64_t* u_off, int64_t* phi_off);

/* Solve every problem of the batch (Algorithm 1 per problem, all in the same
 * launches).  u0, u, phi: packed DEVICE arrays; workspace: DEVICE buffer of
 * pdhg_batch_sizes() bytes (not NULL).  stats: HOST array [nprob], filled on
 * return (iters, residuals, step sizes, constants, mass drift, status per
 * problem; seconds = wall time of the whole batch loop).  Synchronises the
 * stream.  Returns PDHG_OK when every problem converged, PDHG_DIVERGED when one
 * diverged, else PDHG_NOT_CONVERGED; or an error. */
int pdhg_batch_solve(pdhg_batch* b, const void* u0, void* u, void* phi, void* workspace,
                     const pdhg_batch_params* params, pdhg_stats* stats, pdhg_stream_t stream);

/* The one-time-step solver (Algorithm 3, Section 3.5; see pdhg_solve_onestep)
 * for every problem of the batch: one workgroup marches each problem, all in
 * one launch.  u0, u, phi: packed DEVICE arrays as above (no workspace).
 * params: tau_u/tau_phi per problem (<= 0 or NULL: the one-step power-iteration
 * default), eps and max_iter per step, diverge_factor; check_every and
 * warm_start are ignored.  stats: HOST [nprob] (iters = sum of the steps' n*,
 * res_primal/res_dual = largest final step residuals, mass_drift = -1: not
 * computed, variant = 5, seconds = wall time of the march launch).
 * step_iters: nullable HOST array [sum of nt_i], problem i's steps at the
 * exclusive prefix sum of the nt_j.  A diverged step stops only its own
 * problem's march.  Synchronises the stream.  Returns as pdhg_batch_solve. */
int pdhg_batch_solve_onestep(pdhg_batch* b, const void* u0, void* u, void* phi, const pdhg_batch_params* params,
                             pdhg_stats* stats, int64_t* step_iters, pdhg_stream_t stream);

/* Autotuner: times each of the three batched passes on this batch (buffers as
 * for pdhg_batch_solve; their contents are overwritten) for every candidate
 * persistent grid size (1, 2, 4, 8 blocks per compute unit up to the occupancy
 * limit, and one block per tile), keeps the fastest per pass for later solves
 * of this handle, and returns the three grid sizes in grids[3] (host) if not
 * NULL.  Without a call, grids default to the occupancy limit. */
int pdhg_batch_tune(pdhg_batch* b, const void* u0, void* u, void* phi, void* workspace,
                    const pdhg_batch_params* params, int32_t* grids, pdhg_stream_t stream);

/* Average device time (milliseconds, HIP events on `stream`, one event pair
 * per launch) of `reps` launches of one batched pass with the current grid
 * sizes and the buffers of the last pdhg_batch_solve (contents overwritten):
 * kernel 0 = inverse FFT + dual step, 1 = primal step + residual + forward
 * FFT, 2 = column solve (a primal pass refills the spectrum before each timed
 * launch).  Every problem is reset to its initial guess and counts as
 * running.  PDHG_EINVAL before any solve. */
int pdhg_batch_time_kernel(pdhg_batch* b, int32_t kernel, int32_t reps, double* ms_per_launch,
                           pdhg_stream_t stream);

void pdhg_batch_destroy(pdhg_batch* b);
const char* pdhg_batch_last_error(const pdhg_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* PDHG_H_ */
