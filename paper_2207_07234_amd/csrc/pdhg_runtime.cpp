// Host runtime and C ABI of the space-time primal-dual solver.
//
// Responsibilities: validate problems, build the FFT twiddles and the banded
// Cholesky factors of the preconditioner (Section 2.2 / 3.3), lay out the
// workspace, estimate step sizes by power iteration (Proposition 2.1 needs
// tau_u tau_phi nu_max < 1), and drive Algorithm 1: the loop body is captured
// once into a HIP graph of `check_every` iterations and replayed until the
// device-side control block reports convergence, divergence or max_iter.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <algorithm>
#include <vector>

#include "pdhg.h"
#include "pdhg_internal.hpp"

using namespace pdhg;

namespace pdhg {

// Banded Cholesky factors of (B_t B_t^T + s_k I), k = 0..nx/2, computed in
// long double and rounded to T.  B_t is the time difference acting on the
// unknown levels (row l: c0(l) at column l, c1(l) at l-1, c2(l) at l-2, all
// over h_t).  Rows of L converge to those of the infinite Toeplitz factor;
// for each mode only the rows up to the point after which every rounded row
// equals the last one are stored.
template <typename T>
void build_factor_rows_shifts(const pdhg_problem& p, const std::vector<long double>& shifts,
                              std::vector<FacRow<T>>& rows, std::vector<int>& off, std::vector<int>& last) {
  typedef long double LD;
  const int nt = p.nt;
  const LD ht = (LD)p.t_final / nt;
  const bool bdf2 = p.time == PDHG_BDF2;
  auto coef = [&](int l, int d) -> LD {   // B_t[l][l-d] * h_t
    if (d == 0) return (bdf2 && l >= 1) ? 1.5L : 1.0L;
    if (d == 1) return (l >= 1) ? ((bdf2 && l >= 1) ? -2.0L : -1.0L) : 0.0L;
    if (d == 2) return (bdf2 && l >= 2) ? 0.5L : 0.0L;
    return 0.0L;
  };
  // K[l][l-d] for d = 0, 1, 2 (times h_t^2)
  auto kband = [&](int l, int d) -> LD {
    if (l - d < 0) return 0.0L;
    LD s = 0.0L;
    for (int mcol = l - 2; mcol <= l - d; ++mcol) {
      if (mcol < 0) continue;
      const int da = l - mcol, db = (l - d) - mcol;
      if (da > 2 || db < 0 || db > 2) continue;
      s += coef(l, da) * coef(l - d, db);
    }
    return s;
  };
  const int nmodes = (int)shifts.size();
  off.assign(nmodes, 0);
  last.assign(nmodes, 0);
  rows.clear();
  std::vector<LD> d(nt), e1(nt), e2(nt);
  std::vector<FacRow<T>> tmp(nt);
  for (int k = 0; k < nmodes; ++k) {
    const LD shift = shifts[k];
    for (int l = 0; l < nt; ++l) {
      const LD k0 = kband(l, 0) / (ht * ht) + shift;
      const LD k1 = kband(l, 1) / (ht * ht);
      const LD k2 = kband(l, 2) / (ht * ht);
      e2[l] = (l >= 2) ? k2 / d[l - 2] : 0.0L;
      e1[l] = (l >= 1) ? (k1 - ((l >= 2) ? e2[l] * e1[l - 1] : 0.0L)) / d[l - 1] : 0.0L;
      d[l] = sqrtl(k0 - e1[l] * e1[l] - e2[l] * e2[l]);
      tmp[l] = FacRow<T>{(T)(1.0L / d[l]), (T)e1[l], (T)e2[l], (T)0};
    }
    int lst = nt - 1;
    while (lst > 0 && memcmp(&tmp[lst - 1], &tmp[nt - 1], sizeof(FacRow<T>)) == 0) --lst;
    off[k] = (int)rows.size();
    last[k] = lst;
    for (int l = 0; l <= lst; ++l) rows.push_back(tmp[l]);
  }
}

// Banded Cholesky factors of (B_t B_t^T + s_k I), k = 0..nx/2, s_k = c^2 mu_k +
// ghat^2 mu_k^2 with mu_k = 4 sin^2(pi k / nx) / h_x^2, computed in long double and
// rounded to T.  B_t is the time difference acting on the unknown levels (row l:
// c0(l) at column l, c1(l) at l-1, c2(l) at l-2, all over h_t).  Rows of L
// converge to those of the infinite Toeplitz factor; for each mode only the rows
// up to the point after which every rounded row equals the last one are stored.
template <typename T>
void build_factor_rows(const pdhg_problem& p, double c, double ghat, std::vector<FacRow<T>>& rows,
                       std::vector<int>& off, std::vector<int>& last) {
  typedef long double LD;
  const LD hx = (LD)p.length / p.nx;
  const LD PI = 3.141592653589793238462643383279502884L;
  std::vector<LD> shifts(p.nx / 2 + 1);
  for (int k = 0; k <= p.nx / 2; ++k) {
    const LD sn = sinl(PI * k / p.nx);
    const LD mu = 4.0L * sn * sn / (hx * hx);
    shifts[k] = (LD)c * c * mu + (LD)ghat * ghat * mu * mu;
  }
  build_factor_rows_shifts<T>(p, shifts, rows, off, last);
}

template void build_factor_rows<float>(const pdhg_problem&, double, double, std::vector<FacRow<float>>&,
                                        std::vector<int>&, std::vector<int>&);
template void build_factor_rows<double>(const pdhg_problem&, double, double, std::vector<FacRow<double>>&,
                                         std::vector<int>&, std::vector<int>&);
// Symbol of the one-step preconditioner per FFT index k, row r for c0 = 1 (r = 0)
// and c0 = 3/2 (r = 1): 1 / (M K_k), M = N_x / 2 (the 1/M normalises the half-length
// inverse FFT), with K_k = (c0/h_t)^2 + c^2 mu_k + ghat^2 mu_k^2, mu_k = 4 sin^2(pi k / N_x) / h_x^2,
// or, for the full-symbol preconditioner, K_k = |c0/h_t + g_k|^2 with
// g_k = (w (1 - cos theta_k) + i c sin theta_k) / h_x + ghat mu_k (w = lf for Lax-Friedrichs,
// c for upwind).  Computed in long double.
template <typename T>
void onestep_symbol(const pdhg_problem& p, double c, double lf, T* out) {
  typedef long double LD;
  const LD PI = 3.141592653589793238462643383279502884L;
  const int nx = p.nx;
  const LD ht = (LD)p.t_final / p.nt, hx = (LD)p.length / nx, cc = c, g = p.precond_gamma_hat;
  const LD w = p.space == PDHG_FD_LF ? (LD)lf : cc;
  for (int r = 0; r < 2; ++r) {
    const LD a = (r ? 1.5L : 1.0L) / ht;
    for (int k = 0; k < nx; ++k) {
      const LD th = 2.0L * PI * k / nx, sn = sinl(0.5L * th);
      const LD mu = 4.0L * sn * sn / (hx * hx);
      LD kk;
      if (p.precond_kind == PDHG_PRECOND_FULL) {
        const LD gr = a + w * (1.0L - cosl(th)) / hx + g * mu, gi = cc * sinl(th) / hx;
        kk = gr * gr + gi * gi;
      } else {
        kk = a * a + cc * cc * mu + g * g * mu * mu;
      }
      out[(size_t)r * nx + k] = (T)(2.0L / ((LD)nx * kk));
    }
  }
}
bool onestep_pcr(const pdhg_problem& p, double c, double tol, double* out, int* k) {
  typedef long double LD;
  if (p.precond_gamma_hat != 0.0 || p.precond_kind == PDHG_PRECOND_FULL) return false;
  int m = 0;
  while ((1 << (m + 1)) <= p.nx) ++m;   // log2(nx)
  const LD ht = (LD)p.t_final / p.nt, hx = (LD)p.length / p.nx, e0 = (LD)c * c / (hx * hx);
  for (int r = 0; r < 2; ++r) {
    const LD a = (r ? 1.5L : 1.0L) / ht;
    LD d = a * a + 2.0L * e0, e = e0;
    int n = 0;
    for (int i = 0; i < 16; ++i) out[r * 16 + i] = 0.0;
    while (e / d >= (LD)tol) {
      if (n >= m - 1 || n >= 15) return false;   // the wrap-around step would be needed: use the FFT
      out[r * 16 + n] = (double)(e / d);
      const LD d1 = d - 2.0L * e * e / d, e1 = e * e / d;
      d = d1;
      e = e1;
      ++n;
    }
    out[r * 16 + 15] = (double)(1.0L / d);
    k[r] = n;
  }
  return true;
}

template void onestep_symbol<float>(const pdhg_problem&, double, double, float*);
template void onestep_symbol<double>(const pdhg_problem&, double, double, double*);

// DG P1 one-step preconditioner per Fourier mode m = 0..nx/2 over the cells, rows
// c0 = 1 (r = 0) and c0 = 3/2 (r = 1): K = (c0/h_t)^2 I + c^2 G G^*, with
// G(theta) = G_0 + G_-1 e^{-i theta} the unit-speed upwind P1 operator
// (G_0 = [7 3; -11 9] / (4 h_x), G_-1 = [5 -15; -1 3] / (4 h_x)); its Hermitian
// inverse [a b; conj(b) d] divided by nx (the inverse FFT's normalisation) as
// (a, Re b, Im b, d).  Computed in long double.
template <typename T>
void onestep_dg1_kinv(const pdhg_problem& p, double c, T* out) {
  typedef long double LD;
  const LD PI = 3.141592653589793238462643383279502884L;
  const int nx = p.nx, nm = nx / 2 + 1;
  const LD ht = (LD)p.t_final / p.nt, hx = (LD)p.length / nx, cc = c;
  const LD g0[2][2] = {{1.75L, 0.75L}, {-2.75L, 2.25L}}, gm[2][2] = {{1.25L, -3.75L}, {-0.25L, 0.75L}};
  for (int r = 0; r < 2; ++r) {
    const LD a0 = (r ? 1.5L : 1.0L) / ht;
    for (int m = 0; m < nm; ++m) {
      const LD th = 2.0L * PI * m / nx;
      const LD cr = (m == 0) ? 1.0L : (2 * m == nx ? -1.0L : cosl(th));
      const LD ci = (m == 0 || 2 * m == nx) ? 0.0L : -sinl(th);
      LD Gr[2][2], Gi[2][2];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          Gr[i][j] = (g0[i][j] + gm[i][j] * cr) / hx;
          Gi[i][j] = gm[i][j] * ci / hx;
        }
      // H = G G^*: H_ij = sum_k G_ik conj(G_jk)
      LD hr[2][2], hi[2][2];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          hr[i][j] = 0.0L;
          hi[i][j] = 0.0L;
          for (int k = 0; k < 2; ++k) {
            hr[i][j] += Gr[i][k] * Gr[j][k] + Gi[i][k] * Gi[j][k];
            hi[i][j] += Gi[i][k] * Gr[j][k] - Gr[i][k] * Gi[j][k];
          }
        }
      const LD ka = a0 * a0 + cc * cc * hr[0][0], kd = a0 * a0 + cc * cc * hr[1][1];
      const LD kbr = cc * cc * hr[0][1], kbi = cc * cc * hi[0][1];
      const LD det = ka * kd - (kbr * kbr + kbi * kbi);
      T* o = out + ((size_t)r * nm + m) * 4;
      o[0] = (T)(kd / (det * nx));
      o[1] = (T)(-kbr / (det * nx));
      o[2] = (T)(-kbi / (det * nx));
      o[3] = (T)(ka / (det * nx));
    }
  }
}

template void onestep_dg1_kinv<float>(const pdhg_problem&, double, float*);
template void onestep_dg1_kinv<double>(const pdhg_problem&, double, double*);

// Totals of a one-step march from its per-step records; the march stops after a diverged step.
OneStepSummary summarize_steps(const StepStat* rec, int nt, int64_t* step_iters, double* step_res) {
  OneStepSummary sm{0, 0.0, 0.0, PDHG_OK, nt};
  for (int l = 0; l < nt; ++l) {
    const bool ran = l < sm.done;
    if (ran) {
      sm.total += rec[l].iters;
      sm.rp = std::max(sm.rp, rec[l].rp);
      sm.rd = std::max(sm.rd, rec[l].rd);
      if (rec[l].status == 2) {
        sm.status = PDHG_DIVERGED;
        sm.done = l + 1;
      } else if (rec[l].status == 1 && sm.status == PDHG_OK) {
        sm.status = PDHG_NOT_CONVERGED;
      }
    }
    if (step_iters) step_iters[l] = ran ? rec[l].iters : 0;
    if (step_res) {
      step_res[2 * l] = ran ? rec[l].rp : NAN;
      step_res[2 * l + 1] = ran ? rec[l].rd : NAN;
    }
  }
  return sm;
}

template void build_factor_rows_shifts<float>(const pdhg_problem&, const std::vector<long double>&,
                                              std::vector<FacRow<float>>&, std::vector<int>&, std::vector<int>&);
template void build_factor_rows_shifts<double>(const pdhg_problem&, const std::vector<long double>&,
                                               std::vector<FacRow<double>>&, std::vector<int>&, std::vector<int>&);

}  // namespace pdhg

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct WsLayout {
  size_t u_alt, phi_alt, spec0, spec1, srow, phibar, part_rp, part_rd, scal, ctrl, ctrl_t, s0, ck_u, ck_phi, lam, lambar,
      adj, colchunk, total;
  int max_parts;
};

struct GraphKey {
  const void* u = nullptr;
  const void* phi = nullptr;
  const void* ws = nullptr;
  const void* hist = nullptr;
  double tau_u = 0, tau_phi = 0, lf = 0, c = 0;
  int variant = 0, chunk = 0;
  const void* lam_u0 = nullptr;   // multiplier form: the initial data (nullptr: u^0 fixed)
  double tau_u0 = 0, tau_lam = 0;
  bool operator==(const GraphKey& o) const {
    return u == o.u && phi == o.phi && ws == o.ws && hist == o.hist && tau_u == o.tau_u &&
           tau_phi == o.tau_phi && lf == o.lf && c == o.c && variant == o.variant && chunk == o.chunk &&
           lam_u0 == o.lam_u0 && tau_u0 == o.tau_u0 && tau_lam == o.tau_lam;
  }
};

}  // namespace

struct pdhg_handle {
  pdhg_problem prob{};
  int device = 0;
  int lqb = 4;
  size_t esz = 8;
  void* d_tw = nullptr;
  // preconditioner factors
  void* d_fac_rows = nullptr;
  int* d_fac_off = nullptr;
  int* d_fac_last = nullptr;
  double fac_c = -1.0, fac_g = -1.0;
  // chunked column solve (always FP64 arithmetic): per-mode, per-chunk maps, and for FP32 problems an
  // FP64 copy of the factor table
  double* d_cmap = nullptr;
  double* d_cpow = nullptr;
  int* d_ctiles = nullptr;      // the chunked solve's four tile lists (ChunkArgs::tiles)
  int ctoff[4] = {0, 0, 0, 0}, cntile[4] = {0, 0, 0, 0};
  int chunk_g64 = 0;            // column blocks below it run in FP64 when the spectrum is float
  void* d_f64_rows = nullptr;
  int* d_f64_off = nullptr;
  int* d_f64_last = nullptr;
  // single-precision preconditioner of an FP64 problem: float twiddles and factors
  void* d_tw32 = nullptr;
  void* d_vtab = nullptr;       // DG: per-mode 6x6 eigenbases of the coefficient coupling
  // resolved constants
  double lf = 0.0, c = 0.0;
  bool consts_valid = false;
  // own workspace
  void* own_ws = nullptr;
  size_t own_ws_bytes = 0;
  // host staging
  Ctrl* h_ctrl = nullptr;       // pinned, 2 slots
  double* h_scal = nullptr;     // pinned, 64 doubles
  double* scratch_dev = nullptr;   // this device's address of the static scratch array (pdhg_residual_static)
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;
  // graph cache
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  GraphKey gkey;
  // last solve (for kernel timing)
  GraphKey last;
  // mesh refinement in time: plans of the coarse levels, and two (u, phi) buffer pairs
  std::vector<std::pair<int, pdhg_handle*>> refine_sub;
  void* refine_buf = nullptr;
  size_t refine_buf_bytes = 0;
  // one-time-step solver: symbol table, per-step records, flag and problem table
  void* os_buf = nullptr;
  size_t os_buf_bytes = 0;
  double os_c = -1.0;
  // DG P1 one-step: one-level plans (c0 = 1, 3/2) for the step-size power iteration, and their (u, phi)
  pdhg_handle* os_sub[2] = {nullptr, nullptr};
  void* os_sub_buf = nullptr;
  std::string err;
};

namespace {

int set_hip_error(pdhg_handle* h, hipError_t e, const char* what) {
  if (h) {
    h->err = std::string(what) + ": " + hipGetErrorString(e);
  }
  return PDHG_EHIP;
}

#define HIP_TRY(expr)                                        \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return set_hip_error(h, e_, #expr); \
  } while (0)

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Coefficients per cell: 3 for DG P2, 1 for finite differences.
inline int planes(const pdhg_problem& p) {
  return p.space == PDHG_DG_P2_LLF ? 3 : (p.space == PDHG_DG_P1_UPWIND ? 2 : 1);
}
// Either DG discretisation (coefficient planes, per-mode eigenbasis in the column solve).
inline bool is_dg(const pdhg_problem& p) { return p.space == PDHG_DG_P2_LLF || p.space == PDHG_DG_P1_UPWIND; }
inline bool is_full(const pdhg_problem& p) { return p.precond_kind == PDHG_PRECOND_FULL; }
// FP64 state with the Gram preconditioner's spectral pass in single precision
inline bool is_pre32(const pdhg_problem& p) { return p.precond_kind == PDHG_PRECOND_GRAM_F32; }
// The Gram column solve of a finite-difference problem runs in chunks (N_t > 4096, N_x >= 16).
inline bool uses_chunks(const pdhg_problem& p) {
  return !is_dg(p) && !is_full(p) && p.nt >= kChunkMinNt && p.nx >= kChunkCols;
}

WsLayout layout_for(const pdhg_problem& p, size_t esz) {
  WsLayout L{};
  const size_t nx = (size_t)p.nx * planes(p), nt = (size_t)p.nt;
  const size_t field = align_up(nt * nx * esz);
  const size_t ufield = align_up((nt + 1) * nx * esz);
  // per-block partial sums of the element-wise kernels, or nt+1 level sums
  L.max_parts = (int)std::max((nt * nx + 255) / 256 + 256, nt + 1 + 256);
  size_t o = 0;
  L.u_alt = o; o += ufield;
  L.phi_alt = o; o += field;
  L.spec0 = o; o += field;
  L.spec1 = o; o += field;
  L.srow = o; o += field;
  L.phibar = o; o += field;
  L.part_rp = o; o += align_up(sizeof(double) * L.max_parts);
  L.part_rd = o; o += align_up(sizeof(double) * L.max_parts);
  L.scal = o; o += align_up(sizeof(double) * 64);
  L.ctrl = o; o += align_up(sizeof(Ctrl));
  L.ctrl_t = o; o += align_up(sizeof(Ctrl));     // control block used only by kernel timing
  L.s0 = o; o += align_up(sizeof(double) * nt);    // FP64 mode 0 of a float spectrum
  L.ck_u = o; o += ufield;                         // last-good checkpoint (u, phi) of the solve loop
  L.ck_phi = o; o += field;
  L.lam = o; o += align_up(nx * esz);              // multiplier of u^0 = u0 and its extrapolation
  L.lambar = o; o += align_up(nx * esz);
  L.adj = o;                                       // DG adjoint march: block rows and three levels of multipliers
  if (is_dg(p)) o += align_up(sizeof(double) * dg_adjoint_scratch_doubles(p.nx, planes(p)));
  L.colchunk = o;                                  // chunked column solve: pass-1 records and entering states
  if (uses_chunks(p)) o += align_up(sizeof(double) * 8 * (size_t)chunk_count(p.nt) * p.nx);
  L.total = o;
  return L;
}

Scheme scheme_of(const pdhg_handle* h) {
  const pdhg_problem& p = h->prob;
  Scheme s{};
  s.nx = p.nx;
  s.nt = p.nt;
  s.time = p.time;
  s.space = p.space;
  s.ht = p.t_final / p.nt;
  s.hx = p.length / p.nx;
  s.alpha = p.alpha;
  s.beta = p.beta;
  s.gamma = p.gamma;
  s.lf = h->lf;
  return s;
}

// Symbol parameters of the full-symbol preconditioner from the resolved constants.
FullSym full_sym_of(const pdhg_handle* h) {
  const pdhg_problem& p = h->prob;
  const double hx = p.length / p.nx;
  FullSym F{};
  F.inv_ht = p.nt / p.t_final;
  F.wr = (p.space == PDHG_FD_LF ? h->lf : h->c) / hx;
  F.vr = 2.0 * p.precond_gamma_hat / (hx * hx);
  F.ci = h->c / hx;
  F.bdf2 = p.time == PDHG_BDF2 ? 1 : 0;
  return F;
}

// Column blocks of the chunked solve whose recurrences run in FP64 when the
// spectrum is float: block g holds modes 8g .. 8g+7 (block 0: mode 0), and a
// mode whose shift s_k = c^2 mu_k + ghat^2 mu_k^2 is small against (1/h_t)^2
// (s_k h_t^2 < 1e-2) decays slowly along t: its part of s is large and smooth
// in t, and the primal step differences it in time, which amplifies float
// rounding of its recurrences.  Returns the first block whose lowest mode is
// past that bound (N_x / 16 if none is).
int chunk_fp64_blocks(const pdhg_problem& p, double c, double ghat) {
  const double PI = 3.141592653589793;
  const double ht = p.t_final / p.nt, hx = p.length / p.nx;
  const int nblocks = p.nx / kChunkCols;
  for (int g = 1; g < nblocks; ++g) {
    const double sn = std::sin(PI * (8 * g) / p.nx);
    const double mu = 4.0 * sn * sn / (hx * hx);
    if ((c * c * mu + ghat * ghat * mu * mu) * ht * ht >= 1e-2) return g;
  }
  return nblocks;
}

// FP64 factor rows of the chunked column solve: the factor table of an FP64
// problem, the FP64 copy of an FP32 problem's.
FacTab<double> chunk_rows(const pdhg_handle* h) {
  if (h->d_f64_rows) return FacTab<double>{(const FacRow<double>*)h->d_f64_rows, h->d_f64_off, h->d_f64_last};
  return FacTab<double>{(const FacRow<double>*)h->d_fac_rows, h->d_fac_off, h->d_fac_last};
}

// The chunked solve's tiles (g nchunk + c) in the order of its four grids: FP64 recurrences on blocks g < n64
// (general, then constant), float on the others (likewise).  A tile is constant when its chunk is full and
// lies past the last distinct row of every column's mode in the table of its grid (last64: the FP64 rows,
// last32: the float rows of an FP32 problem, else empty).
static void chunk_tile_lists(const pdhg_problem& p, int g64, const std::vector<int>& last64,
                             const std::vector<int>& last32, std::vector<int>& tiles, int toff[4], int ntile[4]) {
  const int nblocks = p.nx / kChunkCols, nch = chunk_count(p.nt);
  const int n64 = last32.empty() ? nblocks : std::min(g64, nblocks);
  std::vector<int> lists[4];
  for (int g = 0; g < nblocks; ++g) {
    const bool f64 = g < n64;
    const std::vector<int>& lst = f64 ? last64 : last32;
    int ml = 0;
    for (int j = g * kChunkCols; j < (g + 1) * kChunkCols; ++j) {
      const int k = j == 0 ? 0 : (j == 1 ? p.nx / 2 : j >> 1);
      ml = std::max(ml, lst[k]);
    }
    for (int c = 0; c < nch; ++c) {
      const bool cst = c * kChunkLevels >= ml && (c + 1) * kChunkLevels <= p.nt;
      lists[(f64 ? 0 : 2) + (cst ? 1 : 0)].push_back(g * nch + c);
    }
  }
  tiles.clear();
  for (int k = 0; k < 4; ++k) {
    toff[k] = (int)tiles.size();
    ntile[k] = (int)lists[k].size();
    tiles.insert(tiles.end(), lists[k].begin(), lists[k].end());
  }
}

template <typename T>
int upload_factors(pdhg_handle* h, double c, double ghat) {
  std::vector<FacRow<T>> rows;
  std::vector<int> off, last;
  build_factor_rows<T>(h->prob, c, ghat, rows, off, last);
  if (h->d_fac_rows) hipFree(h->d_fac_rows);
  if (h->d_fac_off) hipFree(h->d_fac_off);
  if (h->d_fac_last) hipFree(h->d_fac_last);
  h->d_fac_rows = nullptr;
  h->d_fac_off = h->d_fac_last = nullptr;
  HIP_TRY(hipMalloc(&h->d_fac_rows, rows.size() * sizeof(FacRow<T>)));
  HIP_TRY(hipMalloc((void**)&h->d_fac_off, off.size() * sizeof(int)));
  HIP_TRY(hipMalloc((void**)&h->d_fac_last, last.size() * sizeof(int)));
  HIP_TRY(hipMemcpy(h->d_fac_rows, rows.data(), rows.size() * sizeof(FacRow<T>), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_fac_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_fac_last, last.data(), last.size() * sizeof(int), hipMemcpyHostToDevice));
  if (h->d_cmap) hipFree(h->d_cmap);
  if (h->d_cpow) hipFree(h->d_cpow);
  if (h->d_ctiles) hipFree(h->d_ctiles);
  if (h->d_f64_rows) hipFree(h->d_f64_rows);
  if (h->d_f64_off) hipFree(h->d_f64_off);
  if (h->d_f64_last) hipFree(h->d_f64_last);
  h->d_cmap = nullptr;
  h->d_cpow = nullptr;
  h->d_ctiles = nullptr;
  h->d_f64_rows = nullptr;
  h->d_f64_off = h->d_f64_last = nullptr;
  if (uses_chunks(h->prob)) {   // the chunked column solve: FP64 rows and their maps
    std::vector<int> l64 = last;   // the FP64 rows' last distinct rows
    if (sizeof(T) != sizeof(double)) {
      std::vector<FacRow<double>> r64;
      std::vector<int> o64;
      build_factor_rows<double>(h->prob, c, ghat, r64, o64, l64);
      HIP_TRY(hipMalloc(&h->d_f64_rows, r64.size() * sizeof(FacRow<double>)));
      HIP_TRY(hipMalloc((void**)&h->d_f64_off, o64.size() * sizeof(int)));
      HIP_TRY(hipMalloc((void**)&h->d_f64_last, l64.size() * sizeof(int)));
      HIP_TRY(hipMemcpy(h->d_f64_rows, r64.data(), r64.size() * sizeof(FacRow<double>), hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(h->d_f64_off, o64.data(), o64.size() * sizeof(int), hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(h->d_f64_last, l64.data(), l64.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    const int nmodes = h->prob.nx / 2 + 1;
    h->chunk_g64 = chunk_fp64_blocks(h->prob, c, ghat);
    HIP_TRY(hipMalloc((void**)&h->d_cmap, sizeof(double) * 12 * (size_t)nmodes * chunk_count(h->prob.nt)));
    HIP_TRY(launch_colchunk_maps<double>(chunk_rows(h), h->prob.time == PDHG_BDF2 ? 2 : 1, h->prob.nt, nmodes,
                                         h->d_cmap, nullptr));
    HIP_TRY(hipMalloc((void**)&h->d_cpow, sizeof(double) * 4 * kChunkPow * (size_t)nmodes));
    HIP_TRY(launch_colchunk_powers(chunk_rows(h), h->prob.time == PDHG_BDF2 ? 2 : 1, nmodes, h->d_cpow, nullptr));
    std::vector<int> tiles;
    chunk_tile_lists(h->prob, h->chunk_g64, l64, sizeof(T) == sizeof(double) ? std::vector<int>() : last, tiles,
                     h->ctoff, h->cntile);
    HIP_TRY(hipMalloc((void**)&h->d_ctiles, sizeof(int) * tiles.size()));
    HIP_TRY(hipMemcpy(h->d_ctiles, tiles.data(), sizeof(int) * tiles.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipStreamSynchronize(nullptr));
  }
  h->fac_c = c;
  h->fac_g = ghat;
  return PDHG_OK;
}

// Eigen-decomposition of the leading n x n block (n <= 6) of a real symmetric
// matrix by cyclic Jacobi rotations (long double): A = V diag(w) V^T, columns
// of V the eigenvectors.
void jacobi6(long double A[6][6], long double V[6][6], long double w[6], int n = 6) {
  typedef long double LD;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) V[i][j] = (i == j) ? 1.0L : 0.0L;
  LD scale = 0.0L;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) scale += A[i][j] * A[i][j];
  for (int sweep = 0; sweep < 100; ++sweep) {
    LD off = 0.0L;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p][q] * A[p][q];
    if (off <= 1e-36L * scale) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (A[p][q] == 0.0L) continue;
        const LD th = (A[q][q] - A[p][p]) / (2.0L * A[p][q]);
        const LD t = (th >= 0.0L ? 1.0L : -1.0L) / (fabsl(th) + sqrtl(th * th + 1.0L));
        const LD c = 1.0L / sqrtl(t * t + 1.0L), sn = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const LD akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const LD apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const LD vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - sn * vkq;
          V[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < 6; ++i) w[i] = i < n ? A[i][i] : 0.0L;
}

// DG preconditioner data: for each Fourier mode m = 0..nx/2 over the cells, the
// unit-speed upwind DG symbol G(theta) = G_0 + G_-1 e^{-i theta} (theta = 2 pi m / nx)
// of the NP coefficient planes, the Hermitian coupling H = c^2 G G^*, and the
// eigen-decomposition of its real 2NP x 2NP form [Re H, -Im H; Im H, Re H] (acting
// on (Re, Im) of the planes).
//   P2 Legendre: G_0 = [1 1 1; -3 3 3; 5 -5 5] / h_x, G_-1 = [-1 -1 -1; 3 3 3; -5 -5 -5] / h_x.
//   P1 nodal:    G_0 = [7 3; -11 9] / (4 h_x), G_-1 = [5 -15; -1 3] / (4 h_x)
//                (minus the printed A_1, A_2 of Section 3.2.2 at unit speed).
// Uploads the factor tables of B_t B_t^T + lambda (6 per mode, the unused ones
// with lambda = 0 for P1) and the eigenvector matrices (36 values per mode, row
// stride 6).
template <typename T>
int upload_factors_dg(pdhg_handle* h, double c) {
  typedef long double LD;
  const int nx = h->prob.nx, nmodes = nx / 2 + 1;
  const int np = planes(h->prob), n2 = 2 * np;
  const LD hx = (LD)h->prob.length / nx, PI = 3.141592653589793238462643383279502884L;
  LD g0[3][3] = {{1, 1, 1}, {-3, 3, 3}, {5, -5, 5}};
  LD gm[3][3] = {{-1, -1, -1}, {3, 3, 3}, {-5, -5, -5}};
  if (np == 2) {
    const LD a0[2][2] = {{1.75L, 0.75L}, {-2.75L, 2.25L}}, am[2][2] = {{1.25L, -3.75L}, {-0.25L, 0.75L}};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        g0[a][b] = (a < 2 && b < 2) ? a0[a][b] : 0.0L;
        gm[a][b] = (a < 2 && b < 2) ? am[a][b] : 0.0L;
      }
  }
  std::vector<long double> shifts((size_t)nmodes * 6);
  std::vector<T> vtab((size_t)nmodes * 36);
  for (int m = 0; m < nmodes; ++m) {
    // e^{-i theta}; exactly real for the real modes 0 and nx/2
    const LD th = 2.0L * PI * m / nx;
    const LD cr = (m == 0) ? 1.0L : (2 * m == nx ? -1.0L : cosl(th));
    const LD ci = (m == 0 || 2 * m == nx) ? 0.0L : -sinl(th);
    LD Gr[3][3], Gi[3][3];
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < np; ++b) {
        Gr[a][b] = (g0[a][b] + gm[a][b] * cr) / hx;
        Gi[a][b] = (gm[a][b] * ci) / hx;
      }
    LD A[6][6] = {}, V[6][6], w[6];
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < np; ++b) {
        LD hr = 0.0L, hi = 0.0L;   // (G G^*)_ab = sum_k G_ak conj(G_bk)
        for (int k = 0; k < np; ++k) {
          hr += Gr[a][k] * Gr[b][k] + Gi[a][k] * Gi[b][k];
          hi += Gi[a][k] * Gr[b][k] - Gr[a][k] * Gi[b][k];
        }
        hr *= (LD)c * c;
        hi *= (LD)c * c;
        A[a][b] = hr;
        A[a + np][b + np] = hr;
        A[a][b + np] = -hi;
        A[a + np][b] = hi;
      }
    jacobi6(A, V, w, n2);
    for (int b = 0; b < 6; ++b) shifts[(size_t)m * 6 + b] = w[b] > 0.0L ? w[b] : 0.0L;
    for (int r = 0; r < 6; ++r)
      for (int b = 0; b < 6; ++b) vtab[(size_t)m * 36 + r * 6 + b] = (T)V[r][b];
  }
  std::vector<FacRow<T>> rows;
  std::vector<int> off, last;
  build_factor_rows_shifts<T>(h->prob, shifts, rows, off, last);
  if (h->d_fac_rows) hipFree(h->d_fac_rows);
  if (h->d_fac_off) hipFree(h->d_fac_off);
  if (h->d_fac_last) hipFree(h->d_fac_last);
  if (h->d_vtab) hipFree(h->d_vtab);
  h->d_fac_rows = h->d_vtab = nullptr;
  h->d_fac_off = h->d_fac_last = nullptr;
  HIP_TRY(hipMalloc(&h->d_fac_rows, rows.size() * sizeof(FacRow<T>)));
  HIP_TRY(hipMalloc((void**)&h->d_fac_off, off.size() * sizeof(int)));
  HIP_TRY(hipMalloc((void**)&h->d_fac_last, last.size() * sizeof(int)));
  HIP_TRY(hipMalloc(&h->d_vtab, vtab.size() * sizeof(T)));
  HIP_TRY(hipMemcpy(h->d_fac_rows, rows.data(), rows.size() * sizeof(FacRow<T>), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_fac_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_fac_last, last.data(), last.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->d_vtab, vtab.data(), vtab.size() * sizeof(T), hipMemcpyHostToDevice));
  h->fac_c = c;
  h->fac_g = 0.0;
  return PDHG_OK;
}

template <typename T>
int upload_twiddles(pdhg_handle* h, void** dst) {
  const int n = h->prob.nx;
  std::vector<C2<T>> tw(n);
  const long double PI = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    const long double a = -2.0L * PI * i / n;
    tw[i] = C2<T>{(T)cosl(a), (T)sinl(a)};
  }
  HIP_TRY(hipMalloc(dst, n * sizeof(C2<T>)));
  HIP_TRY(hipMemcpy(*dst, tw.data(), n * sizeof(C2<T>), hipMemcpyHostToDevice));
  return PDHG_OK;
}

template <typename T>
FacTab<T> factab(const pdhg_handle* h) {
  return FacTab<T>{(const FacRow<T>*)h->d_fac_rows, h->d_fac_off, h->d_fac_last};
}

int ensure_workspace(pdhg_handle* h, void*& ws) {
  if (ws) return PDHG_OK;
  const WsLayout L = layout_for(h->prob, h->esz);
  if (!h->own_ws || h->own_ws_bytes < L.total) {
    if (h->own_ws) hipFree(h->own_ws);
    h->own_ws = nullptr;
    HIP_TRY(hipMalloc(&h->own_ws, L.total));
    h->own_ws_bytes = L.total;
  }
  ws = h->own_ws;
  return PDHG_OK;
}

inline char* wsp(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

// Arguments of the chunked column solve with its work buffer in workspace ws: FP64 rows for every block,
// and for a float state the float rows of the blocks at and above chunk_g64.
ChunkArgs chunk_args(const pdhg_handle* h, void* ws) {
  ChunkArgs a{};
  a.f64 = chunk_rows(h);
  if (h->prob.dtype == PDHG_F32) a.f32 = factab<float>(h);
  a.cmap = h->d_cmap;
  a.cpow = h->d_cpow;
  a.tiles = h->d_ctiles;
  for (int k = 0; k < 4; ++k) {
    a.toff[k] = h->ctoff[k];
    a.ntile[k] = h->cntile[k];
  }
  a.cwork = (double*)wsp(ws, layout_for(h->prob, h->esz).colchunk);
  a.nchunk = chunk_count(h->prob.nt);
  a.g64 = h->chunk_g64;
  return a;
}

// max |f'(u0)| on the device, read back (synchronous).  part: >= 64 doubles of device scratch.
template <typename T>
int max_abs_dflux(pdhg_handle* h, const T* u0, double* part, hipStream_t st, double* out) {
  if (h->prob.space == PDHG_DG_P2_LLF)   // DG: over the cell-edge traces of u0_h
    HIP_TRY(launch_dg_maxabs_trace<T>(u0, h->prob.nx, 2.0 * h->prob.alpha, h->prob.beta, part, st));
  else if (h->prob.space == PDHG_DG_P1_UPWIND)   // over the nodal values and edge traces
    HIP_TRY(launch_dg1_maxabs<T>(u0, h->prob.nx, 2.0 * h->prob.alpha, h->prob.beta, part, st));
  else
    HIP_TRY(launch_maxabs_dflux<T>(u0, (size_t)h->prob.nx, 2.0 * h->prob.alpha, h->prob.beta, part, st));
  HIP_TRY(hipMemcpyAsync(h->h_scal, part, 64 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double m = 0.0;
  for (int i = 0; i < 64; ++i) m = std::max(m, h->h_scal[i]);
  *out = m;
  return PDHG_OK;
}

// Resolve lf_speed and c from u0 when they default (part: >= 64 doubles of
// device scratch); with factors, also (re)build the banded factor tables.
template <typename T>
int resolve_constants_p(pdhg_handle* h, const T* u0, double* part, hipStream_t st, bool factors) {
  const pdhg_problem& p = h->prob;
  double lf = p.lf_speed, c = p.precond_c;
  if ((p.space == PDHG_FD_LF && lf < 0.0) || (c < 0.0 && !is_full(p))) {
    double m = 0.0;
    int rc = max_abs_dflux<T>(h, u0, part, st, &m);
    if (rc) return rc;
    if (lf < 0.0) lf = m;
    if (c < 0.0 && !is_full(p)) c = m;
  }
  if (c < 0.0 && is_full(p)) {   // the signed mean speed: f'(mean u0) = 2 alpha mean(u0) + beta
    HIP_TRY(launch_level_sums<T>(u0, p.nx, (size_t)p.nx, 1, part, st));
    HIP_TRY(hipMemcpyAsync(h->h_scal, part, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    c = 2.0 * p.alpha * h->h_scal[0] / p.nx + p.beta;
  }
  if (p.space != PDHG_FD_LF) lf = 0.0;
  h->lf = lf;
  h->c = c;
  h->consts_valid = true;
  if (!factors || is_full(p)) return PDHG_OK;   // the full symbol needs no factor tables
  if (is_dg(p)) {
    if (!h->d_fac_rows || h->fac_c != c) {
      int rc = upload_factors_dg<T>(h, c);
      if (rc) return rc;
    }
  } else if (!h->d_fac_rows || h->fac_c != c || h->fac_g != p.precond_gamma_hat) {
    int rc = upload_factors<T>(h, c, p.precond_gamma_hat);
    if (rc) return rc;
  }
  return PDHG_OK;
}

template <typename T>
int resolve_constants(pdhg_handle* h, const T* u0, void* ws, hipStream_t st) {
  const WsLayout L = layout_for(h->prob, h->esz);
  return resolve_constants_p<T>(h, u0, (double*)wsp(ws, L.part_rp), st, true);
}

// Column solve (Gram or full-symbol preconditioner).  With part != NULL it
// also reduces the iteration's residual partial sums (nparts per norm) and
// takes the stopping decision, in the first wavefront of block 0.
template <typename T>
hipError_t colsolve_any(pdhg_handle* h, void* ws, T* spec, Ctrl* ctrl, const double* part, int nparts,
                        double* hist, hipStream_t st) {
  const pdhg_problem& p = h->prob;
  const int bw = p.time == PDHG_BDF2 ? 2 : 1;
  const double wscale = (p.t_final / p.nt) * (p.length / p.nx);
  if (is_full(p))   // nt <= 1024 (checked at set-up)
    return launch_colsolve_full<T>(spec, full_sym_of(h), h->d_tw, p.nt, p.nx, h->lqb, ctrl, part, nparts, wscale,
                                   hist, st);
  if (uses_chunks(p) && h->d_cmap)
    return launch_colsolve_chunk<T>(spec, chunk_args(h, ws), bw, p.nt, p.nx, h->lqb, ctrl, part, nparts, wscale,
                                    hist, st);
  return launch_colsolve_wave<T>(spec, factab<T>(h), bw, p.nt, p.nx, h->lqb, ctrl, part, nparts, wscale, hist, st);
}

// s = K_d^{-1} r through the workspace spectrum buffer spec.
template <typename T>
int precond_apply(pdhg_handle* h, void* ws, const T* r, T* s, T* spec, hipStream_t st) {
  const pdhg_problem& p = h->prob;
  if (is_dg(p)) {   // planes x nt coefficient rows; per-mode eigenbasis in the column solve
    const int nr = planes(p) * p.nt;
    HIP_TRY(launch_rows_fwd<T>(r, nr, spec, nr, h->lqb, p.nx, h->d_tw, nullptr, st));
    HIP_TRY(launch_dg_colsolve<T>(spec, factab<T>(h), (const T*)h->d_vtab, p.time == PDHG_BDF2 ? 2 : 1, p.nt, p.nx,
                                  h->lqb, nullptr, st, planes(p)));
    HIP_TRY(launch_rows_inv<T>(spec, nr, h->lqb, s, nr, p.nx, h->d_tw, nullptr, st));
    return PDHG_OK;
  }
  HIP_TRY(launch_rows_fwd<T>(r, p.nt, spec, p.nt, h->lqb, p.nx, h->d_tw, nullptr, st));
  HIP_TRY(colsolve_any<T>(h, ws, spec, nullptr, nullptr, 0, nullptr, st));
  HIP_TRY(launch_rows_inv<T>(spec, p.nt, h->lqb, s, p.nt, p.nx, h->d_tw, nullptr, st));
  return PDHG_OK;
}

// Largest eigenvalue of J(u)^T K_d^{-1} J(u) at u^l = u0 by power iteration.
template <typename T>
int power_iteration(pdhg_handle* h, const T* u, void* ws, hipStream_t st, int iters, double* nu) {
  const pdhg_problem& p = h->prob;
  const WsLayout L = layout_for(p, h->esz);
  const Scheme s = scheme_of(h);
  const bool dg = is_dg(p);
  const size_t n = (size_t)p.nt * p.nx * planes(p);
  T* v = (T*)wsp(ws, L.srow);
  T* w = (T*)wsp(ws, L.phibar);
  T* t = (T*)wsp(ws, L.spec1);
  T* spec = (T*)wsp(ws, L.spec0);
  double* part = (double*)wsp(ws, L.part_rp);
  double* scal = (double*)wsp(ws, L.scal);
  // deterministic start vector (xorshift64)
  std::vector<T> hv(n);
  unsigned long long x = 0x9E3779B97F4A7C15ull;
  for (size_t i = 0; i < n; ++i) {
    x ^= x << 13; x ^= x >> 7; x ^= x << 17;
    hv[i] = (T)((double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5);
  }
  HIP_TRY(hipMemcpyAsync(v, hv.data(), n * sizeof(T), hipMemcpyHostToDevice, st));
  HIP_TRY(launch_dot<T>(v, nullptr, n, part, scal, st));
  HIP_TRY(launch_normalize<T>(v, n, scal, st));
  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    if (dg) HIP_TRY(dgx_apply_j<T>(s, u, v, w, st));             // w = J v
    else HIP_TRY(launch_apply_j<T>(s, u, v, w, st));
    int rc = precond_apply<T>(h, ws, w, w, spec, st);                 // w = K_d^{-1} w
    if (rc) return rc;
    if (dg) HIP_TRY(dgx_apply_jt<T>(s, u, w, t, nullptr, st, nullptr));         // t = J^T w
    else HIP_TRY(launch_apply_jt<T>(s, u, w, t, nullptr, st, nullptr));
    HIP_TRY(launch_dot<T>(t, v, n, part, scal, st));             // scal[0] = <t, v>
    HIP_TRY(launch_dot<T>(t, nullptr, n, part, scal + 1, st));   // scal[1] = |t|^2
    HIP_TRY(launch_normalize<T>(t, n, scal + 1, st));
    std::swap(v, t);
  }
  HIP_TRY(hipMemcpyAsync(h->h_scal, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  lam = h->h_scal[0];
  *nu = lam;
  return PDHG_OK;
}

}  // namespace

// =================================================================== C ABI
// ------------------------------------------------------------------ static scratch
// Device memory of the allocation-free entry point pdhg_residual_static: a
// file-scope array that every GPU the library runs on holds until the process
// ends.  Layout (doubles): [0, 64) partial maxima for the default constants,
// then kStaticParts partial sums of ||A(u)||^2, kStaticParts of ||J^T phi||^2,
// and the two reduced sums.  In host code `scratch` is only a stand-in for the
// symbol: its device address is taken once per device with hipGetSymbolAddress
// (with that device current) and kept in the handle.
constexpr int kStaticParts = 262080;   // one partial sum per 256 points: nt * nx <= 67,092,480
constexpr size_t kStaticScratchDoubles = 524288;   // 4 MiB
static_assert(64 + 2 * (size_t)kStaticParts + 2 <= kStaticScratchDoubles, "static scratch layout");
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxScratchDevices] = {};

// Address of `scratch` on the current device `device` (looked up once per device).
int static_scratch_address(pdhg_handle* h, int device) {
  if (device < 0 || device >= kMaxScratchDevices) return PDHG_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return set_hip_error(h, e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[device] = static_cast<double*>(ptr);
  }
  h->scratch_dev = g_scratch_dev[device];
  return PDHG_OK;
}

// out[0] = sum a[0..na), out[1] = sum b[0..nb): one block of 256 threads, each
// adding its strided share in index order, then a fixed-order tree in LDS.
__global__ void __launch_bounds__(256) k_static_sums(const double* __restrict__ a, int na,
                                                     const double* __restrict__ b, int nb, double* out) {
  __shared__ double ra[256], rb[256];
  const int t = threadIdx.x;
  double sa = 0.0, sb = 0.0;
  for (int i = t; i < na; i += 256) sa += a[i];
  for (int i = t; i < nb; i += 256) sb += b[i];
  ra[t] = sa;
  rb[t] = sb;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      ra[t] += ra[t + w];
      rb[t] += rb[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = ra[0];
    out[1] = rb[0];
  }
}

// pdhg_residual without allocation: the partial sums live in the static
// scratch, the constants are resolved without building factor tables, and
// the norms are reduced on the device.
template <typename T>
int residual_static_impl(pdhg_handle* h, const T* u, const T* phi, T* Au, T* JTphi, double* res, hipStream_t st) {
  const pdhg_problem& p = h->prob;
  const size_t nparts = ((size_t)p.nt * p.nx + 255) / 256;
  if (nparts > (size_t)kStaticParts) {
    // h->err has capacity reserved at set-up: this assignment does not allocate
    h->err.assign("pdhg_residual_static: nt * nx exceeds the static scratch (at most 67092480 points)");
    return PDHG_EINVAL;
  }
  double* part_c = h->scratch_dev;
  double* prp = part_c + 64;
  double* prd = prp + kStaticParts;
  double* sums = prd + kStaticParts;
  if (!h->consts_valid) {
    const int rc = resolve_constants_p<T>(h, u, part_c, st, false);
    if (rc) return rc;
  }
  const Scheme s = scheme_of(h);
  int nb1 = 0, nb2 = 0;
  if (is_dg(p)) {
    HIP_TRY(dgx_residual<T>(s, u, Au, prp, nullptr, st, &nb1));
    if (phi) HIP_TRY(dgx_apply_jt<T>(s, u, phi, JTphi, prd, st, &nb2));
  } else {
    HIP_TRY(launch_residual<T>(s, u, Au, prp, nullptr, st, &nb1));
    if (phi) HIP_TRY(launch_apply_jt<T>(s, u, phi, JTphi, prd, st, &nb2));
  }
  if ((size_t)nb1 != nparts || (phi && (size_t)nb2 != nparts)) return PDHG_EUNSUPPORTED;
  if (res) {
    hipLaunchKernelGGL(k_static_sums, dim3(1), dim3(256), 0, st, prp, nb1, prd, nb2, sums);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h->h_scal, sums, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    res[0] = std::sqrt(s.ht * s.hx * h->h_scal[0]);
    res[1] = phi ? std::sqrt(s.ht * s.hx * h->h_scal[1]) : 0.0;
  }
  return PDHG_OK;
}
}  // namespace

extern "C" {

const char* pdhg_status_string(int status) {
  switch (status) {
    case PDHG_OK: return "converged";
    case PDHG_NOT_CONVERGED: return "max_iter reached";
    case PDHG_DIVERGED: return "diverged";
    case PDHG_STALLED: return "stalled at the rounding floor";
    case PDHG_EINVAL: return "invalid argument";
    case PDHG_EHIP: return "HIP error";
    case PDHG_EUNSUPPORTED: return "unsupported";
    case PDHG_EWORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

const char* pdhg_last_error(const pdhg_handle* h) { return h ? h->err.c_str() : "null handle"; }

int pdhg_setup(const pdhg_problem* prob, pdhg_handle** out) {
  if (!prob || !out) return PDHG_EINVAL;
  *out = nullptr;
  const pdhg_problem& p = *prob;
  if (!is_pow2(p.nx) || p.nx < 8 || p.nx > 4096 || p.nt < 1) return PDHG_EINVAL;
  if (!(p.length > 0) || !(p.t_final > 0) || p.gamma < 0 || p.precond_gamma_hat < 0) return PDHG_EINVAL;
  if (p.time != PDHG_BE && p.time != PDHG_BDF2) return PDHG_EINVAL;
  if (p.space != PDHG_FD_UPWIND && p.space != PDHG_FD_LF && !is_dg(p)) return PDHG_EINVAL;
  if (p.dtype != PDHG_F32 && p.dtype != PDHG_F64) return PDHG_EINVAL;
  if (p.nt > 8192) return PDHG_EUNSUPPORTED;   // column solve: <= 8 wavefronts of 64 x 16 levels per column
  // DG: nx cells >= 16 (8 spectrum columns per column block), nt <= 512 (8 levels per lane), no viscosity
  if (is_dg(p) && (p.nx < 16 || p.nt > 512 || p.gamma != 0.0)) return PDHG_EUNSUPPORTED;
  if (p.precond_kind != PDHG_PRECOND_GRAM && p.precond_kind != PDHG_PRECOND_FULL && !is_pre32(p))
    return PDHG_EINVAL;
  // single-precision preconditioner: FP64 finite-difference problems
  if (is_pre32(p) && (p.dtype != PDHG_F64 || is_dg(p))) return PDHG_EUNSUPPORTED;
  // full symbol: finite differences, one wavefront per mode in the column solve (nt <= 1024)
  if (is_full(p) && (is_dg(p) || p.nt > 1024)) return PDHG_EUNSUPPORTED;
  pdhg_handle* h = new (std::nothrow) pdhg_handle();
  if (!h) return PDHG_EINVAL;
  h->prob = p;
  h->esz = (p.dtype == PDHG_F64) ? 8 : 4;
  h->lqb = 0;
  while ((1 << (h->lqb + 1)) <= std::min(16, p.nx)) ++h->lqb;
  h->err.reserve(256);   // messages set by the allocation-free entry point fit without reallocation
  int rc = PDHG_OK;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) rc = set_hip_error(h, e, "hipGetDevice");
  if (!rc) rc = static_scratch_address(h, h->device);
  if (!rc) rc = (p.dtype == PDHG_F64) ? upload_twiddles<double>(h, &h->d_tw) : upload_twiddles<float>(h, &h->d_tw);
  if (!rc && is_pre32(p)) rc = upload_twiddles<float>(h, &h->d_tw32);
  if (!rc && (e = hipHostMalloc((void**)&h->h_ctrl, 2 * sizeof(Ctrl), hipHostMallocDefault)) != hipSuccess)
    rc = set_hip_error(h, e, "hipHostMalloc");
  if (!rc && (e = hipHostMalloc((void**)&h->h_scal, 64 * sizeof(double), hipHostMallocDefault)) != hipSuccess)
    rc = set_hip_error(h, e, "hipHostMalloc");
  for (int i = 0; i < 2 && !rc; ++i)
    if ((e = hipEventCreateWithFlags(&h->ev[i], hipEventDisableTiming)) != hipSuccess)
      rc = set_hip_error(h, e, "hipEventCreate");
  if (!rc && (e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking)) != hipSuccess)
    rc = set_hip_error(h, e, "hipStreamCreate");
  if (rc) {
    pdhg_destroy(h);
    return rc;
  }
  *out = h;
  return PDHG_OK;
}

size_t pdhg_workspace_bytes(const pdhg_handle* h) { return h ? layout_for(h->prob, h->esz).total : 0; }

void pdhg_destroy(pdhg_handle* h) {
  if (!h) return;
  for (auto& kv : h->refine_sub) pdhg_destroy(kv.second);
  if (h->refine_buf) hipFree(h->refine_buf);
  if (h->os_buf) hipFree(h->os_buf);
  for (int i = 0; i < 2; ++i) pdhg_destroy(h->os_sub[i]);
  if (h->os_sub_buf) hipFree(h->os_sub_buf);
  if (h->gexec) hipGraphExecDestroy(h->gexec);
  if (h->graph) hipGraphDestroy(h->graph);
  if (h->d_tw) hipFree(h->d_tw);
  if (h->d_fac_rows) hipFree(h->d_fac_rows);
  if (h->d_fac_off) hipFree(h->d_fac_off);
  if (h->d_fac_last) hipFree(h->d_fac_last);
  if (h->d_cmap) hipFree(h->d_cmap);
  if (h->d_cpow) hipFree(h->d_cpow);
  if (h->d_ctiles) hipFree(h->d_ctiles);
  if (h->d_f64_rows) hipFree(h->d_f64_rows);
  if (h->d_f64_off) hipFree(h->d_f64_off);
  if (h->d_f64_last) hipFree(h->d_f64_last);
  if (h->d_tw32) hipFree(h->d_tw32);
  if (h->d_vtab) hipFree(h->d_vtab);
  if (h->own_ws) hipFree(h->own_ws);
  if (h->h_ctrl) hipHostFree(h->h_ctrl);
  if (h->h_scal) hipHostFree(h->h_scal);
  for (int i = 0; i < 2; ++i)
    if (h->ev[i]) hipEventDestroy(h->ev[i]);
  if (h->cap_stream) hipStreamDestroy(h->cap_stream);
  delete h;
}

}  // extern "C"

namespace {

// One unfused loop body (iteration n = ctrl->n_done + 1); `odd` selects the
// ping-pong direction of u: odd n reads u and writes u_alt.
template <typename T>
int enqueue_body_unfused(pdhg_handle* h, bool odd, T* u, T* phi, void* ws, T tau_u, T tau_phi, double* hist,
                         hipStream_t st) {
  const pdhg_problem& p = h->prob;
  const WsLayout L = layout_for(p, h->esz);
  const Scheme s = scheme_of(h);
  T* u_alt = (T*)wsp(ws, L.u_alt);
  T* spec = (T*)wsp(ws, L.spec0);
  T* srow = (T*)wsp(ws, L.srow);
  T* phibar = (T*)wsp(ws, L.phibar);
  double* prp = (double*)wsp(ws, L.part_rp);
  double* prd = (double*)wsp(ws, L.part_rd);
  Ctrl* ctrl = (Ctrl*)wsp(ws, L.ctrl);
  T* uin = odd ? u : u_alt;
  T* uout = odd ? u_alt : u;
  const size_t n = (size_t)p.nt * p.nx;
  int nb_rd = 0, nb_rp = 0;
  HIP_TRY(launch_rows_inv<T>(spec, p.nt, h->lqb, srow, p.nt, p.nx, h->d_tw, ctrl, st));
  HIP_TRY(launch_dual<T>(phi, phibar, srow, n, tau_phi, ctrl, st));
  HIP_TRY(launch_primal<T>(s, uin, uout, phibar, phi, tau_u, prd, ctrl, st, &nb_rd));
  HIP_TRY(launch_residual<T>(s, uout, srow, prp, ctrl, st, &nb_rp));
  HIP_TRY(launch_rows_fwd<T>(srow, p.nt, spec, p.nt, h->lqb, p.nx, h->d_tw, ctrl, st));
  HIP_TRY(colsolve_any<T>(h, ws, spec, ctrl, nullptr, 0, nullptr, st));
  HIP_TRY(launch_finalize(ctrl, prp, nb_rp, prd, nb_rd, s.ht * s.hx, hist, st));
  return PDHG_OK;
}

// One fused loop body: A (inverse FFT + dual step), B (primal step, residual,
// forward FFT, norms, stopping decision), C (column solve).
template <typename T>
int enqueue_body_fused(pdhg_handle* h, bool odd, T* u, T* phi, void* ws, T tau_u, T tau_phi, double* hist,
                       hipStream_t st) {
  const pdhg_problem& p = h->prob;
  const WsLayout L = layout_for(p, h->esz);
  const Scheme s = scheme_of(h);
  T* u_alt = (T*)wsp(ws, L.u_alt);
  T* spec = (T*)wsp(ws, L.spec0);
  T* phibar = (T*)wsp(ws, L.phibar);
  double* part = (double*)wsp(ws, L.part_rp);
  Ctrl* ctrl = (Ctrl*)wsp(ws, L.ctrl);
  T* uin = odd ? u : u_alt;
  T* uout = odd ? u_alt : u;
  const GraphKey& K = h->last;   // the loop being captured
  LamArgs<T> lam{(const T*)K.lam_u0, (T*)wsp(ws, L.lam), (T*)wsp(ws, L.lambar), (T)K.tau_u0, (T)K.tau_lam};
  if (is_pre32(p)) {   // the spectrum, its FFTs and the column solve in float
    float* spec32 = (float*)wsp(ws, L.spec0);
    T* s0 = (T*)wsp(ws, L.s0);   // mode 0 of the spectrum in FP64
    HIP_TRY((launch_dual_fft<T, float>(spec32, p.nt, h->lqb, p.nx, h->d_tw32, phi, phibar, tau_phi, ctrl, st, s0)));
    HIP_TRY((launch_primal_res<T, float>(s, uin, uout, phibar, phi, tau_u, spec32, h->lqb, h->d_tw32, part, ctrl,
                                         st, &lam)));
    const double wscale = (p.t_final / p.nt) * (p.length / p.nx);
    const int bw = p.time == PDHG_BDF2 ? 2 : 1;
    if (uses_chunks(p) && h->d_cmap)
      HIP_TRY(launch_colsolve_chunk<float>(spec32, chunk_args(h, ws), bw, p.nt, p.nx, h->lqb, ctrl, part,
                                           (p.nt + 1) / 2, wscale, hist, st, (double*)s0));
    else
      HIP_TRY((launch_colsolve_wave<float, double>(spec32, factab<double>(h), bw, p.nt, p.nx, h->lqb, ctrl, part,
                                                   (p.nt + 1) / 2, wscale, hist, st, (double*)s0)));
    return PDHG_OK;
  }
  HIP_TRY(launch_dual_fft<T>(spec, p.nt, h->lqb, p.nx, h->d_tw, phi, phibar, tau_phi, ctrl, st));
  HIP_TRY(launch_primal_res<T>(s, uin, uout, phibar, phi, tau_u, spec, h->lqb, h->d_tw, part, ctrl, st, &lam));
  HIP_TRY(colsolve_any<T>(h, ws, spec, ctrl, part, (p.nt + 1) / 2, hist, st));
  return PDHG_OK;
}

// One DG loop body: A (inverse FFT + dual step over the 3 nt coefficient rows),
// primal step + dual residual, implicit residual, forward FFT, column solve in
// the per-mode eigenbasis, norms and stopping decision.
template <typename T>
int enqueue_body_dg(pdhg_handle* h, bool odd, T* u, T* phi, void* ws, T tau_u, T tau_phi, double* hist,
                    hipStream_t st, bool mfma = false) {
  const pdhg_problem& p = h->prob;
  const WsLayout L = layout_for(p, h->esz);
  const Scheme s = scheme_of(h);
  T* u_alt = (T*)wsp(ws, L.u_alt);
  T* spec = (T*)wsp(ws, L.spec0);
  T* srow = (T*)wsp(ws, L.srow);
  T* phibar = (T*)wsp(ws, L.phibar);
  double* prp = (double*)wsp(ws, L.part_rp);
  double* prd = (double*)wsp(ws, L.part_rd);
  Ctrl* ctrl = (Ctrl*)wsp(ws, L.ctrl);
  T* uin = odd ? u : u_alt;
  T* uout = odd ? u_alt : u;
  const int nr = planes(p) * p.nt;
  const bool p2 = p.space == PDHG_DG_P2_LLF;
  int nb_rd = 0, nb_rp = 0;
  if (p.nx >= 64) {
    HIP_TRY(launch_dual_fft<T>(spec, nr, h->lqb, p.nx, h->d_tw, phi, phibar, tau_phi, ctrl, st));
  } else {
    HIP_TRY(launch_rows_inv<T>(spec, nr, h->lqb, srow, nr, p.nx, h->d_tw, ctrl, st));
    HIP_TRY(launch_dual<T>(phi, phibar, srow, (size_t)nr * p.nx, tau_phi, ctrl, st));
  }
  HIP_TRY(dgx_primal<T>(s, uin, uout, phibar, phi, tau_u, prd, ctrl, st, &nb_rd));
  if (mfma) {   // variant 6: the residual with its per-cell products on the matrix cores, then the row FFT
    if constexpr (sizeof(T) == 4) {
      HIP_TRY(launch_dg_residual_mfma(s, (const float*)uout, (float*)srow, prp, ctrl, st, &nb_rp));
    } else {
      return PDHG_EUNSUPPORTED;
    }
    HIP_TRY(launch_rows_fwd<T>(srow, nr, spec, nr, h->lqb, p.nx, h->d_tw, ctrl, st));
  } else if (p2 && p.nx >= 64) {   // P2: residual of two levels + forward FFT of their six coefficient rows, fused
    HIP_TRY(launch_dg_residual_fft<T>(s, uout, spec, h->lqb, h->d_tw, prp, ctrl, st, &nb_rp));
  } else {
    HIP_TRY(dgx_residual<T>(s, uout, srow, prp, ctrl, st, &nb_rp));
    HIP_TRY(launch_rows_fwd<T>(srow, nr, spec, nr, h->lqb, p.nx, h->d_tw, ctrl, st));
  }
  HIP_TRY(launch_dg_colsolve<T>(spec, factab<T>(h), (const T*)h->d_vtab, p.time == PDHG_BDF2 ? 2 : 1, p.nt, p.nx,
                                h->lqb, ctrl, st, planes(p)));
  HIP_TRY(launch_finalize(ctrl, prp, nb_rp, prd, nb_rd, s.ht * s.hx, hist, st));
  return PDHG_OK;
}

template <typename T>
int build_graph(pdhg_handle* h, const GraphKey& key, T* u, T* phi, void* ws, T tau_u, T tau_phi, double* hist) {
  if (h->gexec && h->gkey == key) return PDHG_OK;
  if (h->gexec) { hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
  if (h->graph) { hipGraphDestroy(h->graph); h->graph = nullptr; }
  HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = PDHG_OK;
  for (int b = 0; b < key.chunk && rc == PDHG_OK; ++b) {
    if (key.variant == 4 || key.variant == 6)
      rc = enqueue_body_dg<T>(h, (b % 2) == 0, u, phi, ws, tau_u, tau_phi, hist, h->cap_stream, key.variant == 6);
    else if (key.variant == 1)
      rc = enqueue_body_unfused<T>(h, (b % 2) == 0, u, phi, ws, tau_u, tau_phi, hist, h->cap_stream);
    else
      rc = enqueue_body_fused<T>(h, (b % 2) == 0, u, phi, ws, tau_u, tau_phi, hist, h->cap_stream);
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (rc) { if (g) hipGraphDestroy(g); return rc; }
  if (e != hipSuccess) return set_hip_error(h, e, "hipStreamEndCapture");
  h->graph = g;
  HIP_TRY(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0));
  h->gkey = key;
  return PDHG_OK;
}

// ||A(u)|| and ||J(u)^T phi|| of a state (the partial sums in the workspace, added on the host).
template <typename T>
int state_norms(pdhg_handle* h, const T* u, const T* phi, void* ws, hipStream_t st, double* rp, double* rd) {
  const WsLayout L = layout_for(h->prob, h->esz);
  const Scheme s = scheme_of(h);
  double* prp = (double*)wsp(ws, L.part_rp);
  double* prd = (double*)wsp(ws, L.part_rd);
  int nb1 = 0, nb2 = 0;
  if (is_dg(h->prob)) {
    HIP_TRY(dgx_residual<T>(s, u, (T*)nullptr, prp, nullptr, st, &nb1));
    HIP_TRY(dgx_apply_jt<T>(s, u, phi, (T*)nullptr, prd, st, &nb2));
  } else {
    HIP_TRY(launch_residual<T>(s, u, (T*)nullptr, prp, nullptr, st, &nb1));
    HIP_TRY(launch_apply_jt<T>(s, u, phi, (T*)nullptr, prd, st, &nb2));
  }
  std::vector<double> a(nb1), b(nb2);
  HIP_TRY(hipMemcpyAsync(a.data(), prp, nb1 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(b.data(), prd, nb2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double sa = 0.0, sb = 0.0;
  for (double x : a) sa += x;
  for (double x : b) sb += x;
  *rp = std::sqrt(s.ht * s.hx * sa);
  *rd = std::sqrt(s.ht * s.hx * sb);
  return PDHG_OK;
}

template <typename T>
int solve_impl(pdhg_handle* h, const T* u0, T* u, T* phi, void* ws, const pdhg_params* prm, pdhg_stats* stats,
               hipStream_t st) {
  const pdhg_problem& p = h->prob;
  int rc = ensure_workspace(h, ws);
  if (rc) return rc;
  const WsLayout L = layout_for(p, h->esz);
  const int row = p.nx * planes(p);   // elements per level
  const bool dg = is_dg(p);
  const size_t nlev = (size_t)(p.nt + 1) * row, n = (size_t)p.nt * row;
  T* u_alt = (T*)wsp(ws, L.u_alt);
  T* spec = (T*)wsp(ws, L.spec0);
  Ctrl* ctrl = (Ctrl*)wsp(ws, L.ctrl);
  // initial guess (Section 3.3): u^l = u0, phi = 0 unless warm start; u^0 = u0 always
  if (prm->warm_start) {
    HIP_TRY(launch_copy<T>(u, u0, (size_t)row, st));
  } else {
    HIP_TRY(launch_broadcast_levels<T>(u, u0, row, p.nt + 1, st));
    HIP_TRY(launch_fill<T>(phi, n, T(0), st));
  }
  rc = resolve_constants<T>(h, u0, ws, st);
  if (rc) return rc;
  double tau_u = prm->tau_u, tau_phi = prm->tau_phi, nu = 0.0;
  if (tau_u <= 0.0 || tau_phi <= 0.0) {
    // power iteration at the constant extension u^l = u0 (u_alt used as scratch)
    HIP_TRY(launch_broadcast_levels<T>(u_alt, u0, row, p.nt + 1, st));
    rc = power_iteration<T>(h, u_alt, ws, st, 200, &nu);
    if (rc) return rc;
    if (!(nu > 0.0) || !std::isfinite(nu)) return PDHG_EINVAL;
    tau_u = tau_phi = std::sqrt(0.95 / nu);
  }
  const double div = prm->diverge_factor > 0 ? prm->diverge_factor : 1e6;
  // without a residual history: Rd only where the stopping test needs it
  const int rd_lazy = prm->history ? 0 : 1;
  if (prm->stall_iters < 0) return PDHG_EINVAL;
  // scale-free tolerance: both residuals <= eps_rel ||u0|| / h_t, ||u0|| = sqrt(h_x sum u0^2)
  double eps = prm->eps;
  if (prm->eps_rel > 0.0) {
    double* scal = (double*)wsp(ws, L.scal);
    HIP_TRY(launch_dot<T>(u0, nullptr, (size_t)row, (double*)wsp(ws, L.part_rp), scal, st));
    HIP_TRY(hipMemcpyAsync(h->h_scal, scal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double hx = p.length / p.nx, ht = p.t_final / p.nt;
    eps = std::max(eps, prm->eps_rel * std::sqrt(hx * h->h_scal[0]) / ht);
  }
  int chunk = prm->check_every > 0 ? prm->check_every : 64;
  chunk += chunk & 1;   // even: u ping-pong returns to its start buffer
  GraphKey key;
  key.u = u; key.phi = phi; key.ws = ws; key.hist = prm->history;
  key.lf = h->lf; key.c = h->c;
  // fused passes need at least one full wavefront per row (nx >= 64); DG has its own body
  if (prm->variant == 2 && p.nx < 64 && !dg) return PDHG_EUNSUPPORTED;
  // the single-precision preconditioner runs in the fused passes only
  if (is_pre32(p) && (prm->variant == 1 || p.nx < 64)) return PDHG_EUNSUPPORTED;
  if (dg && prm->variant != 0 && prm->variant != 4 && prm->variant != 6) return PDHG_EUNSUPPORTED;
  // variant 6: the DG P2 body with the residual's per-cell products on the matrix cores (FP32)
  if (prm->variant == 6 && !(p.space == PDHG_DG_P2_LLF && p.dtype == PDHG_F32 && p.nx >= 64))
    return PDHG_EUNSUPPORTED;
  if (prm->backoff < 0) return PDHG_EINVAL;
  key.variant = dg ? (prm->variant == 6 ? 6 : 4) : ((prm->variant == 1 || p.nx < 64) ? 1 : 2);
  key.chunk = chunk;
  if (prm->init_multiplier) {   // the multiplier form: fused finite-difference passes only, no back-off
    if (key.variant != 2 || prm->backoff > 0 || is_full(p)) return PDHG_EUNSUPPORTED;
    key.lam_u0 = u0;
    key.tau_u0 = prm->tau_u0 > 0 ? prm->tau_u0 : 0.5 * tau_u;
    key.tau_lam = prm->tau_lam > 0 ? prm->tau_lam : 0.99;
  }
  // Last-good checkpoint (u, phi, iterate index): refreshed on the device after every chunk while the
  // solve runs (launch_checkpoint), so that it always holds an iterate that passed the tests.
  T* ck_u = (T*)wsp(ws, L.ck_u);
  T* ck_phi = (T*)wsp(ws, L.ck_phi);
  long long done = 0;   // iterations completed before the current run (step-size back-offs)
  int backoffs = 0;
  double rp_ck = 0.0, rd_ck = 0.0;
  bool restored = false;
  Ctrl c{};
  long long nstar = 0;
  int status = PDHG_NOT_CONVERGED;
  auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    HIP_TRY(launch_copy<T>(u_alt, u, nlev, st));
    HIP_TRY(launch_fill<T>(spec, n, T(0), st));
    if (is_pre32(p)) HIP_TRY(launch_fill<T>((T*)wsp(ws, L.s0), (size_t)p.nt, T(0), st));
    if (prm->init_multiplier) {   // lambda = lambdabar = 0; u^0 starts from u0 (the broadcast above)
      HIP_TRY(launch_fill<T>((T*)wsp(ws, L.lam), (size_t)p.nx, T(0), st));
      HIP_TRY(launch_fill<T>((T*)wsp(ws, L.lambar), (size_t)p.nx, T(0), st));
    }
    const long long budget = prm->max_iter - done;
    HIP_TRY(launch_ctrl_init(ctrl, budget, eps, div, st, rd_lazy, prm->stall_iters));
    key.tau_u = tau_u;
    key.tau_phi = tau_phi;
    h->last = key;
    if (budget > 0) {
      HIP_TRY(launch_checkpoint<T>(ctrl, u_alt, phi, ck_u, ck_phi, nlev, n, st));   // iterate 0
      rc = build_graph<T>(h, key, u, phi, ws, (T)tau_u, (T)tau_phi, prm->history);
      if (rc) return rc;
      const long long bodies = budget + 1;
      long long launched = 0;
      int idx = 0;
      bool stop = false;
      while (!stop && launched < bodies) {
        HIP_TRY(hipGraphLaunch(h->gexec, st));
        launched += chunk;
        HIP_TRY(launch_checkpoint<T>(ctrl, u_alt, phi, ck_u, ck_phi, nlev, n, st));
        HIP_TRY(hipMemcpyAsync(&h->h_ctrl[idx & 1], ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipEventRecord(h->ev[idx & 1], st));
        if (idx >= 1) {
          HIP_TRY(hipEventSynchronize(h->ev[(idx - 1) & 1]));
          if (h->h_ctrl[(idx - 1) & 1].status != 0) stop = true;
        }
        ++idx;
      }
    }
    HIP_TRY(hipMemcpyAsync(&h->h_ctrl[0], ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    c = h->h_ctrl[0];
    nstar = c.n_star;
    if (budget <= 0) { nstar = 0; status = PDHG_NOT_CONVERGED; }
    else if (c.status == 1) status = PDHG_OK;
    else if (c.status == 2) status = PDHG_DIVERGED;
    else if (c.status == 4) status = PDHG_STALLED;
    else status = PDHG_NOT_CONVERGED;
    if (status != PDHG_DIVERGED) {
      if (nstar & 1) HIP_TRY(launch_copy<T>(u, u_alt, nlev, st));
      nstar += done;
      break;
    }
    // diverged: back to the last good checkpoint
    HIP_TRY(launch_copy<T>(u, ck_u, nlev, st));
    HIP_TRY(launch_copy<T>(phi, ck_phi, n, st));
    done += c.ck_iter > 0 ? c.ck_iter : 0;
    if (backoffs < prm->backoff && done < prm->max_iter) {   // smaller steps from the checkpoint
      ++backoffs;
      tau_u *= 0.7;
      tau_phi *= 0.7;
      continue;
    }
    nstar = done;
    restored = true;
    rc = state_norms<T>(h, u, phi, ws, st, &rp_ck, &rd_ck);
    if (rc) return rc;
    break;
  }
  auto t1 = std::chrono::steady_clock::now();
  double drift = 0.0;
  {
    double* lev = (double*)wsp(ws, L.part_rp);   // nt+1 <= max_parts
    // mass h_x sum_j of the cell averages: plane 0 for P2 Legendre, (v_1 + v_2) / 2 for P1 nodal
    const bool p1 = p.space == PDHG_DG_P1_UPWIND;
    HIP_TRY(launch_level_sums<T>(u, p1 ? 2 * p.nx : p.nx, (size_t)row, p.nt + 1, lev, st));
    std::vector<double> m(p.nt + 1);
    HIP_TRY(hipMemcpyAsync(m.data(), lev, m.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double hx = (p1 ? 0.5 : 1.0) * p.length / p.nx;
    for (int l = 1; l <= p.nt; ++l) drift = std::max(drift, std::fabs(m[l] - m[0]) * hx);
  }
  if (stats) {
    stats->mass_drift = drift;
    stats->iters = nstar;
    stats->res_primal = restored ? rp_ck : c.rp_star;
    stats->res_dual = restored ? rd_ck : c.rd_star;
    stats->tau_u = tau_u;
    stats->tau_phi = tau_phi;
    stats->nu_max = nu;
    stats->lf_speed = h->lf;
    stats->precond_c = h->c;
    stats->seconds = std::chrono::duration<double>(t1 - t0).count();
    stats->status = status;
    stats->variant = key.variant;
  }
  HIP_TRY(hipStreamSynchronize(st));
  return status;
}

}  // namespace

namespace {

// Algorithm 2 (Section 3.4): Algorithm 1 on N_t0 = nt_start, 2 nt_start, ... levels,
// each warm-started from the previous level's solution interpolated in time.
template <typename T>
int solve_refined_impl(pdhg_handle* h, const T* u0, T* u, T* phi, void* ws, const pdhg_params* prm,
                       const pdhg_refine_params* rp, pdhg_stats* stats, int64_t* level_iters, hipStream_t st) {
  const pdhg_problem& P = h->prob;
  if (is_pre32(P)) return PDHG_EUNSUPPORTED;   // Algorithm 1 only
  std::vector<int> nts;   // coarse levels
  int n = rp->nt_start;
  while (n < P.nt) {
    nts.push_back(n);
    n *= 2;
  }
  if (n != P.nt) return PDHG_EINVAL;   // nt / nt_start must be a power of two
  const size_t row = (size_t)P.nx * planes(P);
  T* ub[2] = {nullptr, nullptr};
  T* pb[2] = {nullptr, nullptr};
  if (!nts.empty()) {
    const size_t ntc = (size_t)nts.back();
    const size_t bu = align_up((ntc + 1) * row * sizeof(T)), bp = align_up(ntc * row * sizeof(T));
    const size_t need = 2 * (bu + bp);
    if (h->refine_buf_bytes < need) {
      if (h->refine_buf) hipFree(h->refine_buf);
      h->refine_buf = nullptr;
      h->refine_buf_bytes = 0;
      HIP_TRY(hipMalloc(&h->refine_buf, need));
      h->refine_buf_bytes = need;
    }
    char* b = static_cast<char*>(h->refine_buf);
    ub[0] = (T*)b;
    pb[0] = (T*)(b + bu);
    ub[1] = (T*)(b + bu + bp);
    pb[1] = (T*)(b + 2 * bu + bp);
  }
  const T* uc = nullptr;
  const T* pc = nullptr;
  int ntc = 0, li = 0;
  for (size_t k = 0; k < nts.size(); ++k) {
    const int nk = nts[k];
    pdhg_handle* sh = nullptr;
    for (auto& kv : h->refine_sub)
      if (kv.first == nk) sh = kv.second;
    if (!sh) {
      pdhg_problem q = P;
      q.nt = nk;
      const int rc = pdhg_setup(&q, &sh);
      if (rc) return rc;
      h->refine_sub.emplace_back(nk, sh);
    }
    T* uk = ub[k & 1];
    T* pk = pb[k & 1];
    if (k > 0) HIP_TRY(launch_refine_time<T>(uc, pc, ntc, row, uk, pk, st));
    pdhg_params p = *prm;
    p.eps = rp->coarse_eps > 0.0 ? rp->coarse_eps : prm->eps;
    p.max_iter = rp->coarse_max_iter;
    p.warm_start = k > 0 ? 1 : 0;
    p.history = nullptr;
    pdhg_stats sk{};
    const int rc = pdhg_solve(sh, u0, uk, pk, nullptr, &p, &sk, (pdhg_stream_t)st);
    if (rc < 0) {
      h->err = std::string("coarse level ") + std::to_string(nk) + ": " + pdhg_last_error(sh);
      return rc;
    }
    if (level_iters) level_iters[li] = sk.iters;
    ++li;
    if (rc == PDHG_DIVERGED) {
      if (stats) *stats = sk;
      return PDHG_DIVERGED;
    }
    uc = uk;
    pc = pk;
    ntc = nk;
  }
  pdhg_params p = *prm;
  if (!nts.empty()) {
    HIP_TRY(launch_refine_time<T>(uc, pc, ntc, row, u, phi, st));
    p.warm_start = 1;
  }
  pdhg_stats sf{};
  const int rc = solve_impl<T>(h, u0, u, phi, ws, &p, &sf, st);
  if (stats) *stats = sf;
  if (level_iters && rc >= 0) level_iters[li] = sf.iters;
  return rc;
}

// Algorithm 3 on the DG P1 scheme: the same march on the two nodal planes
// (k_onestep_dg1).  Default step sizes: sqrt(0.95 / nu_max) with nu_max from the
// power iteration of Algorithm 1 on the one-level problems (backward Euler,
// N_t = 1, time step h_t / c0 for c0 = 1 and, with BDF2, 3/2), whose K_d is the
// step preconditioner.
template <typename T>
int onestep_dg1_impl(pdhg_handle* h, const T* u0, T* u, T* phi, const pdhg_params* prm, pdhg_stats* stats,
                     int64_t* step_iters, double* step_res, hipStream_t st) {
  const pdhg_problem& P = h->prob;
  const int nx = P.nx, nt = P.nt, nm = nx / 2 + 1;
  if (nx < 64 || nx > 4096) return PDHG_EUNSUPPORTED;
  const size_t row = 2 * (size_t)nx;
  const size_t b_sym = align_up((size_t)2 * nm * 4 * sizeof(T));
  const size_t b_stat = align_up((size_t)nt * sizeof(StepStat));
  const size_t b_flag = align_up(sizeof(int));
  const size_t b_part = align_up(sizeof(double) * std::max<size_t>(64, (size_t)nt + 1));
  const size_t need = b_sym + b_stat + b_flag + b_part + align_up(sizeof(OneStepProb<T>));
  if (h->os_buf_bytes < need) {
    if (h->os_buf) hipFree(h->os_buf);
    h->os_buf = nullptr;
    h->os_buf_bytes = 0;
    h->os_c = -1.0;
    HIP_TRY(hipMalloc(&h->os_buf, need));
    h->os_buf_bytes = need;
  }
  char* b = static_cast<char*>(h->os_buf);
  T* sym = (T*)b;
  StepStat* stat = (StepStat*)(b + b_sym);
  int* flag = (int*)(b + b_sym + b_stat);
  double* part = (double*)(b + b_sym + b_stat + b_flag);
  OneStepProb<T>* tab = (OneStepProb<T>*)(b + b_sym + b_stat + b_flag + b_part);
  int rc = resolve_constants_p<T>(h, u0, part, st, false);
  if (rc) return rc;
  if (h->os_c != h->c) {
    std::vector<T> hs((size_t)2 * nm * 4);
    onestep_dg1_kinv<T>(P, h->c, hs.data());
    HIP_TRY(hipMemcpyAsync(sym, hs.data(), hs.size() * sizeof(T), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    h->os_c = h->c;
  }
  double tau_u = prm->tau_u, tau_phi = prm->tau_phi, nu = 0.0;
  const bool auto_tau = !(tau_u > 0.0 && tau_phi > 0.0);
  if (auto_tau) {
    if (!h->os_sub_buf)
      HIP_TRY(hipMalloc(&h->os_sub_buf, 3 * row * sizeof(T)));   // u [2][2][nx], phi [1][2][nx]
    T* su = (T*)h->os_sub_buf;
    T* sp = su + 2 * row;
    const int nrow = (P.time == PDHG_BDF2 && nt > 1) ? 2 : 1;
    for (int r = 0; r < nrow; ++r) {
      if (!h->os_sub[r]) {
        pdhg_problem q = P;
        q.nt = 1;
        q.time = PDHG_BE;
        q.t_final = (P.t_final / nt) / (r ? 1.5 : 1.0);
        q.precond_c = h->c;
        q.lf_speed = h->lf;
        rc = pdhg_setup(&q, &h->os_sub[r]);
        if (rc) return rc;
      }
      pdhg_params pp{};
      pp.tau_u = pp.tau_phi = 0.0;
      pp.eps = 0.0;
      pp.max_iter = 2;
      pp.check_every = 2;
      pdhg_stats ss{};
      rc = pdhg_solve(h->os_sub[r], u0, su, sp, nullptr, &pp, &ss, (pdhg_stream_t)st);
      if (rc < 0) {
        h->err = std::string("one-level step-size plan: ") + pdhg_last_error(h->os_sub[r]);
        return rc;
      }
      nu = std::max(nu, ss.nu_max);
    }
    if (!(nu > 0.0) || !std::isfinite(nu)) return PDHG_EINVAL;
    tau_u = tau_phi = std::sqrt(0.95 / nu);
  }
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
  HIP_TRY(hipMemsetAsync(stat, 0, (size_t)nt * sizeof(StepStat), st));
  OneStepProb<T> tp{};
  tp.s = scheme_of(h);
  tp.tw = (const C2<T>*)h->d_tw;
  tp.sym = sym;
  tp.u0 = u0;
  tp.u = u;
  tp.phi = phi;
  tp.stat = stat;
  tp.flag = flag;
  tp.tau_u = tau_u;
  tp.tau_phi = tau_phi;
  tp.pcr = nullptr;
  HIP_TRY(hipMemcpyAsync(tab, &tp, sizeof(tp), hipMemcpyHostToDevice, st));
  const double div = prm->diverge_factor > 0 ? prm->diverge_factor : 1e6;
  auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(launch_onestep_dg1<T>(tab, 1, nx, 0, nt, prm->eps, (long long)prm->max_iter, div, st));
  std::vector<StepStat> rec(nt);
  HIP_TRY(hipMemcpyAsync(rec.data(), stat, (size_t)nt * sizeof(StepStat), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  OneStepSummary sm = summarize_steps(rec.data(), nt, step_iters, step_res);
  if (stats) {
    stats->iters = sm.total;
    stats->res_primal = sm.rp;
    stats->res_dual = sm.rd;
    stats->tau_u = tau_u;
    stats->tau_phi = tau_phi;
    stats->nu_max = nu;
    stats->lf_speed = h->lf;
    stats->precond_c = h->c;
    stats->seconds = std::chrono::duration<double>(t1 - t0).count();
    stats->mass_drift = -1.0;
    stats->status = sm.status;
    stats->variant = 5;
  }
  return sm.status;
}

// Algorithm 3 (Section 3.5): one launch of k_onestep marches every step (one
// workgroup; u^l stays in registers between steps).  A diverged step stops
// the march and sets the problem's device flag.
template <typename T>
int onestep_impl(pdhg_handle* h, const T* u0, T* u, T* phi, const pdhg_params* prm, pdhg_stats* stats,
                 int64_t* step_iters, double* step_res, hipStream_t st) {
  const pdhg_problem& P = h->prob;
  if (is_pre32(P)) return PDHG_EUNSUPPORTED;   // Algorithm 1 only
  if (P.space == PDHG_DG_P1_UPWIND) return onestep_dg1_impl<T>(h, u0, u, phi, prm, stats, step_iters, step_res, st);
  if (is_dg(P) || P.nx < 64) return PDHG_EUNSUPPORTED;
  const int nx = P.nx, nt = P.nt;
  // sym [2][nx], pcr [2][16] | stat [nt] | flag | part (max |f'|, nu, level sums) | problem table
  const size_t b_sym = align_up((2 * (size_t)nx + 32) * sizeof(T));
  const size_t b_stat = align_up((size_t)nt * sizeof(StepStat));
  const size_t b_flag = align_up(sizeof(int));
  const size_t b_part = align_up(sizeof(double) * std::max<size_t>(64, (size_t)nt + 1));
  const size_t need = b_sym + b_stat + b_flag + b_part + align_up(sizeof(OneStepProb<T>));
  if (h->os_buf_bytes < need) {
    if (h->os_buf) hipFree(h->os_buf);
    h->os_buf = nullptr;
    h->os_buf_bytes = 0;
    h->os_c = -1.0;
    HIP_TRY(hipMalloc(&h->os_buf, need));
    h->os_buf_bytes = need;
  }
  char* b = static_cast<char*>(h->os_buf);
  T* sym = (T*)b;
  StepStat* stat = (StepStat*)(b + b_sym);
  int* flag = (int*)(b + b_sym + b_stat);
  double* part = (double*)(b + b_sym + b_stat + b_flag);
  OneStepProb<T>* tab = (OneStepProb<T>*)(b + b_sym + b_stat + b_flag + b_part);

  int rc = resolve_constants_p<T>(h, u0, part, st, false);
  if (rc) return rc;
  const double ht = P.t_final / nt, hx = P.length / nx;
  double pcr[32];
  int pcr_k[2] = {0, 0};
  const bool use_pcr = onestep_pcr(P, h->c, sizeof(T) == 8 ? 1e-17 : 1e-9, pcr, pcr_k);
  if (!use_pcr) pcr_k[0] = pcr_k[1] = 0;
  if (h->os_c != h->c) {
    std::vector<T> hs(2 * (size_t)nx + 32, T(0));
    onestep_symbol<T>(P, h->c, h->lf, hs.data());
    if (use_pcr)
      for (int i = 0; i < 32; ++i) hs[2 * (size_t)nx + i] = (T)pcr[i];
    HIP_TRY(hipMemcpyAsync(sym, hs.data(), hs.size() * sizeof(T), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    h->os_c = h->c;
  }
  (void)ht;
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
  HIP_TRY(hipMemsetAsync(stat, 0, (size_t)nt * sizeof(StepStat), st));
  const bool auto_tau = !(prm->tau_u > 0.0 && prm->tau_phi > 0.0);
  OneStepProb<T> tp{};
  tp.s = scheme_of(h);
  tp.tw = (const C2<T>*)h->d_tw;
  tp.sym = sym;
  tp.u0 = u0;
  tp.u = u;
  tp.phi = phi;
  tp.stat = stat;
  tp.flag = flag;
  tp.tau_u = auto_tau ? 0.0 : prm->tau_u;
  tp.tau_phi = auto_tau ? 0.0 : prm->tau_phi;
  tp.pcr = sym + 2 * (size_t)nx;
  tp.pcr_k[0] = pcr_k[0];
  tp.pcr_k[1] = pcr_k[1];
  HIP_TRY(hipMemcpyAsync(tab, &tp, sizeof(tp), hipMemcpyHostToDevice, st));
  double tau_u = prm->tau_u, tau_phi = prm->tau_phi, nu = 0.0;
  if (auto_tau) {
    // nu_max over the step operators at u0 (200 power iterations); the kernel sets the table's steps
    HIP_TRY(launch_onestep_power<T>(tab, 1, nx, 200, part, st));
    HIP_TRY(hipMemcpyAsync(h->h_scal, part, sizeof(double), hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (auto_tau) {
    nu = h->h_scal[0];
    if (!(nu > 0.0) || !std::isfinite(nu)) return PDHG_EINVAL;
    tau_u = tau_phi = std::sqrt(0.95 / nu);
  }
  const double div = prm->diverge_factor > 0 ? prm->diverge_factor : 1e6;
  auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(launch_onestep<T>(tab, 1, nx, 0, nt, prm->eps, (long long)prm->max_iter, div, st));
  std::vector<StepStat> rec(nt);
  HIP_TRY(hipMemcpyAsync(rec.data(), stat, (size_t)nt * sizeof(StepStat), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  OneStepSummary sm = summarize_steps(rec.data(), nt, step_iters, step_res);
  double drift = 0.0;
  {
    HIP_TRY(launch_level_sums<T>(u, nx, (size_t)nx, sm.done + 1, part, st));
    std::vector<double> m(sm.done + 1);
    HIP_TRY(hipMemcpyAsync(m.data(), part, m.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int l = 1; l <= sm.done; ++l) drift = std::max(drift, std::fabs(m[l] - m[0]) * hx);
  }
  if (stats) {
    stats->iters = sm.total;
    stats->res_primal = sm.rp;
    stats->res_dual = sm.rd;
    stats->tau_u = tau_u;
    stats->tau_phi = tau_phi;
    stats->nu_max = nu;
    stats->lf_speed = h->lf;
    stats->precond_c = h->c;
    stats->seconds = std::chrono::duration<double>(t1 - t0).count();
    stats->mass_drift = drift;
    stats->status = sm.status;
    stats->variant = 5;
  }
  return sm.status;
}

}  // namespace

extern "C" {

int pdhg_solve_onestep(pdhg_handle* h, const void* u0, void* u, void* phi, const pdhg_params* params,
                       pdhg_stats* stats, int64_t* step_iters, double* step_res, pdhg_stream_t stream) {
  if (!h || !u0 || !u || !phi || !params) return PDHG_EINVAL;
  if (params->max_iter < 0) return PDHG_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return set_hip_error(h, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (h->prob.dtype == PDHG_F64)
    return onestep_impl<double>(h, (const double*)u0, (double*)u, (double*)phi, params, stats, step_iters, step_res,
                                st);
  return onestep_impl<float>(h, (const float*)u0, (float*)u, (float*)phi, params, stats, step_iters, step_res, st);
}

int pdhg_solve_refined(pdhg_handle* h, const void* u0, void* u, void* phi, void* workspace,
                       const pdhg_params* params, const pdhg_refine_params* refine, pdhg_stats* stats,
                       int64_t* level_iters, pdhg_stream_t stream) {
  if (!h || !u0 || !u || !phi || !params || !refine) return PDHG_EINVAL;
  if (params->max_iter < 0 || refine->coarse_max_iter < 0 || refine->nt_start < 1 || refine->nt_start > h->prob.nt)
    return PDHG_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return set_hip_error(h, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (h->prob.dtype == PDHG_F64)
    return solve_refined_impl<double>(h, (const double*)u0, (double*)u, (double*)phi, workspace, params, refine,
                                      stats, level_iters, st);
  return solve_refined_impl<float>(h, (const float*)u0, (float*)u, (float*)phi, workspace, params, refine, stats,
                                   level_iters, st);
}

int pdhg_solve(pdhg_handle* h, const void* u0, void* u, void* phi, void* workspace, const pdhg_params* params,
               pdhg_stats* stats, pdhg_stream_t stream) {
  if (!h || !u0 || !u || !phi || !params) return PDHG_EINVAL;
  if (params->max_iter < 0) return PDHG_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return set_hip_error(h, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (h->prob.dtype == PDHG_F64)
    return solve_impl<double>(h, (const double*)u0, (double*)u, (double*)phi, workspace, params, stats, st);
  return solve_impl<float>(h, (const float*)u0, (float*)u, (float*)phi, workspace, params, stats, st);
}

}  // extern "C"

namespace {

template <typename T>
int residual_impl(pdhg_handle* h, const T* u, const T* phi, T* Au, T* JTphi, double* res, hipStream_t st) {
  void* ws = nullptr;
  int rc = ensure_workspace(h, ws);
  if (rc) return rc;
  if (!h->consts_valid) {
    rc = resolve_constants<T>(h, u, ws, st);   // u[0] is u0
    if (rc) return rc;
  }
  const WsLayout L = layout_for(h->prob, h->esz);
  const Scheme s = scheme_of(h);
  double* prp = (double*)wsp(ws, L.part_rp);
  double* prd = (double*)wsp(ws, L.part_rd);
  int nb1 = 0, nb2 = 0;
  if (is_dg(h->prob)) {
    HIP_TRY(dgx_residual<T>(s, u, Au, prp, nullptr, st, &nb1));
    if (phi) HIP_TRY(dgx_apply_jt<T>(s, u, phi, JTphi, prd, st, &nb2));
  } else {
    HIP_TRY(launch_residual<T>(s, u, Au, prp, nullptr, st, &nb1));
    if (phi) HIP_TRY(launch_apply_jt<T>(s, u, phi, JTphi, prd, st, &nb2));
  }
  if (res) {
    // reduce the partials on the host (few thousand doubles)
    std::vector<double> a(nb1), b(nb2);
    HIP_TRY(hipMemcpyAsync(a.data(), prp, nb1 * sizeof(double), hipMemcpyDeviceToHost, st));
    if (nb2) HIP_TRY(hipMemcpyAsync(b.data(), prd, nb2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double sa = 0, sb = 0;
    for (double x : a) sa += x;
    for (double x : b) sb += x;
    res[0] = std::sqrt(s.ht * s.hx * sa);
    res[1] = phi ? std::sqrt(s.ht * s.hx * sb) : 0.0;
  }
  return PDHG_OK;
}

template <typename T>
int precond_impl(pdhg_handle* h, const T* r, T* s, hipStream_t st) {
  void* ws = nullptr;
  int rc = ensure_workspace(h, ws);
  if (rc) return rc;
  if (is_full(h->prob)) {
    if (!h->consts_valid) {   // constants as given (no u0 to resolve them from)
      if (h->prob.precond_c < 0.0 || (h->prob.space == PDHG_FD_LF && h->prob.lf_speed < 0.0)) return PDHG_EINVAL;
      h->c = h->prob.precond_c;
      h->lf = h->prob.space == PDHG_FD_LF ? h->prob.lf_speed : 0.0;
    }
  } else if (!h->d_fac_rows) {
    if (h->prob.precond_c < 0.0) return PDHG_EINVAL;
    rc = is_dg(h->prob) ? upload_factors_dg<T>(h, h->prob.precond_c)
                                          : upload_factors<T>(h, h->prob.precond_c, h->prob.precond_gamma_hat);
    if (rc) return rc;
  }
  const WsLayout L = layout_for(h->prob, h->esz);
  return precond_apply<T>(h, ws, r, s, (T*)wsp(ws, L.spec0), st);
}

template <typename T>
int adjoint_impl(pdhg_handle* h, int mode, const T* u, const T* in, T* out, T* mu, void* ws, hipStream_t st) {
  int rc = ensure_workspace(h, ws);
  if (rc) return rc;
  if (!h->consts_valid) {
    rc = resolve_constants<T>(h, u, ws, st);
    if (rc) return rc;
  }
  const Scheme s = scheme_of(h);
  const bool dg = is_dg(h->prob);
  if (mode == PDHG_ADJ_APPLY) {
    if (dg) HIP_TRY(dgx_apply_jt<T>(s, u, in, out, nullptr, st, nullptr));
    else HIP_TRY(launch_apply_jt<T>(s, u, in, out, nullptr, st, nullptr));
    return PDHG_OK;
  }
  if (mode != PDHG_ADJ_SOLVE) return PDHG_EINVAL;
  if (dg) {
    const WsLayout L = layout_for(h->prob, h->esz);
    HIP_TRY(launch_dg_adjoint_march<T>(s, u, in, mu, out, (double*)wsp(ws, L.adj), st));
    return PDHG_OK;
  }
  HIP_TRY(launch_adjoint_march<T>(s, u, in, mu, out, st));
  return PDHG_OK;
}

// Launch one kernel of the unfused loop body `reps` times between two timing
// events on `st`, with the buffers of the last solve (status checks disabled).
template <typename T>
int time_kernel_impl(pdhg_handle* h, int kernel, int reps, double* ms, hipStream_t st) {
  const pdhg_problem& p = h->prob;
  void* ws = const_cast<void*>(h->last.ws);
  const WsLayout L = layout_for(p, h->esz);
  const Scheme s = scheme_of(h);
  T* u = (T*)const_cast<void*>(h->last.u);
  T* phi = (T*)const_cast<void*>(h->last.phi);
  T* u_alt = (T*)wsp(ws, L.u_alt);
  T* spec = (T*)wsp(ws, L.spec0);
  T* srow = (T*)wsp(ws, L.srow);
  T* phibar = (T*)wsp(ws, L.phibar);
  double* prp = (double*)wsp(ws, L.part_rp);
  double* prd = (double*)wsp(ws, L.part_rd);
  const size_t n = (size_t)p.nt * p.nx * planes(p);
  const T tu = (T)h->last.tau_u, tp = (T)h->last.tau_phi;
  Ctrl* ctrl_t = (Ctrl*)wsp(ws, L.ctrl_t);
  // B as in the steady state of a solve (Rp above eps: no dual residual)
  if (kernel == 0) HIP_TRY(launch_ctrl_init(ctrl_t, 1ll << 60, 0.0, 1e300, st, 1));
  const int nr = planes(p) * p.nt;
  auto launch_dg = [&]() -> hipError_t {
    switch (kernel) {
      case 1: return launch_dg_colsolve<T>(spec, factab<T>(h), (const T*)h->d_vtab, p.time == PDHG_BDF2 ? 2 : 1,
                                           p.nt, p.nx, h->lqb, nullptr, st, planes(p));
      case 4: return dgx_primal<T>(s, u, u_alt, phibar, phi, tu, prd, nullptr, st, nullptr);
      case 0: return launch_dg_residual_fft<T>(s, u_alt, spec, h->lqb, h->d_tw, prp, nullptr, st, nullptr);
      case 5: return dgx_residual<T>(s, u_alt, srow, prp, nullptr, st, nullptr);
      case 6: return launch_rows_fwd<T>(srow, nr, spec, nr, h->lqb, p.nx, h->d_tw, nullptr, st);
      case 7: return launch_dual_fft<T>(spec, nr, h->lqb, p.nx, h->d_tw, phi, phibar, tp, nullptr, st);
      case 8: return launch_copy<T>(srow, phibar, n, st);
      case 9:
        if constexpr (sizeof(T) == 4) return launch_dg_residual_mfma(s, (const float*)u_alt, (float*)srow, prp,
                                                                     nullptr, st, nullptr);
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
  };
  if (is_dg(p) && kernel == 9 && !(p.space == PDHG_DG_P2_LLF && p.dtype == PDHG_F32)) return PDHG_EUNSUPPORTED;
  if (is_dg(p) && !(kernel <= 1 || (kernel >= 4 && kernel <= 9))) return PDHG_EUNSUPPORTED;
  if (is_dg(p) && (kernel == 7 || kernel == 0) && p.nx < 64) return PDHG_EUNSUPPORTED;
  if (p.space == PDHG_DG_P1_UPWIND && kernel == 0) return PDHG_EUNSUPPORTED;   // fused residual + FFT: P2 only
  float* spec32 = (float*)spec;
  auto launch = [&]() -> hipError_t {
    if (is_dg(p)) return launch_dg();
    if (is_pre32(p) && h->last.variant == 2) {   // the fused passes as the solve ran them
      switch (kernel) {
        case 0:
          return launch_primal_res<T, float>(s, u, u_alt, phibar, phi, tu, spec32, h->lqb, h->d_tw32, prp, ctrl_t,
                                             st);
        case 7:
          return launch_dual_fft<T, float>(spec32, p.nt, h->lqb, p.nx, h->d_tw32, phi, phibar, tp, nullptr, st,
                                           (const T*)wsp(ws, L.s0));
        case 1:
          if (uses_chunks(p) && h->d_cmap)
            return launch_colsolve_chunk<float>(spec32, chunk_args(h, ws), p.time == PDHG_BDF2 ? 2 : 1, p.nt, p.nx,
                                                h->lqb, nullptr, nullptr, 0, 0.0, nullptr, st,
                                                (double*)wsp(ws, L.s0));
          return launch_colsolve_wave<float, double>(spec32, factab<double>(h), p.time == PDHG_BDF2 ? 2 : 1, p.nt,
                                                      p.nx, h->lqb, nullptr, nullptr, 0, 0.0, nullptr, st,
                                                      (double*)wsp(ws, L.s0));
        default: break;
      }
    }
    switch (kernel) {
      case 0: return launch_primal_res<T>(s, u, u_alt, phibar, phi, tu, spec, h->lqb, h->d_tw, prp, ctrl_t, st);
      case 7: return launch_dual_fft<T>(spec, p.nt, h->lqb, p.nx, h->d_tw, phi, phibar, tp, nullptr, st);
      case 1: return colsolve_any<T>(h, ws, spec, nullptr, nullptr, 0, nullptr, st);
      case 2: return launch_rows_inv<T>(spec, p.nt, h->lqb, srow, p.nt, p.nx, h->d_tw, nullptr, st);
      case 3: return launch_dual<T>(phi, phibar, srow, n, tp, nullptr, st);
      case 4: return launch_primal<T>(s, u, u_alt, phibar, phi, tu, prd, nullptr, st, nullptr);
      case 5: return launch_residual<T>(s, u_alt, srow, prp, nullptr, st, nullptr);
      case 6: return launch_rows_fwd<T>(srow, p.nt, spec, p.nt, h->lqb, p.nx, h->d_tw, nullptr, st);
      case 8: return launch_copy<T>(srow, phibar, n, st);   // plain copy: calibrates bandwidth and counters
      default: return hipErrorInvalidValue;
    }
  };
  if (kernel < 0 || kernel > (is_dg(p) ? 9 : 8)) return PDHG_EUNSUPPORTED;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(launch());   // warm-up
  HIP_TRY(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i) HIP_TRY(launch());
  HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(hipEventSynchronize(e1));
  float t = 0.f;
  HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *ms = (double)t / reps;
  return PDHG_OK;
}

}  // namespace

extern "C" {

int pdhg_residual(pdhg_handle* h, const void* u, const void* phi, void* Au, void* JTphi, double* res,
                  pdhg_stream_t stream) {
  if (!h || !u) return PDHG_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return set_hip_error(h, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (h->prob.dtype == PDHG_F64)
    return residual_impl<double>(h, (const double*)u, (const double*)phi, (double*)Au, (double*)JTphi, res, st);
  return residual_impl<float>(h, (const float*)u, (const float*)phi, (float*)Au, (float*)JTphi, res, st);
}

int pdhg_residual_static(pdhg_handle* h, const void* u, const void* phi, void* Au, void* JTphi, double* res,
                         pdhg_stream_t stream) {
  if (!h || !u) return PDHG_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return set_hip_error(h, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (h->prob.dtype == PDHG_F64)
    return residual_static_impl<double>(h, (const double*)u, (const double*)phi, (double*)Au, (double*)JTphi, res,
                                        st);
  return residual_static_impl<float>(h, (const float*)u, (const float*)phi, (float*)Au, (float*)JTphi, res, st);
}

int pdhg_precond(pdhg_handle* h, const void* r, void* s, pdhg_stream_t stream) {
  if (!h || !r || !s) return PDHG_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return set_hip_error(h, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (h->prob.dtype == PDHG_F64) return precond_impl<double>(h, (const double*)r, (double*)s, st);
  return precond_impl<float>(h, (const float*)r, (float*)s, st);
}

int pdhg_adjoint(pdhg_handle* h, int32_t mode, const void* u, const void* in, void* out, void* mu, void* workspace,
                 pdhg_stream_t stream) {
  if (!h || !u || !in || !out) return PDHG_EINVAL;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return set_hip_error(h, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (h->prob.dtype == PDHG_F64)
    return adjoint_impl<double>(h, mode, (const double*)u, (const double*)in, (double*)out, (double*)mu, workspace,
                                st);
  return adjoint_impl<float>(h, mode, (const float*)u, (const float*)in, (float*)out, (float*)mu, workspace, st);
}

int pdhg_time_kernel(pdhg_handle* h, int32_t kernel, int32_t reps, double* ms_per_launch, pdhg_stream_t stream) {
  if (!h || !ms_per_launch || reps < 1) return PDHG_EINVAL;
  if (!h->last.ws) return PDHG_EINVAL;   // needs a previous solve
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return set_hip_error(h, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (h->prob.dtype == PDHG_F64) return time_kernel_impl<double>(h, kernel, reps, ms_per_launch, st);
  return time_kernel_impl<float>(h, kernel, reps, ms_per_launch, st);
}

}  // extern "C"
