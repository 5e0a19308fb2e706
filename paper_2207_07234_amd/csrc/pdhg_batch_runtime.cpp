// Host runtime of the batched solver (C ABI pdhg_batch_*).
//
// Set-up packs the problems (offsets, problem table, twiddles per distinct
// N_x, tile orders).  A solve resolves each problem's flux constants from its
// u0 (one launch for the batch), builds the per-problem preconditioner factor
// tables on the host threads, estimates step sizes where none are given (the
// single-problem power iteration), then replays a captured HIP graph of
// `check_every` iterations (three batched passes per iteration, then the
// work-list rebuild) until no problem is left running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "pdhg.h"
#include "pdhg_internal.hpp"

using namespace pdhg;

namespace {
constexpr size_t kAlignB = 256;
inline size_t align_b(size_t x) { return (x + kAlignB - 1) & ~(kAlignB - 1); }
}  // namespace

struct pdhg_batch {
  int nprob = 0, dtype = 0, device = 0, ncu = 0;
  size_t esz = 8;
  std::vector<pdhg_problem> probs;
  std::vector<BatchProb> table;
  std::vector<int64_t> u0_off, u_off, f_off;
  int64_t u0_elems = 0, u_elems = 0, f_elems = 0;
  int total_pairs = 0, total_rtiles = 0, total_colg = 0, max_nx = 0;
  // device
  BatchProb* d_probs = nullptr;
  Ctrl* d_ctrls = nullptr;
  int2* d_row_tiles = nullptr;
  int2* d_col_tiles = nullptr;
  int* d_counts = nullptr;
  int* d_order = nullptr;
  int* d_corder = nullptr;
  double* d_part = nullptr;
  double* d_scal = nullptr;
  std::map<int, void*> d_tw;
  void* d_fac_rows = nullptr;
  int* d_fac_off = nullptr;
  int* d_fac_last = nullptr;
  std::vector<double> fac_c, fac_g;   // constants the current factor tables were built with
  std::vector<double> lf, c;
  // host staging (pinned)
  Ctrl* h_ctrls = nullptr;
  int* h_counts = nullptr;            // 2 slots of 4
  double* h_scal = nullptr;           // nprob
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;
  // persistent grid sizes of the passes A, B, C
  int grid[3] = {0, 0, 0};
  // graph cache
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  const void* gk_u = nullptr;
  const void* gk_phi = nullptr;
  const void* gk_ws = nullptr;
  int gk_chunk = 0, gk_grid[3] = {0, 0, 0};
  // one-time-step solver: symbols, per-step records, flags, nu, problem table
  void* os_buf = nullptr;
  size_t os_buf_bytes = 0;
  std::vector<double> os_c;
  // buffers of the last solve (kernel timing)
  const void* last_u0 = nullptr;
  void* last_u = nullptr;
  void* last_phi = nullptr;
  void* last_ws = nullptr;
  std::string err;
};

namespace {

int bset_hip_error(pdhg_batch* b, hipError_t e, const char* what) {
  if (b) b->err = std::string(what) + ": " + hipGetErrorString(e);
  return PDHG_EHIP;
}

#define BHIP_TRY(expr)                                         \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return bset_hip_error(b, e_, #expr); \
  } while (0)

bool is_pow2_b(int x) { return x > 0 && (x & (x - 1)) == 0; }

struct BatchWs {
  size_t u_alt, phibar, spec, ck_u, ck_phi, total;
};

BatchWs batch_ws(const pdhg_batch* b) {
  BatchWs L{};
  size_t o = 0;
  L.u_alt = o; o += align_b((size_t)b->u_elems * b->esz);
  L.phibar = o; o += align_b((size_t)b->f_elems * b->esz);
  L.spec = o; o += align_b((size_t)b->f_elems * b->esz);
  L.ck_u = o; o += align_b((size_t)b->u_elems * b->esz);     // last-good checkpoints of the packed (u, phi)
  L.ck_phi = o; o += align_b((size_t)b->f_elems * b->esz);
  L.total = o;
  return L;
}

BatchLaunch launch_of(const pdhg_batch* b) {
  BatchLaunch L{};
  L.probs = b->d_probs;
  L.ctrls = b->d_ctrls;
  L.row_tiles = b->d_row_tiles;
  L.col_tiles = b->d_col_tiles;
  L.counts = b->d_counts;
  L.order = b->d_order;
  L.corder = b->d_corder;
  L.nprob = b->nprob;
  L.max_nx = b->max_nx;
  return L;
}

template <typename T>
int upload_twiddles_b(pdhg_batch* b, int n) {
  std::vector<C2<T>> tw(n);
  const long double PI = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    const long double a = -2.0L * PI * i / n;
    tw[i] = C2<T>{(T)cosl(a), (T)sinl(a)};
  }
  void* d = nullptr;
  BHIP_TRY(hipMalloc(&d, n * sizeof(C2<T>)));
  b->d_tw[n] = d;
  BHIP_TRY(hipMemcpy(d, tw.data(), n * sizeof(C2<T>), hipMemcpyHostToDevice));
  return PDHG_OK;
}

template <typename T>
int setup_impl(pdhg_batch* b) {
  const int P = b->nprob;
  const int TB = batch_row_block_threads<T>();
  b->table.assign(P, BatchProb{});
  b->u0_off.resize(P);
  b->u_off.resize(P);
  b->f_off.resize(P);
  int64_t o0 = 0, ou = 0, of = 0;
  int pairs = 0, rt = 0, cg = 0;
  for (int i = 0; i < P; ++i) {
    const pdhg_problem& p = b->probs[i];
    BatchProb& q = b->table[i];
    q.s.nx = p.nx;
    q.s.nt = p.nt;
    q.s.time = p.time;
    q.s.space = p.space;
    q.s.ht = p.t_final / p.nt;
    q.s.hx = p.length / p.nx;
    q.s.alpha = p.alpha;
    q.s.beta = p.beta;
    q.s.gamma = p.gamma;
    q.s.lf = 0.0;
    b->u0_off[i] = o0;
    b->u_off[i] = ou;
    b->f_off[i] = of;
    q.u0_off = o0;
    q.u_off = ou;
    q.f_off = of;
    o0 += p.nx;
    ou += (int64_t)(p.nt + 1) * p.nx;
    of += (int64_t)p.nt * p.nx;
    int lqb = 0;
    while ((1 << (lqb + 1)) <= std::min(16, p.nx)) ++lqb;
    q.lqb = lqb;
    q.wscale = q.s.ht * q.s.hx;
    q.npairs = (p.nt + 1) / 2;
    q.part_off = pairs;
    pairs += q.npairs;
    const int W = batch_row_width<T>(p.nx);
    q.pairs_per_tile = TB / W;
    q.rtiles = (q.npairs + q.pairs_per_tile - 1) / q.pairs_per_tile;
    rt += q.rtiles;
    q.ncolg = p.nx / (p.nt <= 256 ? 16 : 8);   // column tiles: 16 columns of 16 lanes up to N_t = 256
    cg += q.ncolg;
    b->max_nx = std::max(b->max_nx, p.nx);
  }
  b->u0_elems = o0;
  b->u_elems = ou;
  b->f_elems = of;
  b->total_pairs = pairs;
  b->total_rtiles = rt;
  b->total_colg = cg;
  for (int i = 0; i < P; ++i) {
    const int n = b->probs[i].nx;
    if (!b->d_tw.count(n)) {
      int rc = upload_twiddles_b<T>(b, n);
      if (rc) return rc;
    }
    b->table[i].tw = b->d_tw[n];
  }
  // tile orders: rows in problem order, those of 4 points per thread before those of 8 (the primal pass runs
  // a grid for each); columns by decreasing nt (stable)
  std::vector<int> order(P), corder(P);
  for (int i = 0; i < P; ++i) order[i] = corder[i] = i;
  const int w4 = 4 * batch_row_block_threads<T>();   // widest row of 4 points per thread
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return (b->probs[x].nx > w4) < (b->probs[y].nx > w4); });
  std::stable_sort(corder.begin(), corder.end(),
                   [&](int x, int y) { return b->probs[x].nt > b->probs[y].nt; });
  BHIP_TRY(hipMalloc((void**)&b->d_probs, sizeof(BatchProb) * P));
  BHIP_TRY(hipMalloc((void**)&b->d_ctrls, sizeof(Ctrl) * P));
  BHIP_TRY(hipMalloc((void**)&b->d_row_tiles, sizeof(int2) * std::max(rt, 1)));
  BHIP_TRY(hipMalloc((void**)&b->d_col_tiles, sizeof(int2) * std::max(cg, 1)));
  BHIP_TRY(hipMalloc((void**)&b->d_counts, sizeof(int) * 4));
  BHIP_TRY(hipMalloc((void**)&b->d_order, sizeof(int) * P));
  BHIP_TRY(hipMalloc((void**)&b->d_corder, sizeof(int) * P));
  BHIP_TRY(hipMalloc((void**)&b->d_part, sizeof(double) * 2 * std::max(pairs, 1)));
  BHIP_TRY(hipMalloc((void**)&b->d_scal, sizeof(double) * P));
  BHIP_TRY(hipMemcpy(b->d_order, order.data(), sizeof(int) * P, hipMemcpyHostToDevice));
  BHIP_TRY(hipMemcpy(b->d_corder, corder.data(), sizeof(int) * P, hipMemcpyHostToDevice));
  BHIP_TRY(hipMemcpy(b->d_probs, b->table.data(), sizeof(BatchProb) * P, hipMemcpyHostToDevice));
  BHIP_TRY(hipHostMalloc((void**)&b->h_ctrls, sizeof(Ctrl) * P, hipHostMallocDefault));
  BHIP_TRY(hipHostMalloc((void**)&b->h_counts, sizeof(int) * 8, hipHostMallocDefault));
  BHIP_TRY(hipHostMalloc((void**)&b->h_scal, sizeof(double) * P, hipHostMallocDefault));
  for (int i = 0; i < 2; ++i) BHIP_TRY(hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming));
  BHIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  BHIP_TRY(hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, b->device));
  for (int k = 0; k < 3; ++k) {
    int occ = 1;
    BHIP_TRY(batch_occupancy<T>(k, b->max_nx, &occ));
    b->grid[k] = std::max(1, occ) * b->ncu;
  }
  b->fac_c.assign(P, -1.0);
  b->fac_g.assign(P, -1.0);
  b->lf.assign(P, 0.0);
  b->c.assign(P, 0.0);
  return PDHG_OK;
}

// Factor tables of every problem (host threads), pooled into one allocation.
template <typename T>
int build_factors_b(pdhg_batch* b) {
  const int P = b->nprob;
  std::vector<std::vector<FacRow<T>>> rows(P);
  std::vector<std::vector<int>> off(P), last(P);
  const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nth; ++t) {
    pool.emplace_back([&, t]() {
      for (int i = (int)t; i < P; i += (int)nth)
        build_factor_rows<T>(b->probs[i], b->c[i], b->probs[i].precond_gamma_hat, rows[i], off[i], last[i]);
    });
  }
  for (auto& th : pool) th.join();
  size_t nrows = 0, nmodes = 0;
  for (int i = 0; i < P; ++i) {
    nrows += rows[i].size();
    nmodes += off[i].size();
  }
  std::vector<FacRow<T>> all_rows;
  std::vector<int> all_off, all_last;
  all_rows.reserve(nrows);
  all_off.reserve(nmodes);
  all_last.reserve(nmodes);
  std::vector<size_t> rbase(P), mbase(P);
  for (int i = 0; i < P; ++i) {
    rbase[i] = all_rows.size();
    mbase[i] = all_off.size();
    all_rows.insert(all_rows.end(), rows[i].begin(), rows[i].end());
    all_off.insert(all_off.end(), off[i].begin(), off[i].end());
    all_last.insert(all_last.end(), last[i].begin(), last[i].end());
  }
  if (b->d_fac_rows) hipFree(b->d_fac_rows);
  if (b->d_fac_off) hipFree(b->d_fac_off);
  if (b->d_fac_last) hipFree(b->d_fac_last);
  b->d_fac_rows = nullptr;
  b->d_fac_off = b->d_fac_last = nullptr;
  BHIP_TRY(hipMalloc(&b->d_fac_rows, all_rows.size() * sizeof(FacRow<T>)));
  BHIP_TRY(hipMalloc((void**)&b->d_fac_off, all_off.size() * sizeof(int)));
  BHIP_TRY(hipMalloc((void**)&b->d_fac_last, all_last.size() * sizeof(int)));
  BHIP_TRY(hipMemcpy(b->d_fac_rows, all_rows.data(), all_rows.size() * sizeof(FacRow<T>), hipMemcpyHostToDevice));
  BHIP_TRY(hipMemcpy(b->d_fac_off, all_off.data(), all_off.size() * sizeof(int), hipMemcpyHostToDevice));
  BHIP_TRY(hipMemcpy(b->d_fac_last, all_last.data(), all_last.size() * sizeof(int), hipMemcpyHostToDevice));
  for (int i = 0; i < P; ++i) {
    b->table[i].fac_rows = static_cast<const FacRow<T>*>(b->d_fac_rows) + rbase[i];
    b->table[i].fac_off = b->d_fac_off + mbase[i];
    b->table[i].fac_last = b->d_fac_last + mbase[i];
    b->fac_c[i] = b->c[i];
    b->fac_g[i] = b->probs[i].precond_gamma_hat;
  }
  return PDHG_OK;
}

// Constants, factor tables and step sizes of every problem; uploads the table.
// nu[i] receives the power-iteration estimate (0 where steps were given).
// Each problem's lf_speed and c from its u0 where they default (one launch for the batch).
template <typename T>
int resolve_b(pdhg_batch* b, const T* u0, hipStream_t st) {
  const int P = b->nprob;
  BHIP_TRY(launch_batch_maxabs_dflux<T>(launch_of(b), u0, b->d_scal, st));
  BHIP_TRY(hipMemcpyAsync(b->h_scal, b->d_scal, sizeof(double) * P, hipMemcpyDeviceToHost, st));
  BHIP_TRY(hipStreamSynchronize(st));
  for (int i = 0; i < P; ++i) {
    const pdhg_problem& p = b->probs[i];
    const double m = b->h_scal[i];
    double lf = p.lf_speed < 0.0 ? m : p.lf_speed;
    if (p.space != PDHG_FD_LF) lf = 0.0;
    b->lf[i] = lf;
    b->c[i] = p.precond_c < 0.0 ? m : p.precond_c;
    b->table[i].s.lf = lf;
  }
  return PDHG_OK;
}

template <typename T>
int prepare(pdhg_batch* b, const T* u0, T* u, T* phi, const pdhg_batch_params* prm, std::vector<double>& tau_u,
            std::vector<double>& tau_phi, std::vector<double>& nu, hipStream_t st) {
  const int P = b->nprob;
  int rc0 = resolve_b<T>(b, u0, st);
  if (rc0) return rc0;
  bool refactor = b->d_fac_rows == nullptr;
  for (int i = 0; i < P; ++i)
    if (b->fac_c[i] != b->c[i] || b->fac_g[i] != b->probs[i].precond_gamma_hat) refactor = true;
  if (refactor) {
    int rc = build_factors_b<T>(b);
    if (rc) return rc;
  }
  tau_u.assign(P, 0.0);
  tau_phi.assign(P, 0.0);
  nu.assign(P, 0.0);
  for (int i = 0; i < P; ++i) {
    const double tu = prm->tau_u ? prm->tau_u[i] : 0.0;
    const double tp = prm->tau_phi ? prm->tau_phi[i] : 0.0;
    if (tu > 0.0 && tp > 0.0) {
      tau_u[i] = tu;
      tau_phi[i] = tp;
      continue;
    }
    // the single-problem power iteration on this problem's slices
    pdhg_problem q = b->probs[i];
    q.lf_speed = b->lf[i];
    q.precond_c = b->c[i];
    pdhg_handle* h = nullptr;
    int rc = pdhg_setup(&q, &h);
    if (rc) return rc;
    pdhg_params sp{};
    sp.max_iter = 0;        // set-up and power iteration only
    sp.check_every = 2;
    sp.warm_start = 1;      // leaves the caller's u (levels >= 1) and phi untouched
    pdhg_stats ss{};
    rc = pdhg_solve(h, u0 + b->u0_off[i], u + b->u_off[i], phi + b->f_off[i], nullptr, &sp, &ss, st);
    if (rc < 0) {
      b->err = std::string("step-size estimate of problem ") + std::to_string(i) + ": " + pdhg_last_error(h);
      pdhg_destroy(h);
      return rc;
    }
    pdhg_destroy(h);
    tau_u[i] = ss.tau_u;
    tau_phi[i] = ss.tau_phi;
    nu[i] = ss.nu_max;
  }
  for (int i = 0; i < P; ++i) {
    b->table[i].tau_u = tau_u[i];
    b->table[i].tau_phi = tau_phi[i];
  }
  BHIP_TRY(hipMemcpyAsync(b->d_probs, b->table.data(), sizeof(BatchProb) * P, hipMemcpyHostToDevice, st));
  BHIP_TRY(hipStreamSynchronize(st));
  return PDHG_OK;
}

inline char* bws(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

// One iteration of every running problem: A, B, C.  `odd` selects the u
// ping-pong direction (odd iterations read u and write u_alt).
template <typename T>
int enqueue_batch_body(pdhg_batch* b, bool odd, T* u, T* phi, void* ws, const int* grid, hipStream_t st) {
  const BatchWs W = batch_ws(b);
  const BatchLaunch L = launch_of(b);
  T* u_alt = (T*)bws(ws, W.u_alt);
  T* phibar = (T*)bws(ws, W.phibar);
  T* spec = (T*)bws(ws, W.spec);
  T* uin = odd ? u : u_alt;
  T* uout = odd ? u_alt : u;
  BHIP_TRY(launch_batch_dual_fft<T>(L, grid[0], spec, phi, phibar, st));
  BHIP_TRY(launch_batch_primal_res<T>(L, grid[1], uin, uout, phibar, phi, spec, b->d_part, b->total_pairs, st));
  BHIP_TRY(launch_batch_colsolve<T>(L, grid[2], spec, b->d_part, b->total_pairs, st));
  return PDHG_OK;
}

template <typename T>
int build_batch_graph(pdhg_batch* b, int chunk, T* u, T* phi, void* ws, const int* grid) {
  if (b->gexec && b->gk_u == u && b->gk_phi == phi && b->gk_ws == ws && b->gk_chunk == chunk &&
      std::equal(grid, grid + 3, b->gk_grid))
    return PDHG_OK;
  if (b->gexec) { hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
  if (b->graph) { hipGraphDestroy(b->graph); b->graph = nullptr; }
  BHIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = PDHG_OK;
  for (int k = 0; k < chunk && rc == PDHG_OK; ++k)
    rc = enqueue_batch_body<T>(b, (k % 2) == 0, u, phi, ws, grid, b->cap_stream);
  if (rc == PDHG_OK) {
    hipError_t e = launch_batch_compact(launch_of(b), b->cap_stream);
    if (e != hipSuccess) rc = bset_hip_error(b, e, "launch_batch_compact");
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (rc) { if (g) hipGraphDestroy(g); return rc; }
  if (e != hipSuccess) return bset_hip_error(b, e, "hipStreamEndCapture");
  b->graph = g;
  BHIP_TRY(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
  b->gk_u = u;
  b->gk_phi = phi;
  b->gk_ws = ws;
  b->gk_chunk = chunk;
  std::copy(grid, grid + 3, b->gk_grid);
  return PDHG_OK;
}

// Persistent grids for the tiles still running: the tuned grid of a pass divided by 4 while a quarter of it
// still gives every tile a block (row tiles for A and B, column tiles for C) and every CU one; any grid
// covers all tiles, so only the time changes.
static void running_grids(const pdhg_batch* b, int row_tiles, int col_tiles, int* grid) {
  auto shrink = [&](int g, int n) {
    const int floor = std::max(n, b->ncu);
    while (g / 4 >= floor) g /= 4;
    return g;
  };
  grid[0] = shrink(b->grid[0], row_tiles);
  grid[1] = shrink(b->grid[1], row_tiles);
  grid[2] = shrink(b->grid[2], col_tiles);
}

// Copy problem i's slices of a checkpoint into u and phi and recompute its residual norms and
// mass drift there (scratch: a spectrum-sized workspace region, free after the loop).
template <typename T>
int restore_checkpoint(pdhg_batch* b, int i, const T* cku, const T* ckphi, T* u, T* phi, double* scratch,
                       hipStream_t st, double* rp, double* rd, double* drift) {
  const pdhg_problem& q = b->probs[i];
  const size_t nlev = (size_t)(q.nt + 1) * q.nx, nf = (size_t)q.nt * q.nx;
  T* ui = u + b->u_off[i];
  T* pi = phi + b->f_off[i];
  BHIP_TRY(launch_copy<T>(ui, cku + b->u_off[i], nlev, st));
  BHIP_TRY(launch_copy<T>(pi, ckphi + b->f_off[i], nf, st));
  const Scheme& s = b->table[i].s;
  const size_t np = (nf + 255) / 256;
  double* prp = scratch;
  double* prd = scratch + np;
  double* lev = scratch + 2 * np;
  int nb1 = 0, nb2 = 0;
  BHIP_TRY(launch_residual<T>(s, ui, (T*)nullptr, prp, nullptr, st, &nb1));
  BHIP_TRY(launch_apply_jt<T>(s, ui, pi, (T*)nullptr, prd, st, &nb2));
  BHIP_TRY(launch_level_sums<T>(ui, q.nx, (size_t)q.nx, q.nt + 1, lev, st));
  std::vector<double> h(2 * np + q.nt + 1);
  BHIP_TRY(hipMemcpyAsync(h.data(), scratch, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  BHIP_TRY(hipStreamSynchronize(st));
  double sa = 0.0, sb = 0.0;
  for (int k = 0; k < nb1; ++k) sa += h[k];
  for (int k = 0; k < nb2; ++k) sb += h[np + k];
  *rp = std::sqrt(s.ht * s.hx * sa);
  *rd = std::sqrt(s.ht * s.hx * sb);
  double d = 0.0;
  for (int l = 1; l <= q.nt; ++l) d = std::max(d, std::fabs(h[2 * np + l] - h[2 * np]) * s.hx);
  *drift = d;
  return PDHG_OK;
}

template <typename T>
int batch_solve_impl(pdhg_batch* b, const T* u0, T* u, T* phi, void* ws, const pdhg_batch_params* prm,
                     pdhg_stats* stats, hipStream_t st) {
  const int P = b->nprob;
  std::vector<double> tau_u, tau_phi, nu;
  int rc = prepare<T>(b, u0, u, phi, prm, tau_u, tau_phi, nu, st);
  if (rc) return rc;
  const BatchWs W = batch_ws(b);
  const BatchLaunch L = launch_of(b);
  T* u_alt = (T*)bws(ws, W.u_alt);
  T* spec = (T*)bws(ws, W.spec);
  const double div = prm->diverge_factor > 0 ? prm->diverge_factor : 1e6;
  BHIP_TRY(launch_batch_init<T>(L, u0, u, u_alt, phi, spec, prm->warm_start ? 1 : 0, (long long)prm->max_iter,
                                prm->eps, div, st));
  BHIP_TRY(launch_batch_compact(L, st));
  int chunk = prm->check_every > 0 ? prm->check_every : 64;
  chunk += chunk & 1;   // even: the u ping-pong returns to its start buffer
  b->last_u0 = u0;
  b->last_u = u;
  b->last_phi = phi;
  b->last_ws = ws;
  // last-good checkpoints of every running problem, refreshed on the device after each chunk
  T* ck_u = (T*)bws(ws, W.ck_u);
  T* ck_phi = (T*)bws(ws, W.ck_phi);
  auto t0 = std::chrono::steady_clock::now();
  // graphs of grids shrunk as problems drop out: kept until the stream has drained (a launch may be in flight)
  std::vector<hipGraphExec_t> retired_exec;
  std::vector<hipGraph_t> retired_graph;
  auto retire_all = [&]() {
    for (hipGraphExec_t g : retired_exec) hipGraphExecDestroy(g);
    for (hipGraph_t g : retired_graph) hipGraphDestroy(g);
    retired_exec.clear();
    retired_graph.clear();
  };
  if (prm->max_iter > 0) {
    BHIP_TRY(launch_batch_checkpoint<T>(L, u_alt, phi, ck_u, ck_phi, st));   // iterate 0
    int run[3] = {b->grid[0], b->grid[1], b->grid[2]};
    rc = build_batch_graph<T>(b, chunk, u, phi, ws, run);
    if (rc) return rc;
    const long long bodies = prm->max_iter + 1;
    long long launched = 0;
    int idx = 0;
    bool stop = false;
    while (!stop && launched < bodies) {
      hipError_t le = hipGraphLaunch(b->gexec, st);
      if (le != hipSuccess) {
        hipStreamSynchronize(st);
        retire_all();
        return bset_hip_error(b, le, "hipGraphLaunch");
      }
      launched += chunk;
      BHIP_TRY(launch_batch_checkpoint<T>(L, u_alt, phi, ck_u, ck_phi, st));
      int* slot = b->h_counts + 4 * (idx & 1);
      BHIP_TRY(hipMemcpyAsync(slot, b->d_counts, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
      BHIP_TRY(hipEventRecord(b->ev[idx & 1], st));
      if (idx >= 1) {
        BHIP_TRY(hipEventSynchronize(b->ev[(idx - 1) & 1]));
        const int* c = b->h_counts + 4 * ((idx - 1) & 1);
        if (c[2] == 0) {
          stop = true;
        } else if (launched < bodies) {
          int want[3];
          running_grids(b, c[0], c[1], want);
          if (!std::equal(want, want + 3, run)) {
            retired_exec.push_back(b->gexec);
            retired_graph.push_back(b->graph);
            b->gexec = nullptr;
            b->graph = nullptr;
            std::copy(want, want + 3, run);
            rc = build_batch_graph<T>(b, chunk, u, phi, ws, run);
            if (rc) {
              hipStreamSynchronize(st);
              retire_all();
              return rc;
            }
          }
        }
      }
      ++idx;
    }
  }
  BHIP_TRY(launch_batch_finish<T>(L, u, u_alt, b->d_scal, st));
  BHIP_TRY(hipMemcpyAsync(b->h_ctrls, b->d_ctrls, sizeof(Ctrl) * P, hipMemcpyDeviceToHost, st));
  BHIP_TRY(hipMemcpyAsync(b->h_scal, b->d_scal, sizeof(double) * P, hipMemcpyDeviceToHost, st));
  BHIP_TRY(hipStreamSynchronize(st));
  retire_all();
  auto t1 = std::chrono::steady_clock::now();
  const double secs = std::chrono::duration<double>(t1 - t0).count();
  int worst = PDHG_OK;
  for (int i = 0; i < P; ++i) {
    const Ctrl& c = b->h_ctrls[i];
    int status;
    long long nstar = c.n_star;
    double rp = c.rp_star, rd = c.rd_star, drift = b->h_scal[i];
    if (prm->max_iter <= 0) { nstar = 0; status = PDHG_NOT_CONVERGED; }
    else if (c.status == 1) status = PDHG_OK;
    else if (c.status == 2) status = PDHG_DIVERGED;
    else status = PDHG_NOT_CONVERGED;
    if (status == PDHG_DIVERGED) {   // back to the last good checkpoint
      rc = restore_checkpoint<T>(b, i, ck_u, ck_phi, u, phi, (double*)bws(ws, W.spec), st, &rp, &rd, &drift);
      if (rc) return rc;
      nstar = c.ck_iter > 0 ? c.ck_iter : 0;
    }
    if (status == PDHG_DIVERGED) worst = PDHG_DIVERGED;
    else if (status == PDHG_NOT_CONVERGED && worst == PDHG_OK) worst = PDHG_NOT_CONVERGED;
    if (stats) {
      pdhg_stats& s = stats[i];
      s.iters = nstar;
      s.res_primal = rp;
      s.res_dual = rd;
      s.tau_u = tau_u[i];
      s.tau_phi = tau_phi[i];
      s.nu_max = nu[i];
      s.lf_speed = b->lf[i];
      s.precond_c = b->c[i];
      s.seconds = secs;
      s.mass_drift = drift;
      s.status = status;
      s.variant = 3;
    }
  }
  return worst;
}

// Algorithm 3 for every problem of the batch: one launch of the one-step march
// with a block per problem (after one power-iteration launch where step sizes
// are not given).  Problems are tabled in decreasing N_t N_x order so that the
// longest marches start first when there are more problems than compute units.
template <typename T>
int batch_onestep_impl(pdhg_batch* b, const T* u0, T* u, T* phi, const pdhg_batch_params* prm, pdhg_stats* stats,
                       int64_t* step_iters, hipStream_t st) {
  const int P = b->nprob;
  int rc = resolve_b<T>(b, u0, st);
  if (rc) return rc;
  std::vector<size_t> sym_off(P), st_off(P);
  size_t nsym = 0, nst = 0;
  int max_nt = 0;
  for (int i = 0; i < P; ++i) {
    sym_off[i] = nsym;
    st_off[i] = nst;
    nsym += 2 * (size_t)b->probs[i].nx + 32;   // symbol [2][nx], cyclic-reduction coefficients [2][16]
    nst += (size_t)b->probs[i].nt;
    max_nt = std::max(max_nt, b->probs[i].nt);
  }
  const size_t b_sym = align_b(nsym * sizeof(T)), b_stat = align_b(nst * sizeof(StepStat));
  const size_t b_flag = align_b(P * sizeof(int)), b_nu = align_b(P * sizeof(double));
  const size_t need = b_sym + b_stat + b_flag + b_nu + align_b(P * sizeof(OneStepProb<T>));
  if (b->os_buf_bytes < need) {
    if (b->os_buf) hipFree(b->os_buf);
    b->os_buf = nullptr;
    b->os_buf_bytes = 0;
    b->os_c.clear();
    BHIP_TRY(hipMalloc(&b->os_buf, need));
    b->os_buf_bytes = need;
  }
  char* base = static_cast<char*>(b->os_buf);
  T* sym = (T*)base;
  StepStat* stat = (StepStat*)(base + b_sym);
  int* flag = (int*)(base + b_sym + b_stat);
  double* nu_d = (double*)(base + b_sym + b_stat + b_flag);
  OneStepProb<T>* tab = (OneStepProb<T>*)(base + b_sym + b_stat + b_flag + b_nu);
  std::vector<int> pk(2 * (size_t)P, 0);
  std::vector<double> pcr(32 * (size_t)P, 0.0);
  for (int i = 0; i < P; ++i)
    if (!onestep_pcr(b->probs[i], b->c[i], sizeof(T) == 8 ? 1e-17 : 1e-9, &pcr[32 * (size_t)i], &pk[2 * (size_t)i]))
      pk[2 * (size_t)i] = pk[2 * (size_t)i + 1] = 0;
  if (b->os_c != b->c) {
    std::vector<T> hs(nsym, T(0));
    for (int i = 0; i < P; ++i) {
      const size_t nx2 = 2 * (size_t)b->probs[i].nx;
      onestep_symbol<T>(b->probs[i], b->c[i], b->lf[i], hs.data() + sym_off[i]);
      for (int q = 0; q < 32; ++q) hs[sym_off[i] + nx2 + q] = (T)pcr[32 * (size_t)i + q];
    }
    BHIP_TRY(hipMemcpyAsync(sym, hs.data(), nsym * sizeof(T), hipMemcpyHostToDevice, st));
    BHIP_TRY(hipStreamSynchronize(st));
    b->os_c = b->c;
  }
  BHIP_TRY(hipMemsetAsync(flag, 0, P * sizeof(int), st));
  BHIP_TRY(hipMemsetAsync(stat, 0, nst * sizeof(StepStat), st));
  std::vector<int> order(P);
  for (int i = 0; i < P; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return (long long)b->probs[x].nt * b->probs[x].nx > (long long)b->probs[y].nt * b->probs[y].nx;
  });
  std::vector<OneStepProb<T>> tp(P);
  bool any_auto = false;
  for (int r = 0; r < P; ++r) {
    const int i = order[r];
    OneStepProb<T>& e = tp[r];
    e.s = b->table[i].s;
    e.tw = (const C2<T>*)b->d_tw.at(b->probs[i].nx);
    e.sym = sym + sym_off[i];
    e.pcr = e.sym + 2 * (size_t)b->probs[i].nx;
    e.pcr_k[0] = pk[2 * (size_t)i];
    e.pcr_k[1] = pk[2 * (size_t)i + 1];
    e.u0 = u0 + b->u0_off[i];
    e.u = u + b->u_off[i];
    e.phi = phi + b->f_off[i];
    e.stat = stat + st_off[i];
    e.flag = flag + i;
    const double tu = prm->tau_u ? prm->tau_u[i] : 0.0, tq = prm->tau_phi ? prm->tau_phi[i] : 0.0;
    const bool given = tu > 0.0 && tq > 0.0;
    e.tau_u = given ? tu : 0.0;
    e.tau_phi = given ? tq : 0.0;
    any_auto = any_auto || !given;
  }
  BHIP_TRY(hipMemcpyAsync(tab, tp.data(), P * sizeof(OneStepProb<T>), hipMemcpyHostToDevice, st));
  BHIP_TRY(hipMemsetAsync(nu_d, 0, P * sizeof(double), st));
  if (any_auto) BHIP_TRY(launch_onestep_power<T>(tab, P, b->max_nx, 200, nu_d, st));
  BHIP_TRY(hipStreamSynchronize(st));
  const double div = prm->diverge_factor > 0 ? prm->diverge_factor : 1e6;
  auto t0 = std::chrono::steady_clock::now();
  BHIP_TRY(launch_onestep<T>(tab, P, b->max_nx, 0, max_nt, prm->eps, (long long)prm->max_iter, div, st));
  std::vector<StepStat> rec(nst);
  std::vector<double> nu(P);
  BHIP_TRY(hipMemcpyAsync(rec.data(), stat, nst * sizeof(StepStat), hipMemcpyDeviceToHost, st));
  BHIP_TRY(hipMemcpyAsync(tp.data(), tab, P * sizeof(OneStepProb<T>), hipMemcpyDeviceToHost, st));
  BHIP_TRY(hipMemcpyAsync(nu.data(), nu_d, P * sizeof(double), hipMemcpyDeviceToHost, st));
  BHIP_TRY(hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  const double secs = std::chrono::duration<double>(t1 - t0).count();
  int worst = PDHG_OK;
  for (int r = 0; r < P; ++r) {
    const int i = order[r];
    const OneStepSummary sm = summarize_steps(rec.data() + st_off[i], b->probs[i].nt,
                                              step_iters ? step_iters + st_off[i] : nullptr, nullptr);
    if (!(tp[r].tau_u > 0.0)) {
      b->err = std::string("step-size estimate of problem ") + std::to_string(i) + " failed";
      return PDHG_EINVAL;
    }
    if (sm.status == PDHG_DIVERGED) worst = PDHG_DIVERGED;
    else if (sm.status == PDHG_NOT_CONVERGED && worst == PDHG_OK) worst = PDHG_NOT_CONVERGED;
    if (stats) {
      pdhg_stats& s = stats[i];
      s.iters = sm.total;
      s.res_primal = sm.rp;
      s.res_dual = sm.rd;
      s.tau_u = tp[r].tau_u;
      s.tau_phi = tp[r].tau_phi;
      s.nu_max = nu[r];
      s.lf_speed = b->lf[i];
      s.precond_c = b->c[i];
      s.seconds = secs;
      s.mass_drift = -1.0;
      s.status = sm.status;
      s.variant = 5;
    }
  }
  return worst;
}

// Average device time of one launch of pass k with `grid` blocks (events per
// launch; for the column pass a primal pass refills the spectrum before each
// timed launch).
template <typename T>
int time_pass(pdhg_batch* b, int k, int grid, T* u, T* phi, void* ws, hipStream_t st, double* ms, int reps = 8) {
  const BatchWs W = batch_ws(b);
  const BatchLaunch L = launch_of(b);
  T* u_alt = (T*)bws(ws, W.u_alt);
  T* phibar = (T*)bws(ws, W.phibar);
  T* spec = (T*)bws(ws, W.spec);
  hipEvent_t e0, e1;
  BHIP_TRY(hipEventCreate(&e0));
  BHIP_TRY(hipEventCreate(&e1));
  double total = 0.0;
  const int warm = 2;
  for (int r = 0; r < warm + reps; ++r) {
    if (k == 2)
      BHIP_TRY(launch_batch_primal_res<T>(L, b->grid[1], u, u_alt, phibar, phi, spec, b->d_part, b->total_pairs, st));
    BHIP_TRY(hipEventRecord(e0, st));
    if (k == 0) BHIP_TRY(launch_batch_dual_fft<T>(L, grid, spec, phi, phibar, st));
    else if (k == 1)
      BHIP_TRY(launch_batch_primal_res<T>(L, grid, u, u_alt, phibar, phi, spec, b->d_part, b->total_pairs, st));
    else BHIP_TRY(launch_batch_colsolve<T>(L, grid, spec, b->d_part, b->total_pairs, st));
    BHIP_TRY(hipEventRecord(e1, st));
    BHIP_TRY(hipEventSynchronize(e1));
    float t = 0.f;
    BHIP_TRY(hipEventElapsedTime(&t, e0, e1));
    if (r >= warm) total += t;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *ms = total / reps;
  return PDHG_OK;
}

template <typename T>
int batch_tune_impl(pdhg_batch* b, const T* u0, T* u, T* phi, void* ws, const pdhg_batch_params* prm, int32_t* out,
                    hipStream_t st) {
  std::vector<double> tau_u, tau_phi, nu;
  int rc = prepare<T>(b, u0, u, phi, prm, tau_u, tau_phi, nu, st);
  if (rc) return rc;
  const BatchWs W = batch_ws(b);
  const BatchLaunch L = launch_of(b);
  // the control blocks stay "running" during timing: huge max_iter, no tolerance
  BHIP_TRY(launch_batch_init<T>(L, u0, u, (T*)bws(ws, W.u_alt), phi, (T*)bws(ws, W.spec), 0, 1ll << 60, 0.0, 1e300,
                                st));
  BHIP_TRY(launch_batch_compact(L, st));
  const int ntiles[3] = {b->total_rtiles, b->total_rtiles, b->total_colg};
  for (int k = 0; k < 3; ++k) {
    int occ = 1;
    BHIP_TRY(batch_occupancy<T>(k, b->max_nx, &occ));
    occ = std::max(occ, 1);
    std::vector<int> cand;
    for (int m : {1, 2, 4, 8})
      if (m <= occ) cand.push_back(m * b->ncu);
    cand.push_back(ntiles[k]);
    double best = 1e300;
    int best_g = b->grid[k];
    for (int g : cand) {
      if (g < 1) continue;
      double ms = 0.0;
      rc = time_pass<T>(b, k, g, u, phi, ws, st, &ms);
      if (rc) return rc;
      if (ms < best) { best = ms; best_g = g; }
    }
    b->grid[k] = best_g;
  }
  if (out)
    for (int k = 0; k < 3; ++k) out[k] = b->grid[k];
  return PDHG_OK;
}

// Time pass k on the last solve's buffers, every problem running again.
template <typename T>
int time_kernel_b(pdhg_batch* b, int k, int reps, double* ms, hipStream_t st) {
  const BatchWs W = batch_ws(b);
  void* ws = b->last_ws;
  T* u = (T*)b->last_u;
  BHIP_TRY(launch_batch_init<T>(launch_of(b), (const T*)b->last_u0, u, (T*)bws(ws, W.u_alt), (T*)b->last_phi,
                                (T*)bws(ws, W.spec), 0, 1ll << 60, 0.0, 1e300, st));
  BHIP_TRY(launch_batch_compact(launch_of(b), st));
  return time_pass<T>(b, k, b->grid[k], u, (T*)b->last_phi, ws, st, ms, reps);
}

int validate_batch_problem(const pdhg_problem& p, int dtype) {
  if (!is_pow2_b(p.nx) || p.nt < 1) return PDHG_EINVAL;
  if (!(p.length > 0) || !(p.t_final > 0) || p.gamma < 0 || p.precond_gamma_hat < 0) return PDHG_EINVAL;
  if (p.time != PDHG_BE && p.time != PDHG_BDF2) return PDHG_EINVAL;
  if (p.space != PDHG_FD_UPWIND && p.space != PDHG_FD_LF) return PDHG_EINVAL;
  if (p.dtype != PDHG_F32 && p.dtype != PDHG_F64) return PDHG_EINVAL;
  if (p.dtype != dtype) return PDHG_EINVAL;
  if (p.precond_kind != PDHG_PRECOND_GRAM) return PDHG_EUNSUPPORTED;   // batches use the Gram preconditioner
  if (p.nx < 256 || p.nx > 4096 || p.nt > 512) return PDHG_EUNSUPPORTED;
  return PDHG_OK;
}

}  // namespace

extern "C" {

int pdhg_batch_setup(const pdhg_problem* probs, int32_t nprob, pdhg_batch** out) {
  if (!probs || !out || nprob < 1) return PDHG_EINVAL;
  *out = nullptr;
  for (int i = 0; i < nprob; ++i) {
    const int rc = validate_batch_problem(probs[i], probs[0].dtype);
    if (rc) return rc;
  }
  pdhg_batch* b = new (std::nothrow) pdhg_batch();
  if (!b) return PDHG_EINVAL;
  b->nprob = nprob;
  b->dtype = probs[0].dtype;
  b->esz = b->dtype == PDHG_F64 ? 8 : 4;
  b->probs.assign(probs, probs + nprob);
  int rc = PDHG_OK;
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) rc = bset_hip_error(b, e, "hipGetDevice");
  if (!rc) rc = b->dtype == PDHG_F64 ? setup_impl<double>(b) : setup_impl<float>(b);
  if (rc) {
    pdhg_batch_destroy(b);
    return rc;
  }
  *out = b;
  return PDHG_OK;
}

int pdhg_batch_sizes(const pdhg_batch* b, int64_t* u0_elems, int64_t* u_elems, int64_t* phi_elems,
                     size_t* workspace_bytes) {
  if (!b) return PDHG_EINVAL;
  if (u0_elems) *u0_elems = b->u0_elems;
  if (u_elems) *u_elems = b->u_elems;
  if (phi_elems) *phi_elems = b->f_elems;
  if (workspace_bytes) *workspace_bytes = batch_ws(b).total;
  return PDHG_OK;
}

int pdhg_batch_offsets(const pdhg_batch* b, int32_t i, int64_t* u0_off, int64_t* u_off, int64_t* phi_off) {
  if (!b || i < 0 || i >= b->nprob) return PDHG_EINVAL;
  if (u0_off) *u0_off = b->u0_off[i];
  if (u_off) *u_off = b->u_off[i];
  if (phi_off) *phi_off = b->f_off[i];
  return PDHG_OK;
}

int pdhg_batch_solve(pdhg_batch* b, const void* u0, void* u, void* phi, void* workspace,
                     const pdhg_batch_params* params, pdhg_stats* stats, pdhg_stream_t stream) {
  if (!b || !u0 || !u || !phi || !workspace || !params || params->max_iter < 0) return PDHG_EINVAL;
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return bset_hip_error(b, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (b->dtype == PDHG_F64)
    return batch_solve_impl<double>(b, (const double*)u0, (double*)u, (double*)phi, workspace, params, stats, st);
  return batch_solve_impl<float>(b, (const float*)u0, (float*)u, (float*)phi, workspace, params, stats, st);
}

int pdhg_batch_solve_onestep(pdhg_batch* b, const void* u0, void* u, void* phi, const pdhg_batch_params* params,
                             pdhg_stats* stats, int64_t* step_iters, pdhg_stream_t stream) {
  if (!b || !u0 || !u || !phi || !params || params->max_iter < 0) return PDHG_EINVAL;
  if (b->max_nx < 64) return PDHG_EUNSUPPORTED;
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return bset_hip_error(b, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (b->dtype == PDHG_F64)
    return batch_onestep_impl<double>(b, (const double*)u0, (double*)u, (double*)phi, params, stats, step_iters, st);
  return batch_onestep_impl<float>(b, (const float*)u0, (float*)u, (float*)phi, params, stats, step_iters, st);
}

int pdhg_batch_tune(pdhg_batch* b, const void* u0, void* u, void* phi, void* workspace,
                    const pdhg_batch_params* params, int32_t* grids, pdhg_stream_t stream) {
  if (!b || !u0 || !u || !phi || !workspace || !params) return PDHG_EINVAL;
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return bset_hip_error(b, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (b->dtype == PDHG_F64)
    return batch_tune_impl<double>(b, (const double*)u0, (double*)u, (double*)phi, workspace, params, grids, st);
  return batch_tune_impl<float>(b, (const float*)u0, (float*)u, (float*)phi, workspace, params, grids, st);
}

void pdhg_batch_destroy(pdhg_batch* b) {
  if (!b) return;
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (auto& kv : b->d_tw) hipFree(kv.second);
  if (b->d_fac_rows) hipFree(b->d_fac_rows);
  if (b->d_fac_off) hipFree(b->d_fac_off);
  if (b->d_fac_last) hipFree(b->d_fac_last);
  if (b->d_probs) hipFree(b->d_probs);
  if (b->d_ctrls) hipFree(b->d_ctrls);
  if (b->d_row_tiles) hipFree(b->d_row_tiles);
  if (b->d_col_tiles) hipFree(b->d_col_tiles);
  if (b->d_counts) hipFree(b->d_counts);
  if (b->d_order) hipFree(b->d_order);
  if (b->d_corder) hipFree(b->d_corder);
  if (b->d_part) hipFree(b->d_part);
  if (b->d_scal) hipFree(b->d_scal);
  if (b->os_buf) hipFree(b->os_buf);
  if (b->h_ctrls) hipHostFree(b->h_ctrls);
  if (b->h_counts) hipHostFree(b->h_counts);
  if (b->h_scal) hipHostFree(b->h_scal);
  for (int i = 0; i < 2; ++i)
    if (b->ev[i]) hipEventDestroy(b->ev[i]);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  delete b;
}

int pdhg_batch_time_kernel(pdhg_batch* b, int32_t kernel, int32_t reps, double* ms_per_launch,
                           pdhg_stream_t stream) {
  if (!b || !ms_per_launch || kernel < 0 || kernel > 2 || reps < 1) return PDHG_EINVAL;
  if (!b->last_ws) return PDHG_EINVAL;
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return bset_hip_error(b, e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  if (b->dtype == PDHG_F64) return time_kernel_b<double>(b, kernel, reps, ms_per_launch, st);
  return time_kernel_b<float>(b, kernel, reps, ms_per_launch, st);
}

const char* pdhg_batch_last_error(const pdhg_batch* b) { return b ? b->err.c_str() : "null handle"; }

}  // extern "C"
