"""Space-time primal-dual solver for implicit conservation-law schemes on MI355X.

Python face of the HIP library libpdhg.so (include/pdhg.h).  The method is
Algorithm 1 of Liu, Osher, Li, Shu, "A primal-dual approach for solving
conservation laws with implicit in time approximations": the whole implicit
space-time system A(u) = 0 (backward Euler or BDF2 in time, finite
differences in space, Sections 3.1-3.2) is solved as the saddle point of
<phi, A(u)> by a preconditioned primal-dual hybrid gradient iteration.

Every numerical step runs in the HIP kernels; this module only passes torch
device pointers and the current stream across the C ABI.

    import torch, paper_2207_07234_amd as pk
    prob = pk.Problem(nx=2048, nt=512, t_final=0.5, alpha=0.5, beta=0.0,
                      time="bdf2", space="fd_lf", dtype=torch.float64)
    solver = pk.Solver(prob)
    res = solver.solve(u0, eps=1e-8, max_iter=50000)
    res.u, res.phi, res.stats
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional

from . import _binding as B

__all__ = ["Problem", "Solver", "SolveResult", "BatchSolver", "BatchResult", "PdhgError", "lib_path",
           "differentiable_solve"]

lib_path = B.LIB_PATH
_TIME = {"be": B.PDHG_BE, "bdf2": B.PDHG_BDF2}
_SPACE = {"fd_upwind": B.PDHG_FD_UPWIND, "fd_lf": B.PDHG_FD_LF, "dg_p2_llf": B.PDHG_DG_P2_LLF,
          "dg_p1_upwind": B.PDHG_DG_P1_UPWIND}


class PdhgError(RuntimeError):
    pass


@dataclass
class Problem:
    """u_t + (alpha u^2 + beta u)_x - gamma u_xx = 0 on [0, length) x [0, t_final], periodic."""
    nx: int
    nt: int
    length: float = 1.0
    t_final: float = 1.0
    alpha: float = 0.0
    beta: float = 1.0
    gamma: float = 0.0
    time: str = "be"
    space: str = "fd_upwind"
    dtype: object = None            # torch.float32 / torch.float64 (default float64)
    lf_speed: float = -1.0          # < 0: max |f'(u0)|
    precond_c: float = -1.0         # < 0: max |f'(u0)| ("gram") or mean f'(u0) ("full")
    precond_gamma_hat: float = 0.0
    precond_kind: str = "gram"      # "gram" (Section 3.3), "full" (with the cross term), or "gram_f32"
                                    # (FP64 problem, the Gram preconditioner's spectral pass in float)

    def to_c(self) -> B.pdhg_problem:
        import torch
        dt = torch.float64 if self.dtype is None else self.dtype
        p = B.pdhg_problem()
        p.nx, p.nt = int(self.nx), int(self.nt)
        p.length, p.t_final = float(self.length), float(self.t_final)
        p.alpha, p.beta, p.gamma = float(self.alpha), float(self.beta), float(self.gamma)
        p.time, p.space = _TIME[self.time], _SPACE[self.space]
        p.dtype = B.PDHG_F64 if dt == torch.float64 else B.PDHG_F32
        p.lf_speed, p.precond_c = float(self.lf_speed), float(self.precond_c)
        p.precond_gamma_hat = float(self.precond_gamma_hat)
        p.precond_kind = {"gram": B.PDHG_PRECOND_GRAM, "full": B.PDHG_PRECOND_FULL,
                          "gram_f32": B.PDHG_PRECOND_GRAM_F32}[self.precond_kind]
        return p

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.dtype is None else self.dtype

    @property
    def level_shape(self):
        """Shape of one time level: (nx,) for finite differences, (3, nx) for DG P2, (2, nx) for DG P1."""
        return {"dg_p2_llf": (3, self.nx), "dg_p1_upwind": (2, self.nx)}.get(self.space, (self.nx,))


@dataclass
class SolveResult:
    u: object
    phi: object
    status: int
    stats: dict
    history: Optional[object] = None


def _stream_ptr(device) -> C.c_void_p:
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class Solver:
    """One plan (pdhg_setup) for one problem on the current device."""

    def __init__(self, prob: Problem):
        import torch
        self.prob = prob
        self.lib = B.lib()
        self._h = C.c_void_p()
        self.device = torch.device("cuda", torch.cuda.current_device())
        rc = self.lib.pdhg_setup(C.byref(prob.to_c()), C.byref(self._h))
        if rc != B.PDHG_OK:
            raise PdhgError(f"pdhg_setup failed: {self._status(rc)}")

    # ----------------------------------------------------------------- helpers
    def _status(self, rc: int) -> str:
        s = self.lib.pdhg_status_string(rc).decode()
        if rc == B.PDHG_EHIP and self._h:
            s += ": " + self.lib.pdhg_last_error(self._h).decode()
        return f"{s} ({rc})"

    def _check(self, t, shape, name):
        import torch
        if t.device.type != "cuda" or t.dtype != self.prob.torch_dtype or not t.is_contiguous():
            raise PdhgError(f"{name}: need a contiguous {self.prob.torch_dtype} CUDA tensor")
        if tuple(t.shape) != tuple(shape):
            raise PdhgError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")
        return t

    def _empty(self, *shape):
        import torch
        return torch.empty(shape, dtype=self.prob.torch_dtype, device=self.device)

    @property
    def workspace_bytes(self) -> int:
        return int(self.lib.pdhg_workspace_bytes(self._h))

    # ----------------------------------------------------------------- API
    def solve(self, u0, tau_u: float = 0.0, tau_phi: float = 0.0, eps: float = 1e-8, max_iter: int = 10000,
              check_every: int = 64, u=None, phi=None, warm_start: bool = False, workspace=None,
              history: bool = False, diverge_factor: float = 0.0, variant: int = 0,
              backoff: int = 0, eps_rel: float = 0.0, stall_iters: int = 0, init_multiplier: bool = False,
              tau_u0: float = 0.0, tau_lam: float = 0.0) -> SolveResult:
        import torch
        nt, lv = self.prob.nt, self.prob.level_shape
        self._check(u0, lv, "u0")
        u = self._empty(nt + 1, *lv) if u is None else self._check(u, (nt + 1,) + lv, "u")
        phi = self._empty(nt, *lv) if phi is None else self._check(phi, (nt,) + lv, "phi")
        hist = torch.full((max_iter + 2, 2), float("nan"), dtype=torch.float64, device=self.device) \
            if history else None
        p = B.pdhg_params()
        p.tau_u, p.tau_phi, p.eps = float(tau_u), float(tau_phi), float(eps)
        p.max_iter, p.check_every, p.warm_start = int(max_iter), int(check_every), int(bool(warm_start))
        p.diverge_factor, p.variant, p.backoff = float(diverge_factor), int(variant), int(backoff)
        p.eps_rel, p.stall_iters = float(eps_rel), int(stall_iters)
        p.init_multiplier, p.tau_u0, p.tau_lam = int(bool(init_multiplier)), float(tau_u0), float(tau_lam)
        p.history = hist.data_ptr() if hist is not None else None
        st = B.pdhg_stats()
        rc = self.lib.pdhg_solve(self._h, _ptr(u0), _ptr(u), _ptr(phi), _ptr(workspace), C.byref(p),
                                 C.byref(st), _stream_ptr(self.device))
        if rc < 0:
            raise PdhgError(f"pdhg_solve failed: {self._status(rc)}")
        stats = {k: getattr(st, k) for k, _ in B.pdhg_stats._fields_}
        if hist is not None:
            hist = hist[: stats["iters"] + 1]
        return SolveResult(u, phi, rc, stats, hist)

    def solve_refined(self, u0, nt_start: int = 1, coarse_max_iter: int = 100000, coarse_eps: float = 0.0,
                      tau_u: float = 0.0, tau_phi: float = 0.0, eps: float = 1e-8, max_iter: int = 10000,
                      check_every: int = 64, u=None, phi=None, workspace=None, diverge_factor: float = 0.0) -> SolveResult:
        """Algorithm 2: Algorithm 1 on nt_start, 2 nt_start, ..., nt levels, each warm-started from the
        previous level interpolated in time.  stats["level_iters"] lists n* per level."""
        nt, lv = self.prob.nt, self.prob.level_shape
        self._check(u0, lv, "u0")
        u = self._empty(nt + 1, *lv) if u is None else self._check(u, (nt + 1,) + lv, "u")
        phi = self._empty(nt, *lv) if phi is None else self._check(phi, (nt,) + lv, "phi")
        p = B.pdhg_params()
        p.tau_u, p.tau_phi, p.eps = float(tau_u), float(tau_phi), float(eps)
        p.max_iter, p.check_every, p.warm_start = int(max_iter), int(check_every), 0
        p.diverge_factor, p.variant, p.history = float(diverge_factor), 0, None
        r = B.pdhg_refine_params()
        r.nt_start, r.coarse_max_iter, r.coarse_eps = int(nt_start), int(coarse_max_iter), float(coarse_eps)
        nlev = 1
        while (int(nt_start) << (nlev - 1)) < nt:
            nlev += 1
        li = (C.c_int64 * nlev)()
        st = B.pdhg_stats()
        rc = self.lib.pdhg_solve_refined(self._h, _ptr(u0), _ptr(u), _ptr(phi), _ptr(workspace), C.byref(p),
                                         C.byref(r), C.byref(st), li, _stream_ptr(self.device))
        if rc < 0:
            raise PdhgError(f"pdhg_solve_refined failed: {self._status(rc)}")
        stats = {k: getattr(st, k) for k, _ in B.pdhg_stats._fields_}
        stats["level_iters"] = list(li)
        return SolveResult(u, phi, rc, stats)

    def solve_onestep(self, u0, tau_u: float = 0.0, tau_phi: float = 0.0, eps: float = 1e-8,
                      max_iter: int = 10000, u=None, phi=None, diverge_factor: float = 0.0) -> SolveResult:
        """Algorithm 3: Algorithm 1 on one implicit step at a time (eps and max_iter per step, residuals in
        the norm of the time slice).  stats["step_iters"] lists n* per step, stats["step_res"] the final
        (Rp, Rd) per step."""
        nt, lv = self.prob.nt, self.prob.level_shape
        self._check(u0, lv, "u0")
        u = self._empty(nt + 1, *lv) if u is None else self._check(u, (nt + 1,) + lv, "u")
        phi = self._empty(nt, *lv) if phi is None else self._check(phi, (nt,) + lv, "phi")
        p = B.pdhg_params()
        p.tau_u, p.tau_phi, p.eps = float(tau_u), float(tau_phi), float(eps)
        p.max_iter, p.check_every, p.warm_start = int(max_iter), 1, 0
        p.diverge_factor, p.variant, p.history = float(diverge_factor), 0, None
        its = (C.c_int64 * nt)()
        res = (C.c_double * (2 * nt))()
        st = B.pdhg_stats()
        rc = self.lib.pdhg_solve_onestep(self._h, _ptr(u0), _ptr(u), _ptr(phi), C.byref(p), C.byref(st), its, res,
                                         _stream_ptr(self.device))
        if rc < 0:
            raise PdhgError(f"pdhg_solve_onestep failed: {self._status(rc)}")
        stats = {k: getattr(st, k) for k, _ in B.pdhg_stats._fields_}
        stats["step_iters"] = list(its)
        stats["step_res"] = [(res[2 * i], res[2 * i + 1]) for i in range(nt)]
        return SolveResult(u, phi, rc, stats)

    def residual(self, u, phi=None, want_fields: bool = True):
        """(A(u), J(u)^T phi, [||A(u)||, ||J(u)^T phi||])."""
        nt, lv = self.prob.nt, self.prob.level_shape
        self._check(u, (nt + 1,) + lv, "u")
        if phi is not None:
            self._check(phi, (nt,) + lv, "phi")
        au = self._empty(nt, *lv) if want_fields else None
        jt = self._empty(nt, *lv) if (want_fields and phi is not None) else None
        res = (C.c_double * 2)()
        rc = self.lib.pdhg_residual(self._h, _ptr(u), _ptr(phi), _ptr(au), _ptr(jt), res,
                                    _stream_ptr(self.device))
        if rc != B.PDHG_OK:
            raise PdhgError(f"pdhg_residual failed: {self._status(rc)}")
        return au, jt, (res[0], res[1])

    def residual_static(self, u, phi=None, Au=None, JTphi=None):
        """pdhg_residual_static: the residual without any allocation inside the library (the caller
        passes the outputs Au, JTphi or None for either)."""
        nt, lv = self.prob.nt, self.prob.level_shape
        self._check(u, (nt + 1,) + lv, "u")
        for t, name in ((phi, "phi"), (Au, "Au"), (JTphi, "JTphi")):
            if t is not None:
                self._check(t, (nt,) + lv, name)
        res = (C.c_double * 2)()
        rc = self.lib.pdhg_residual_static(self._h, _ptr(u), _ptr(phi), _ptr(Au), _ptr(JTphi), res,
                                           _stream_ptr(self.device))
        if rc != B.PDHG_OK:
            raise PdhgError(f"pdhg_residual_static failed: {self._status(rc)}")
        return Au, JTphi, (res[0], res[1])

    def precond(self, r, out=None):
        """s = K_d^{-1} r."""
        nt, lv = self.prob.nt, self.prob.level_shape
        self._check(r, (nt,) + lv, "r")
        s = self._empty(nt, *lv) if out is None else self._check(out, (nt,) + lv, "out")
        rc = self.lib.pdhg_precond(self._h, _ptr(r), _ptr(s), _stream_ptr(self.device))
        if rc != B.PDHG_OK:
            raise PdhgError(f"pdhg_precond failed: {self._status(rc)}")
        return s

    def apply_jt(self, u, phi):
        """J(u)^T phi, rows indexed by unknown level m-1."""
        nt, lv = self.prob.nt, self.prob.level_shape
        self._check(u, (nt + 1,) + lv, "u")
        self._check(phi, (nt,) + lv, "phi")
        out = self._empty(nt, *lv)
        rc = self.lib.pdhg_adjoint(self._h, B.PDHG_ADJ_APPLY, _ptr(u), _ptr(phi), _ptr(out), None, None,
                                   _stream_ptr(self.device))
        if rc != B.PDHG_OK:
            raise PdhgError(f"pdhg_adjoint failed: {self._status(rc)}")
        return out

    def adjoint_solve(self, u, g, want_mu: bool = False):
        """dL/du0 from dL/du (all levels) through the implicit scheme at its solution u."""
        nt, lv = self.prob.nt, self.prob.level_shape
        self._check(u, (nt + 1,) + lv, "u")
        self._check(g, (nt + 1,) + lv, "g")
        out = self._empty(*lv)
        mu = self._empty(nt, *lv) if want_mu else None
        rc = self.lib.pdhg_adjoint(self._h, B.PDHG_ADJ_SOLVE, _ptr(u), _ptr(g), _ptr(out), _ptr(mu), None,
                                   _stream_ptr(self.device))
        if rc != B.PDHG_OK:
            raise PdhgError(f"pdhg_adjoint failed: {self._status(rc)}")
        return (out, mu) if want_mu else out

    def time_kernel(self, kernel: int, reps: int = 20) -> float:
        ms = C.c_double()
        rc = self.lib.pdhg_time_kernel(self._h, int(kernel), int(reps), C.byref(ms), _stream_ptr(self.device))
        if rc != B.PDHG_OK:
            raise PdhgError(f"pdhg_time_kernel failed: {self._status(rc)}")
        return ms.value

    def close(self):
        if self._h:
            self.lib.pdhg_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class BatchResult:
    u: object                       # packed [sum (nt_i+1) nx_i]
    phi: object                     # packed [sum nt_i nx_i]
    status: int                     # worst over the batch (0 all converged)
    stats: list                     # one dict per problem
    views_u: list = field(default_factory=list)     # [nt_i+1, nx_i] views into u
    views_phi: list = field(default_factory=list)   # [nt_i, nx_i] views into phi


class BatchSolver:
    """One plan (pdhg_batch_setup) for a batch of independent problems of one dtype."""

    def __init__(self, probs):
        import torch
        self.probs = list(probs)
        if not self.probs:
            raise PdhgError("empty batch")
        self.dtype = self.probs[0].torch_dtype
        if any(p.torch_dtype != self.dtype for p in self.probs):
            raise PdhgError("all problems of a batch must have the same dtype")
        self.lib = B.lib()
        self._h = C.c_void_p()
        self.device = torch.device("cuda", torch.cuda.current_device())
        arr = (B.pdhg_problem * len(self.probs))(*[p.to_c() for p in self.probs])
        rc = self.lib.pdhg_batch_setup(arr, len(self.probs), C.byref(self._h))
        if rc != B.PDHG_OK:
            raise PdhgError(f"pdhg_batch_setup failed: {self.lib.pdhg_status_string(rc).decode()} ({rc})")
        n0, nu, nf, ws = C.c_int64(), C.c_int64(), C.c_int64(), C.c_size_t()
        self.lib.pdhg_batch_sizes(self._h, C.byref(n0), C.byref(nu), C.byref(nf), C.byref(ws))
        self.u0_elems, self.u_elems, self.phi_elems, self.workspace_bytes = n0.value, nu.value, nf.value, ws.value
        self.offsets = []
        for i in range(len(self.probs)):
            a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
            self.lib.pdhg_batch_offsets(self._h, i, C.byref(a), C.byref(b), C.byref(c))
            self.offsets.append((a.value, b.value, c.value))
        self._ws = None

    def _status(self, rc: int) -> str:
        s = self.lib.pdhg_status_string(rc).decode()
        if rc == B.PDHG_EHIP and self._h:
            s += ": " + self.lib.pdhg_batch_last_error(self._h).decode()
        return f"{s} ({rc})"

    def pack_u0(self, u0_list):
        """Concatenate per-problem initial data into the packed u0 layout."""
        import torch
        return torch.cat([torch.as_tensor(x, dtype=self.dtype, device=self.device).reshape(-1) for x in u0_list])

    def _views(self, u, phi):
        vu, vp = [], []
        for p, (_, ou, of) in zip(self.probs, self.offsets):
            vu.append(u[ou: ou + (p.nt + 1) * p.nx].view(p.nt + 1, p.nx))
            vp.append(phi[of: of + p.nt * p.nx].view(p.nt, p.nx))
        return vu, vp

    def _params(self, tau_u, tau_phi, eps, max_iter, check_every, warm_start, diverge_factor):
        n = len(self.probs)
        self._tu = (C.c_double * n)(*([0.0] * n if tau_u is None else [float(x) for x in tau_u]))
        self._tp = (C.c_double * n)(*([0.0] * n if tau_phi is None else [float(x) for x in tau_phi]))
        p = B.pdhg_batch_params()
        p.tau_u = C.cast(self._tu, C.c_void_p)
        p.tau_phi = C.cast(self._tp, C.c_void_p)
        p.eps, p.max_iter, p.check_every = float(eps), int(max_iter), int(check_every)
        p.warm_start, p.diverge_factor = int(bool(warm_start)), float(diverge_factor)
        return p

    def _buffers(self, u, phi, workspace):
        import torch
        if u is None:
            u = torch.empty(self.u_elems, dtype=self.dtype, device=self.device)
        if phi is None:
            phi = torch.empty(self.phi_elems, dtype=self.dtype, device=self.device)
        for t, n, name in ((u, self.u_elems, "u"), (phi, self.phi_elems, "phi")):
            if t.dtype != self.dtype or t.device.type != "cuda" or not t.is_contiguous() or t.numel() != n:
                raise PdhgError(f"{name}: need a contiguous CUDA tensor of {n} {self.dtype} elements")
        if workspace is None:
            if self._ws is None:
                self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            workspace = self._ws
        return u, phi, workspace

    def solve(self, u0, tau_u=None, tau_phi=None, eps: float = 1e-8, max_iter: int = 10000, check_every: int = 64,
              u=None, phi=None, warm_start: bool = False, workspace=None, diverge_factor: float = 0.0) -> BatchResult:
        if u0.dtype != self.dtype or u0.numel() != self.u0_elems or not u0.is_contiguous():
            raise PdhgError(f"u0: need a contiguous tensor of {self.u0_elems} {self.dtype} elements")
        u, phi, workspace = self._buffers(u, phi, workspace)
        p = self._params(tau_u, tau_phi, eps, max_iter, check_every, warm_start, diverge_factor)
        st = (B.pdhg_stats * len(self.probs))()
        rc = self.lib.pdhg_batch_solve(self._h, _ptr(u0), _ptr(u), _ptr(phi), _ptr(workspace), C.byref(p), st,
                                       _stream_ptr(self.device))
        if rc < 0:
            raise PdhgError(f"pdhg_batch_solve failed: {self._status(rc)}")
        stats = [{k: getattr(s, k) for k, _ in B.pdhg_stats._fields_} for s in st]
        vu, vp = self._views(u, phi)
        return BatchResult(u, phi, rc, stats, vu, vp)

    def solve_onestep(self, u0, tau_u=None, tau_phi=None, eps: float = 1e-8, max_iter: int = 10000, u=None,
                      phi=None, diverge_factor: float = 0.0, want_steps: bool = False) -> BatchResult:
        """Algorithm 3 for every problem (one workgroup per problem, one launch).  With want_steps,
        stats[i]["step_iters"] lists problem i's n* per step."""
        import torch
        if u0.dtype != self.dtype or u0.numel() != self.u0_elems or not u0.is_contiguous():
            raise PdhgError(f"u0: need a contiguous tensor of {self.u0_elems} {self.dtype} elements")
        if u is None:
            u = torch.empty(self.u_elems, dtype=self.dtype, device=self.device)
        if phi is None:
            phi = torch.empty(self.phi_elems, dtype=self.dtype, device=self.device)
        p = self._params(tau_u, tau_phi, eps, max_iter, 0, False, diverge_factor)
        st = (B.pdhg_stats * len(self.probs))()
        nst = sum(q.nt for q in self.probs)
        its = (C.c_int64 * nst)() if want_steps else None
        rc = self.lib.pdhg_batch_solve_onestep(self._h, _ptr(u0), _ptr(u), _ptr(phi), C.byref(p), st, its,
                                               _stream_ptr(self.device))
        if rc < 0:
            raise PdhgError(f"pdhg_batch_solve_onestep failed: {self._status(rc)}")
        stats = [{k: getattr(s, k) for k, _ in B.pdhg_stats._fields_} for s in st]
        if want_steps:
            o = 0
            for q, d in zip(self.probs, stats):
                d["step_iters"] = list(its[o:o + q.nt])
                o += q.nt
        vu, vp = self._views(u, phi)
        return BatchResult(u, phi, rc, stats, vu, vp)

    def tune(self, u0, tau_u=None, tau_phi=None, u=None, phi=None, workspace=None):
        """Autotune the persistent grid sizes of the three passes; returns them."""
        u, phi, workspace = self._buffers(u, phi, workspace)
        p = self._params(tau_u, tau_phi, 0.0, 1, 64, False, 0.0)
        grids = (C.c_int32 * 3)()
        rc = self.lib.pdhg_batch_tune(self._h, _ptr(u0), _ptr(u), _ptr(phi), _ptr(workspace), C.byref(p), grids,
                                      _stream_ptr(self.device))
        if rc != B.PDHG_OK:
            raise PdhgError(f"pdhg_batch_tune failed: {self._status(rc)}")
        return list(grids)

    def time_kernel(self, kernel: int, reps: int = 20) -> float:
        """Milliseconds per launch of batched pass `kernel` (0 A, 1 B, 2 C) on the last solve's buffers."""
        ms = C.c_double()
        rc = self.lib.pdhg_batch_time_kernel(self._h, int(kernel), int(reps), C.byref(ms), _stream_ptr(self.device))
        if rc != B.PDHG_OK:
            raise PdhgError(f"pdhg_batch_time_kernel failed: {self._status(rc)}")
        return ms.value

    def close(self):
        if self._h:
            self.lib.pdhg_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def differentiable_solve(u0, solver, allow_unconverged: bool = False, **solve_kwargs):
    """u (all levels) as a differentiable function of u0 (implicit adjoint backward).  Raises when the
    solve ends at max_iter, unless allow_unconverged (then it warns)."""
    from .autograd import solve
    return solve(u0, solver, allow_unconverged=allow_unconverged, **solve_kwargs)
