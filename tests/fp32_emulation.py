"""Single-precision emulations of Algorithm 1 beside the FP64 oracle (test infrastructure; no GPU).

Element-wise parity of an FP32 iterate with the FP64 oracle cannot hold at the
flat FP32 bar on fine grids: the rounding of the stored dual (|phibar| up to
2 max|phi|) is multiplied in the primal step by tau times the row sum of
|J^T|, about 4/h_t plus the flux part, and the float rounding of the
preconditioned residual s is differenced in time there as well.  Where the flat
bar does not hold, the GPU's FP32 iterates are held to twice the error of these
emulations, which round where the GPU path rounds:

* ``run_fp32``: the FP32 problem.  u, phi, phibar, the residual rows and the
  spectrum are float32; the dual step and extrapolation are float32
  arithmetic (phi_new = phi + tau s, phibar = phi_new + tau s); J(u)^T phibar
  and A(u) are the oracle's operators evaluated on the float values and
  rounded once.  For finite differences the preconditioner is emulated as the
  GPU runs it: float FFTs along x, and the banded Cholesky recurrences along t
  in float, cut into per-lane segments whose affine maps are composed across
  the lanes (16 lanes per column up to N_t = 256, 32 up to 512, 64 beyond);
  for DG likewise: float FFTs over the cells, the per-mode eigenbasis rotation
  in float and one float segmented recurrence per eigen-branch.
* ``segmented_solve``: that segmented recurrence on its own (any type), also
  used to show where the single-precision spectral pass of FP64 problems loses
  accuracy.

The operators themselves (A, J^T, K_d) are the oracle's: this module adds
only rounding, never arithmetic of the method.
"""
from __future__ import annotations

import numpy as np

from oracle import pdhg as opdhg
from oracle import precond as opre

F32 = np.float32


def cholesky_bands(prob):
    """Per mode k = 0..N_x/2: (1/L_ll, L_{l,l-1}, L_{l,l-2}) of the Cholesky factor of
    B_t B_t^T + s_k I, as arrays (N_t, M) and (N_t + 2, M) (zero outside the matrix)."""
    kt = opre.time_gram(prob)
    sh = opre.mode_shifts(prob)
    nt, m = prob.nt, prob.nx // 2 + 1
    invd = np.zeros((nt, m))
    e1 = np.zeros((nt + 2, m))
    e2 = np.zeros((nt + 2, m))
    for k in range(m):
        L = np.linalg.cholesky(kt + sh[k] * np.eye(nt))
        invd[:, k] = 1.0 / np.diag(L)
        e1[1:nt, k] = np.diagonal(L, -1)
        if nt > 2:
            e2[2:nt, k] = np.diagonal(L, -2)
    return invd, e1, e2


def segmented_solve(invd, e1, e2, b, nlanes, dt):
    """L L^T y = b along axis 0 for every column of b, in arithmetic type dt: the time axis is cut
    into nlanes segments; each segment's affine map (particular solution from a zero state and the
    responses to the two incoming values) is formed, the maps are composed from segment to
    segment, and each segment is re-run from its incoming state.  Forward, then backward."""
    invd, e1, e2 = invd.astype(dt), e1.astype(dt), e2.astype(dt)
    b = b.astype(dt)
    nt = b.shape[0]
    lpl = -(-nt // nlanes)

    def sweep(rhs, fwd):
        out = np.zeros_like(rhs)
        segs = [list(range(j * lpl, min(nt, (j + 1) * lpl))) for j in range(-(-nt // lpl))]
        if not fwd:
            segs = [s[::-1] for s in segs[::-1]]

        def coef(l):
            return (e1[l], e2[l]) if fwd else (e1[l + 1], e2[l + 2])

        s2 = np.zeros(rhs.shape[1:], dt)
        s1 = np.zeros(rhs.shape[1:], dt)
        for seg in segs:
            p2, p1 = np.zeros_like(s2), np.zeros_like(s2)
            a2, a1 = np.ones_like(s2), np.zeros_like(s2)
            b2, b1 = np.zeros_like(s2), np.ones_like(s2)
            for l in seg:
                c1, c2 = coef(l)
                pz = invd[l] * (rhs[l] - c1 * p1 - c2 * p2)
                az = invd[l] * (-(c1 * a1) - c2 * a2)
                bz = invd[l] * (-(c1 * b1) - c2 * b2)
                p2, p1, a2, a1, b2, b1 = p1, pz, a1, az, b1, bz
            zm2, zm1 = s2, s1
            for l in seg:
                c1, c2 = coef(l)
                zz = invd[l] * (rhs[l] - c1 * zm1 - c2 * zm2)
                out[l] = zz
                zm2, zm1 = zm1, zz
            s2, s1 = a2 * s2 + b2 * s1 + p2, a1 * s2 + b1 * s1 + p1
        return out

    return sweep(sweep(b, True), False)


def gpu_lanes_per_column(nt: int) -> int:
    return 16 if nt <= 256 else (32 if nt <= 512 else 64)


def kd_solve_fp32_fd(prob, bands, r32):
    """K_d^{-1} r as the FP32 finite-difference path computes it (float FFTs, float segmented
    recurrences, float spectrum)."""
    nx = prob.nx
    rh = np.fft.rfft(r32.astype(F32), axis=1).astype(np.complex64)
    lanes = gpu_lanes_per_column(prob.nt)
    re = segmented_solve(*bands, rh.real, lanes, F32)
    im = segmented_solve(*bands, rh.imag, lanes, F32)
    sh = (re + 1j * im).astype(np.complex64)
    return np.fft.irfft(sh, n=nx, axis=1).astype(F32)


def kd_solve_fp32_dg(prob, r32):
    """K_d^{-1} r for the DG planes as the FP32 DG path computes it: float FFTs over the cells, the
    per-mode eigenbasis rotation of c^2 G G^* in float, one float segmented recurrence per
    eigen-branch (64 lanes per column), and the rotation back in float."""
    from oracle import dg, dg1
    mod = dg if prob.space == "dg_p2_llf" else dg1
    nt, npl, nx = r32.shape
    lam, Q = mod.mode_eig(prob)
    m_half = nx // 2 + 1
    R = np.fft.fft(r32.astype(F32), axis=-1).astype(np.complex64)[:, :, :m_half]    # (nt, npl, M)
    Qc = Q[:m_half].astype(np.complex64)                                          # (M, npl, npl)
    W = np.einsum("lpm,mpb->lbm", R, np.conj(Qc)).astype(np.complex64)            # rows: Q^* rhat_l
    kt = opre.time_gram(prob)
    Z = np.empty_like(W)
    for br in range(npl):
        invd = np.zeros((nt, m_half))
        e1 = np.zeros((nt + 2, m_half))
        e2 = np.zeros((nt + 2, m_half))
        for m in range(m_half):
            L = np.linalg.cholesky(kt + lam[m, br] * np.eye(nt))
            invd[:, m] = 1.0 / np.diag(L)
            e1[1:nt, m] = np.diagonal(L, -1)
            if nt > 2:
                e2[2:nt, m] = np.diagonal(L, -2)
        re = segmented_solve(invd, e1, e2, W[:, br, :].real, 64, F32)
        im = segmented_solve(invd, e1, e2, W[:, br, :].imag, 64, F32)
        Z[:, br, :] = (re + 1j * im).astype(np.complex64)
    S = np.einsum("lbm,mpb->lpm", Z, Qc).astype(np.complex64)                     # rows: Q z_l
    full = np.zeros((nt, npl, nx), dtype=np.complex64)
    full[:, :, :m_half] = S
    full[:, :, m_half:] = np.conj(S[:, :, 1:nx - m_half + 1][:, :, ::-1])
    return np.real(np.fft.ifft(full, axis=-1)).astype(F32)


def run_fp32(prob, u0, tau, n_iter):
    """n_iter iterations of Algorithm 1 (u^0 fixed, standard signs) with FP32 storage; returns (u, phi)."""
    residual, _, _ = opdhg._ops(prob)
    fd = prob.space.startswith("fd")
    bands = cholesky_bands(prob) if fd and prob.precond_kind == "gram" else None
    u0 = np.asarray(u0, dtype=np.float64)
    u = np.broadcast_to(u0.astype(F32), (prob.nt + 1,) + u0.shape).copy()
    phi = np.zeros((prob.nt,) + u0.shape, F32)
    phibar = phi.copy()
    t = F32(tau)
    for _ in range(n_iter):
        jt = opdhg.jt_operator(prob, u.astype(np.float64))
        u[1:] = (u[1:].astype(np.float64) - tau * jt(phibar.astype(np.float64))).astype(F32)
        r = residual(prob, u.astype(np.float64)).astype(F32)
        if bands is not None:
            s = kd_solve_fp32_fd(prob, bands, r)
        elif prob.space in ("dg_p2_llf", "dg_p1_upwind"):
            s = kd_solve_fp32_dg(prob, r)
        else:
            s = opdhg.kd_solve_any(prob, r.astype(np.float64)).astype(F32)
        ts = t * s
        phin = phi + ts
        phibar = phin + ts
        phi = phin
    return u.astype(np.float64), phi.astype(np.float64)


def rel_err(a, ref):
    return float(np.max(np.abs(np.asarray(a) - ref)) / max(1.0, float(np.max(np.abs(ref)))))


def fp32_bar(prob, u0, tau, n_iter, ref_u, ref_phi, flat=1e-5):
    """(bar for u, bar for phi): the flat FP32 bar, or twice the emulated FP32 error where that is larger."""
    eu, ep = run_fp32(prob, u0, tau, n_iter)
    return max(flat, 2.0 * rel_err(eu, ref_u)), max(flat, 2.0 * rel_err(ep, ref_phi))
