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
  from N_t = 4097 on (N_x >= 16) the column solve runs in chunks of 256
  levels: the slowly decaying low modes (``gpu_fp64_modes``) with FP64
  recurrences rounded to float once, the others with float recurrences from
  chunk states carried in FP64 (``chunked_solve``);
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

from oracle import fd as ofd
from oracle import pdhg as opdhg
from oracle import precond as opre

F32 = np.float32


def cholesky_bands(prob):
    """Per mode k = 0..N_x/2: (1/L_ll, L_{l,l-1}, L_{l,l-2}) of the Cholesky factor of
    B_t B_t^T + s_k I, as arrays (N_t, M) and (N_t + 2, M) (zero outside the matrix); the factor
    of the banded matrix in banded storage (LAPACK pbtrf)."""
    import scipy.linalg as sla
    kt = opre.time_gram(prob)
    sh = opre.mode_shifts(prob)
    nt, m = prob.nt, prob.nx // 2 + 1
    band = np.zeros((3, nt))   # lower banded storage: band[d, l] = K[l + d, l]
    for d in range(3):
        if d < nt:
            band[d, :nt - d] = np.diagonal(kt, -d)
    invd = np.zeros((nt, m))
    e1 = np.zeros((nt + 2, m))
    e2 = np.zeros((nt + 2, m))
    for k in range(m):
        b = band.copy()
        b[0] += sh[k]
        lb = sla.cholesky_banded(b, lower=True)
        invd[:, k] = 1.0 / lb[0]
        e1[1:nt, k] = lb[1, :nt - 1]
        if nt > 2:
            e2[2:nt, k] = lb[2, :nt - 2]
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


CHUNK_LEVELS = 256


def gpu_chunked_columns(nt: int, nx: int) -> bool:
    """Whether the GPU's column solve runs in chunks."""
    return nt >= 4097 and nx >= 16


def gpu_fp64_modes(prob) -> int:
    """Modes 0 .. k-1 whose chunked column solve the GPU runs in FP64 for a float spectrum: those of
    the column blocks (8 modes each, block 0 with mode 0) before the first block whose lowest mode
    has s_k h_t^2 >= 1e-2 (the shift against (1/h_t)^2: slower decay along t below it)."""
    sh = opre.mode_shifts(prob)
    ht = prob.t_final / prob.nt
    for g in range(1, prob.nx // 16):
        if sh[8 * g] * ht * ht >= 1e-2:
            return 8 * g
    return prob.nx // 2 + 1


def chunked_solve(invd, e1, e2, b, dt):
    """L L^T y = b along axis 0 for every column of b as the GPU's chunked column solve computes it
    with recurrences in type dt: each chunk of CHUNK_LEVELS levels is solved from zero entering
    states (forward state leaving it P, backward state leaving it R); the states entering every
    chunk follow in FP64 from P, R and the chunk's maps (H, G: homogeneous responses over the
    chunk; K: its backward solve of the forward homogeneous responses); each chunk is solved again
    from its entering states, rounded to dt.  Forward, then backward within a chunk."""
    nt, m = b.shape
    nc = -(-nt // CHUNK_LEVELS)
    f64 = np.float64
    iv, f1, f2 = invd.astype(dt), e1.astype(dt), e2.astype(dt)
    bb = b.astype(dt)

    def solve(c, x2, x1, w2, w1):
        s, e = c * CHUNK_LEVELS, min(nt, (c + 1) * CHUNK_LEVELS)
        z = np.zeros((e - s, m), dt)
        zm2, zm1 = x2.astype(dt), x1.astype(dt)
        for l in range(s, e):
            zz = iv[l] * (bb[l] - f1[l] * zm1 - f2[l] * zm2)
            z[l - s] = zz
            zm2, zm1 = zm1, zz
        p = (zm2, zm1)
        ym2, ym1 = w2.astype(dt), w1.astype(dt)
        for l in range(e - 1, s - 1, -1):
            yy = iv[l] * (z[l - s] - f1[l + 1] * ym1 - f2[l + 2] * ym2)
            z[l - s] = yy
            ym2, ym1 = ym1, yy
        return z, p, (ym2, ym1)

    zero = np.zeros(m, f64)
    one = np.ones(m, f64)
    rec = [solve(c, zero, zero, zero, zero)[1:] for c in range(nc)]
    i8, g1, g2 = invd.astype(f64), e1.astype(f64), e2.astype(f64)
    maps = []
    for c in range(nc):
        s, e = c * CHUNK_LEVELS, min(nt, (c + 1) * CHUNK_LEVELS)
        a2, a1, b2, b1, u2, u1, v2, v1 = one, zero, zero, one, zero, zero, zero, zero
        k = [zero, zero, zero, zero]
        for l in range(s, e):
            az = i8[l] * (-(g1[l] * a1) - g2[l] * a2)
            bz = i8[l] * (-(g1[l] * b1) - g2[l] * b2)
            uz = i8[l] * ((one if l == s else zero) - g1[l] * u1 - g2[l] * u2)
            vz = i8[l] * ((one if l == s + 1 else zero) - g1[l] * v1 - g2[l] * v2)
            a2, a1, b2, b1, u2, u1, v2, v1 = a1, az, b1, bz, u1, uz, v1, vz
            k = [k[0] + vz * az, k[1] + vz * bz, k[2] + uz * az, k[3] + uz * bz]
        hmap = (a2, b2, a1, b1)
        a2, a1, b2, b1 = one, zero, zero, one
        for l in range(e - 1, s - 1, -1):
            az = i8[l] * (-(g1[l + 1] * a1) - g2[l + 2] * a2)
            bz = i8[l] * (-(g1[l + 1] * b1) - g2[l + 2] * b2)
            a2, a1, b2, b1 = a1, az, b1, bz
        maps.append((hmap, (a2, b2, a1, b1), k))
    t, h = [None] * nc, [None] * nc
    t2 = t1 = zero
    for c in range(nc):
        t[c] = (t2, t1)
        hm, p = maps[c][0], rec[c][0]
        t2, t1 = (hm[0] * t2 + hm[1] * t1 + p[0].astype(f64), hm[2] * t2 + hm[3] * t1 + p[1].astype(f64))
    h2 = h1 = zero
    for c in range(nc - 1, -1, -1):
        h[c] = (h2, h1)
        gm, km, r = maps[c][1], maps[c][2], rec[c][1]
        u2, u1 = t[c]
        h2, h1 = (gm[0] * h2 + gm[1] * h1 + km[0] * u2 + km[1] * u1 + r[0].astype(f64),
                  gm[2] * h2 + gm[3] * h1 + km[2] * u2 + km[3] * u1 + r[1].astype(f64))
    return np.concatenate([solve(c, *t[c], *h[c])[0] for c in range(nc)])


def constant_chunk_solve(invd, e1, e2, b, x, w, lpl=8, lanes=32):
    """One chunk of lanes * lpl levels of L L^T y = b, every level on the same factor row
    (invd, e1, e2: scalars), entered with forward state x = (z_{-2}, z_{-1}) and backward state
    w = (y_{n+1}, y_n), as the GPU's constant-tile kernels compute it (FP64): each lane's
    particular part P from zero; M, the homogeneous map of lpl levels, and M^2, M^4, M^8; the
    entering state folded into the first lane (P += M x); an inclusive scan within each row of 16
    lanes (P_q += M^d P_{q-d} at d = 1, 2, 4, 8, lanes without a lane d before them unchanged);
    the second row adds the scan of a vector started from M S in its first lane (S: the first
    row's total); the state entering a lane is the inclusive P of the lane before it; every lane
    solved again from it.  Backward mirrors it from the last lane.  b: (lanes * lpl, m)."""
    n, m = b.shape
    assert n == lanes * lpl and lanes == 32

    def seg(z, s2, s1, fwd):   # lpl levels of one lane from state (s2, s1); returns values and state
        out = np.zeros_like(z)
        order = range(lpl) if fwd else range(lpl - 1, -1, -1)
        for i in order:
            v = invd * (z[i] - e1 * s1 - e2 * s2)
            out[i] = v
            s2, s1 = s1, v
        return out, s2, s1

    # M: states (a2, a1) and (b2, b1) after lpl homogeneous levels from (1, 0) and (0, 1)
    _, a2, a1 = seg(np.zeros((lpl, 1)), np.ones(1), np.zeros(1), True)
    _, b2, b1 = seg(np.zeros((lpl, 1)), np.zeros(1), np.ones(1), True)
    m1 = np.array([[a2[0], b2[0]], [a1[0], b1[0]]])
    pw = [m1]
    for _ in range(3):
        pw.append(pw[-1] @ pw[-1])

    def row_scan(v, fwd):   # v: (lanes, 2, m), in place per row of 16 lanes
        for s_, mp in enumerate(pw):
            d = 1 << s_
            new = v.copy()
            for q in range(lanes):
                r = q % 16
                src = q - d if fwd else q + d
                if (fwd and r >= d) or (not fwd and r + d <= 15):
                    new[q] = v[q] + np.einsum("ij,jm->im", mp, v[src])
            v[:] = new

    def scan(blocks, x2, x1, fwd):
        P = np.zeros((lanes, 2, m))
        for q in range(lanes):
            _, p2, p1 = seg(blocks[q], np.zeros(m), np.zeros(m), fwd)
            P[q] = (p2, p1)
        first = 0 if fwd else lanes - 1
        P[first] += np.einsum("ij,jm->im", m1, np.stack([x2, x1]))
        row_scan(P, fwd)
        S = P[15] if fwd else P[16]
        D = np.zeros_like(P)
        D[16 if fwd else 15] = np.einsum("ij,jm->im", m1, S)
        row_scan(D, fwd)
        P += D
        ent = np.zeros_like(P)
        for q in range(lanes):
            if q == first:
                ent[q] = (x2, x1)
            else:
                ent[q] = P[q - 1] if fwd else P[q + 1]
        return ent

    blocks = b.reshape(lanes, lpl, m).astype(np.float64)
    ent = scan(blocks, x[0], x[1], True)
    z = np.stack([seg(blocks[q], ent[q][0], ent[q][1], True)[0] for q in range(lanes)])
    ent = scan(z, w[0], w[1], False)
    y = np.stack([seg(z[q], ent[q][0], ent[q][1], False)[0] for q in range(lanes)])
    return y.reshape(n, m)


def kd_solve_fp32_fd(prob, bands, r32):
    """K_d^{-1} r as the FP32 finite-difference path computes it (float FFTs, float spectrum; float
    segmented recurrences, or the chunked solve on long time axes)."""
    nx = prob.nx
    rh = np.fft.rfft(r32.astype(F32), axis=1).astype(np.complex64)
    if gpu_chunked_columns(prob.nt, nx):
        k64 = gpu_fp64_modes(prob)
        lo = [x[:, :k64] for x in bands]
        hi = [x[:, k64:] for x in bands]
        re = np.concatenate([chunked_solve(*lo, rh.real[:, :k64], np.float64).astype(F32),
                             chunked_solve(*hi, rh.real[:, k64:], F32)], axis=1)
        im = np.concatenate([chunked_solve(*lo, rh.imag[:, :k64], np.float64).astype(F32),
                             chunked_solve(*hi, rh.imag[:, k64:], F32)], axis=1)
    else:
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


def run_float_spectrum(prob, u0, tau, n_iter, ft=F32):
    """Algorithm 1 (u^0 fixed) with the single-precision spectral pass of an FP64 problem emulated:
    the residual rows rounded to float and transformed in float, a float spectrum, the banded
    recurrences in FP64 on it, mode 0 of s kept in FP64 through the inverse transform; FP64
    elsewhere.  ft is the type of the float pass (np.float64 removes the rounding).  Returns
    (u, phi) after n_iter iterations."""
    cx = np.complex64 if ft == F32 else np.complex128
    invd, e1, e2 = cholesky_bands(prob)
    nx, nt = prob.nx, prob.nt
    cols = (np.repeat(invd, 2, axis=1), np.repeat(e1, 2, axis=1), np.repeat(e2, 2, axis=1))

    def kd(r):
        rh = np.fft.rfft(r.astype(ft), axis=1).astype(cx)
        b = np.empty((nt, 2 * rh.shape[1]))
        b[:, 0::2], b[:, 1::2] = rh.real, rh.imag
        y = segmented_solve(*cols, b, 1, np.float64)
        sh = y[:, 0::2] + 1j * y[:, 1::2]
        s0 = sh[:, 0].real.copy()
        sh[:, 0] = 0.0
        s = np.fft.irfft(sh.astype(cx), n=nx, axis=1).astype(np.float64)
        return s + s0[:, None] / nx

    u = np.broadcast_to(np.asarray(u0, dtype=np.float64), (nt + 1, nx)).copy()
    phi = np.zeros((nt, nx))
    phibar = phi.copy()
    for _ in range(n_iter):
        jt = ofd.jacobian(prob, u).T.tocsr()
        u[1:] -= tau * (jt @ phibar.ravel()).reshape(phibar.shape)
        sv = kd(ofd.residual(prob, u))
        phibar = phi + 2.0 * tau * sv
        phi = phi + tau * sv
    return u, phi


def float_spectrum_bar(prob, u0, tau, n_iter, ref_u, ref_phi, flat=1e-5):
    """(bar for u, bar for phi) of the single-precision spectral pass: the flat bar, or twice the
    emulated error where that is larger."""
    eu, ep = run_float_spectrum(prob, u0, tau, n_iter)
    return max(flat, 2.0 * rel_err(eu, ref_u)), max(flat, 2.0 * rel_err(ep, ref_phi))


def rel_err(a, ref):
    return float(np.max(np.abs(np.asarray(a) - ref)) / max(1.0, float(np.max(np.abs(ref)))))


def fp32_bar(prob, u0, tau, n_iter, ref_u, ref_phi, flat=1e-5):
    """(bar for u, bar for phi): the flat FP32 bar, or twice the emulated FP32 error where that is larger."""
    eu, ep = run_fp32(prob, u0, tau, n_iter)
    return max(flat, 2.0 * rel_err(eu, ref_u)), max(flat, 2.0 * rel_err(ep, ref_phi))
