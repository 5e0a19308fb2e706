"""Benchmark: space-time PDHG on the inviscid Burgers workload, one MI355X.

Workload (one "step" = one full solve of Algorithm 1 from the initial guess
u^l = u0, phi = 0 to residual 1e-8): u_t + (u^2/2)_x = 0 on [0,1) periodic,
N_x = 2048, N_t = 512, T = 0.5 (h_t = 2 h_x), BDF2 in time with a backward
Euler first row, global Lax-Friedrichs flux, seeded Fourier-sum u0 (seed 0),
FP64, step sizes sqrt(0.95/nu_max) from the library's power iteration.

Printed (one JSON line on stdout): DOF-iterations/s of the timed solves,
time to residual 1e-8, the dominant kernel's achieved bandwidth from HIP
event timing against the 8 TB/s HBM peak, and the FP64 CPU oracle timed on a
bounded sample of iterations of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --workload batch [--batch-iters N] [--ttr-problems M]
    python bench.py --workload dg [--dg-iters N] [--dtype f32|f64]
    python bench.py --workload adjoint [--dtype f32|f64]

The default run also measures the other workloads, under config.variants:
the DG P2 workload (4096 cells x 512 levels, FP32 to its rounding floor and
FP64 to 1e-8), the 256-problem batch (FP32 throughput batched against one solve
per problem; FP64 time to residual 1e-8 over all problems with Algorithms 1
and 3, batched against one solve per problem), the differentiable solve
(viscous Burgers, forward + adjoint, FP32 and FP64), the FP32 run of the
headline workload and single problems too large for the 256 MB MALL.  The
cpu_baseline leg then runs the FP64 oracle: its timing on all host cores and in
a one-thread process, and the Newton march / adjoint gradient of each workload,
against which the FP64 error of every GPU result is reported.

The single workload also reports the paper's three variants side by side
(Section 4, comparison of the variants): Algorithm 1, mesh refinement in time
(Algorithm 2, levels N_t = 1, 2, ..., 512) and the one-time-step solver
(Algorithm 3, step residual 1e-8 in the slice norm, so the space-time residual
is at most sqrt(T) 1e-8), each with its iterations, "world time" (iterations
in sequence) and work in units of N_x (sum over levels of iterations times
N_t + 1 levels; two levels per one-step iteration), and measured seconds.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PDHG space-time DOF-iterations/s; time to residual 1e-8; achieved HBM GB/s"
HBM_PEAK_GBS = 8000.0

NX, NT, T_FINAL, EPS, SEED = 2048, 512, 0.5, 1e-8, 0

# Algorithmic words moved per DOF by each kernel of one iteration (library kernel ids
# of pdhg_time_kernel).  Fused variant: A reads shat and phi, writes phi and phibar;
# B reads phibar and u, writes u and rhat (and reads phi where the dual residual is needed:
# near convergence and at the last iteration); C reads rhat and writes shat.
KERNELS_FUSED = {
    7: ("A: inverse FFT + dual step", 4),
    0: ("B: primal step + residual + forward FFT", 4),   # steady state: phi is read only near convergence
    1: ("C: column solve (banded Cholesky in t)", 2),
}
COPY_KERNEL = 8   # plain copy of N_t*N_x elements: one read and one write per element

# HBM traffic of the dominant kernel from hardware counters (rocprofv3 --pmc FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch, median over dispatches), each scaled by the ratio of known bytes to
# the same counter's reading for the plain copy kernel in the same run.  The readings are valid
# only for the kernel sources they were taken on (SHA-256 below); after any change to those
# sources the traffic field is reported as null until the counters are taken again.
# Summary and commands: profiles/primal_res_burgers_2048x512_f64_pmc.md.
COUNTER_SOURCES = ("paper_2207_07234_amd/csrc/pdhg_fused.hip", "paper_2207_07234_amd/csrc/pdhg_passes.hpp",
                   "paper_2207_07234_amd/csrc/pdhg_device.hpp")
COUNTERS = {
    # (dtype, variant, kernel id): per-dispatch KiB of the kernel and of the copy kernel
    ("f64", 2, 0): {"fetch_kib": 8781.5, "write_kib": 16388.0, "copy_fetch_kib": 4105.5, "copy_write_kib": 8192.0,
                    "sha": "5e55490639db92d7c989ef42b7a75e3dd394c85fad3d596113ed644de39e3dd2"},
}

KERNELS_UNFUSED = {
    1: ("column solve (banded Cholesky in t)", 2),
    2: ("inverse row FFT", 2),
    3: ("dual update", 4),
    4: ("primal update", 4),
    5: ("implicit residual", 2),
    6: ("forward row FFT", 2),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in COUNTER_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(dtype: str, variant: int, kid: int, copy_bytes: float):
    """HBM bytes per launch of kernel `kid` from the recorded counters, or None."""
    rec = COUNTERS.get((dtype, variant, kid))
    if rec is None or rec["sha"] != sources_sha():
        return None
    fetch = rec["fetch_kib"] * (copy_bytes / 2) / rec["copy_fetch_kib"]
    write = rec["write_kib"] * (copy_bytes / 2) / rec["copy_write_kib"]
    return fetch + write


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or 'unknown CPU'."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def host_cores() -> int:
    """CPU cores this process may run on (the affinity mask), else os.cpu_count()."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


_ORACLE_SAMPLE = """
import sys, time
sys.path.insert(0, {root!r})
import synthetic as syn
from oracle import pdhg as opdhg
from oracle.problem import Problem as OProblem, default_constants
u0 = syn.fourier_u0({seed}, {nx})
op = default_constants(OProblem(nx={nx}, nt={nt}, t_final={tf}, alpha=0.5, beta=0.0, space="fd_lf", time="bdf2"), u0)
t0 = time.perf_counter()
opdhg.run(op, u0, 0.6, 0.6, eps=0.0, max_iter={iters})
print(time.perf_counter() - t0)
"""


def oracle_single_thread(sample_iters: int) -> float:
    """Wall seconds of the same oracle sample in a fresh CPU-only process limited to one thread (the BLAS
    and FFT thread counts are fixed before numpy is imported)."""
    import subprocess
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS",
              "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    env["HIP_VISIBLE_DEVICES"] = ""
    code = _ORACLE_SAMPLE.format(root=ROOT, seed=SEED, nx=NX, nt=NT, tf=T_FINAL, iters=sample_iters)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600,
                         check=True)
    return float(out.stdout.strip().splitlines()[-1])


def cpu_baseline(sample_iters: int, u_gpu=None, gpu_iters=None):
    """FP64 oracle Algorithm 1 on the same workload, timed over `sample_iters` iterations on every host core
    and again in a one-thread process.  With the GPU's iteration count to 1e-8, the oracle's time to
    residual 1e-8 is extrapolated as that count times its seconds per iteration.  With the GPU solution
    u_gpu (to residual 1e-8) also the oracle's sequential Newton march of the same BDF2 scheme: its wall
    time and the max-norm difference to u_gpu (returned second, else None)."""
    import numpy as np

    import synthetic as syn
    from oracle import newton as onewton
    from oracle import pdhg as opdhg
    from oracle.problem import Problem as OProblem, default_constants
    u0 = syn.fourier_u0(SEED, NX)
    oprob = default_constants(OProblem(nx=NX, nt=NT, t_final=T_FINAL, alpha=0.5, beta=0.0, space="fd_lf",
                                       time="bdf2"), u0)
    c0, t0 = time.process_time(), time.perf_counter()
    opdhg.run(oprob, u0, 0.6, 0.6, eps=0.0, max_iter=sample_iters)
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    cores = host_cores()
    try:
        wall1 = oracle_single_thread(sample_iters)
    except Exception as exc:   # the one-thread leg is informative only
        log(f"one-thread oracle leg failed: {exc}")
        wall1 = None
    base = {
        "value": NX * NT * sample_iters / wall,
        "unit": "DOF-iterations/s",
        "cores": cores,
        "kind": "oracle",
        "nproc": os.cpu_count(),
        "concurrency": cpu / wall,
        "single_thread_value": NX * NT * sample_iters / wall1 if wall1 else None,
        "seconds_per_iteration": wall / sample_iters,
        "time_to_residual_1e-8_extrapolated_s": wall / sample_iters * gpu_iters if gpu_iters else None,
        "sample": f"{sample_iters} iterations of the FP64 NumPy/SciPy oracle (Algorithm 1) on the same "
                  f"{NX}x{NT} BDF2 LF Burgers problem; {wall:.1f} s wall on {cores} cores (process CPU time / wall "
                  f"= {cpu / wall:.1f}), " + (f"{wall1:.1f} s in a one-thread process; " if wall1 else "") +
                  f"{cpu_model()}",
    }
    if u_gpu is None:
        return base, None, None
    t0 = time.perf_counter()
    nw = onewton.march(oprob, u0)
    march_s = time.perf_counter() - t0
    err = {"max_abs_u_minus_newton_march": float(np.max(np.abs(u_gpu - nw))),
           "max_abs_u": float(np.max(np.abs(nw))), "newton_march_seconds": march_s}
    log(f"oracle Newton march: {march_s:.2f} s; max |u_gpu - u_newton| = {err['max_abs_u_minus_newton_march']:.3e}")
    return base, err, nw


BATCH_COUNT, BATCH_ITERS, BATCH_SEED = 256, 300, 0
BATCH_WORDS = {0: ("A: inverse FFT + dual step", 4), 1: ("B: primal step + residual + forward FFT", 4),
               2: ("C: column solve (banded Cholesky in t)", 2)}


def batch_problems(pk, torch_dtype, count=BATCH_COUNT):
    import synthetic as syn
    shapes = syn.batch_shapes(BATCH_SEED, count)
    probs = [pk.Problem(nx=nx, nt=nt, t_final=T_FINAL, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                        dtype=torch_dtype) for nx, nt, _ in shapes]
    u0s = [syn.fourier_u0(s, nx) for nx, _, s in shapes]
    return probs, u0s


def run_batch(args):
    """256 independent Burgers problems (BDF2, LF, T = 0.5, nx in {256..4096}, nt in {64..512}):
    the batched solver against one solve per problem, at a fixed iteration budget (FP32 by default),
    and FP64 time to residual 1e-8 on the first --ttr-problems problems."""
    import torch

    import paper_2207_07234_amd as pk
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    dtype = torch.float32 if args.dtype == "f32" or args.dtype is None else torch.float64
    esz = 4 if dtype == torch.float32 else 8
    probs, u0s = batch_problems(pk, dtype)
    bs = pk.BatchSolver(probs)
    u0 = bs.pack_u0(u0s)
    iters = args.batch_iters
    first = bs.solve(u0, eps=0.0, max_iter=2, check_every=2)          # step sizes (power iterations)
    taus = [s["tau_u"] for s in first.stats]
    grids = bs.tune(u0, tau_u=taus, tau_phi=taus)
    log(f"batch of {len(probs)}: {bs.u_elems} u points, tuned grids {grids}")
    for _ in range(args.warmup):
        bs.solve(u0, tau_u=taus, tau_phi=taus, eps=0.0, max_iter=iters, check_every=50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dofit = 0
    for k in range(args.steps):
        r = bs.solve(u0, tau_u=taus, tau_phi=taus, eps=0.0, max_iter=iters, check_every=50)
        dofit += sum(p.nx * p.nt * s["iters"] for p, s in zip(probs, r.stats))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = dofit / wall
    ndiv = sum(s["status"] == 2 for s in r.stats)
    log(f"batched: {wall / args.steps * 1e3:.1f} ms per solve of {iters} iterations, {value:.3e} DOF-it/s, "
        f"{ndiv} problems diverged")
    # one solve per problem, same step sizes and iteration budget
    singles = [pk.Solver(p) for p in probs]
    u0d = [torch.tensor(x, dtype=dtype, device=dev) for x in u0s]
    for i, s in enumerate(singles):
        s.solve(u0d[i], tau_u=taus[i], tau_phi=taus[i], eps=0.0, max_iter=2, check_every=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dofit_s = 0
    for i, s in enumerate(singles):
        rr = s.solve(u0d[i], tau_u=taus[i], tau_phi=taus[i], eps=0.0, max_iter=iters, check_every=50)
        dofit_s += probs[i].nx * probs[i].nt * rr.stats["iters"]
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    value_s = dofit_s / wall_s
    log(f"one solve per problem: {wall_s * 1e3:.1f} ms, {value_s:.3e} DOF-it/s")
    # per-pass device time (every problem running), dominant pass against the HBM roofline
    dof = sum(p.nx * p.nt for p in probs)
    kern = {}
    for kid, (name, words) in BATCH_WORDS.items():
        ms = bs.time_kernel(kid, reps=10)
        kern[kid] = (name, words, ms, words * esz * dof / (ms * 1e-3) / 1e9)
        log(f"batched pass {kid} {name}: {ms*1e3:.1f} us/launch, {kern[kid][3]:.0f} GB/s algorithmic")
    dom = max(kern, key=lambda k: kern[k][2])
    name, words, ms, gbs = kern[dom]
    ttr = None
    if args.ttr_problems > 0:
        ttr = batch_time_to_residual(pk, args.ttr_problems, dev)
    onestep = batch_onestep_time_to_residual(pk, dev)
    out = {
        "metric": METRIC, "value": value, "unit": "DOF-iterations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if dtype == torch.float32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{len(probs)} independent Burgers IVPs, FD Lax-Friedrichs, BDF2, T={T_FINAL}, "
                        f"nx in {{256..4096}}, nt in {{64..512}}, seeded Fourier u0, {iters} iterations per solve",
            "problems": len(probs), "dof": dof, "iterations_per_solve": iters, "diverged": ndiv,
            "grids": grids, "per_instance_value": value_s, "speedup_vs_per_instance": value / value_s,
            "time_to_residual_1e-8": ttr,
            "one_step_time_to_residual_1e-8": onestep,
        },
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "batched " + name,
                     "bytes_per_launch": words * esz * dof, "ms_per_launch": ms},
    }
    print(json.dumps(out), flush=True)


def fp32_run(pk, checks):
    """The same Burgers workload in FP32.  Its rounding floor lies far above 1e-8, so the solve stops on
    the single-precision rule: 500 iterations without a new best ||A(u)|| (the floor).  Reported:
    DOF-iterations/s, the status and the fused passes' event times at 4 bytes per word; the returned u
    goes to the oracle check (FP64 error against the Newton march)."""
    import torch
    import synthetic as syn
    s = pk.Solver(pk.Problem(nx=NX, nt=NT, t_final=T_FINAL, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                             dtype=torch.float32))
    u0 = torch.tensor(syn.fourier_u0(SEED, NX), dtype=torch.float32, device="cuda")
    kw = dict(eps=EPS, max_iter=100000, check_every=128, stall_iters=500)
    first = s.solve(u0, **kw)
    tau = first.stats["tau_u"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.solve(u0, tau_u=tau, tau_phi=tau, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n = r.stats["iters"]
    kern = {}
    for kid, (name, words) in KERNELS_FUSED.items():
        ms = s.time_kernel(kid, reps=50)
        kern[name] = {"us_per_launch": ms * 1e3, "algorithmic_GBs": words * 4 * NX * NT / (ms * 1e-3) / 1e9}
    checks["burgers_f32"] = r.u.double().cpu().numpy()
    log(f"FP32 run: status {r.status}, {n} iterations, {wall:.3f} s, {NX * NT * n / wall:.3e} DOF-it/s, "
        f"Rp {r.stats['res_primal']:.2e}")
    return {"status": r.status, "stop_rule": "500 iterations without a new best ||A(u)|| (eps 1e-8 unreachable)",
            "iterations": n, "seconds": wall, "dof_iterations_per_s": NX * NT * n / wall,
            "us_per_iteration": wall / n * 1e6, "res_primal": r.stats["res_primal"],
            "res_dual": r.stats["res_dual"], "kernels": kern, "fp64_error": None}


def advection_cfl4(pk):
    """Linear advection u_t + u_x = 0, 64 x 32, T = 2 (CFL 4), BE upwind, u0 = sin(2 pi x), FP64, sigma = tau =
    0.7, to residual 1e-10: the small latency-bound case (one graph chunk of a few microseconds per
    iteration).  The GPU tests pin its solution to the closed-form BE amplification at 1e-10."""
    import numpy as np
    import torch
    import synthetic as syn
    s = pk.Solver(pk.Problem(nx=64, nt=32, t_final=2.0, alpha=0.0, beta=1.0, time="be", space="fd_upwind",
                             dtype=torch.float64))
    u0 = torch.tensor(syn.sine_u0(64), dtype=torch.float64, device="cuda")
    s.solve(u0, tau_u=0.7, tau_phi=0.7, eps=1e-10, max_iter=5000, check_every=64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.solve(u0, tau_u=0.7, tau_phi=0.7, eps=1e-10, max_iter=5000, check_every=64)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n = r.stats["iters"]
    log(f"advection 64x32 CFL 4 to 1e-10: {n} iterations, {wall * 1e3:.2f} ms ({wall / n * 1e6:.2f} us/iteration)")
    return {"iterations": n, "seconds": wall, "us_per_iteration": wall / n * 1e6, "status": r.status,
            "variant": r.stats["variant"], "u_T_max": float(np.max(np.abs(r.u[-1].cpu().numpy())))}


# single problems too large for the MALL: (N_x, N_t, dtype)
LARGE_SIZES = ((2048, 2048, "f64"), (4096, 2048, "f64"), (4096, 2048, "f32"), (2048, 8192, "f64"),
               (4096, 8192, "f32"))


def large_single_sweep(pk):
    """Per-kernel device time of the fused passes on single problems large enough to fill the GPU many
    times over (N_t = 2048: 1024 row-pair blocks, four per CU; N_t = 8192, the column solve's limit, with
    each spectrum column spread over 8 wavefronts), against the HBM roofline; from 4096 x 2048 on, the
    working set (five arrays of N_x N_t values) exceeds the MALL."""
    import torch
    import synthetic as syn
    out = []
    for nx, nt, dts in LARGE_SIZES:
        dt = torch.float64 if dts == "f64" else torch.float32
        esz = 8 if dt == torch.float64 else 4
        prob = pk.Problem(nx=nx, nt=nt, t_final=T_FINAL, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf", dtype=dt)
        s = pk.Solver(prob)
        u0 = torch.tensor(syn.fourier_u0(SEED, nx), dtype=dt, device="cuda")
        s.solve(u0, tau_u=0.5, tau_phi=0.5, eps=0.0, max_iter=2, check_every=2)
        dof = nx * nt
        rec = {"nx": nx, "nt": nt, "dtype": "f64" if esz == 8 else "f32", "kernels": {}}
        for kid, (name, words) in KERNELS_FUSED.items():
            ms = s.time_kernel(kid, reps=20)
            gbs = words * esz * dof / (ms * 1e-3) / 1e9
            rec["kernels"][name] = {"us_per_launch": ms * 1e3, "algorithmic_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
            log(f"large single {nx}x{nt} {rec['dtype']}: {name}: {ms * 1e3:.1f} us/launch, {gbs:.0f} GB/s "
                f"({gbs / HBM_PEAK_GBS:.2f} of peak)")
        ms = s.time_kernel(COPY_KERNEL, reps=20)
        rec["copy_GBs"] = 2 * esz * dof / (ms * 1e-3) / 1e9
        out.append(rec)
        s.close()
        del s, u0
        torch.cuda.empty_cache()
    return out


def run_kernels(args):
    """Profiling driver: the fused passes only, event-timed (--kernel-reps launches each) on the single
    problems of the large sweep, and the three batched passes on the 256-problem batch (FP32, every
    problem running).  Each configuration is set up by a 2-iteration solve and also times the plain copy
    kernel of its size, whose counter readings calibrate the HBM counters of a profiler run."""
    import torch

    import paper_2207_07234_amd as pk
    import synthetic as syn
    torch.cuda.set_device(torch.device("cuda", 0))
    reps = args.kernel_reps
    out = {"single": [], "batch": None}
    for nx, nt, dt in LARGE_SIZES:
        tdt = torch.float64 if dt == "f64" else torch.float32
        esz = 8 if dt == "f64" else 4
        prob = pk.Problem(nx=nx, nt=nt, t_final=T_FINAL, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf", dtype=tdt)
        s = pk.Solver(prob)
        s.solve(torch.tensor(syn.fourier_u0(SEED, nx), dtype=tdt, device="cuda"), tau_u=0.5, tau_phi=0.5, eps=0.0,
                max_iter=2, check_every=2)
        rec = {"nx": nx, "nt": nt, "dtype": dt, "kernels": {}}
        for kid, (name, words) in KERNELS_FUSED.items():
            ms = s.time_kernel(kid, reps=reps)
            gbs = words * esz * nx * nt / (ms * 1e-3) / 1e9
            rec["kernels"][name] = {"us_per_launch": ms * 1e3, "algorithmic_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
            log(f"{nx}x{nt} {dt}: {name}: {ms * 1e3:.1f} us/launch, {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.2f})")
        ms = s.time_kernel(COPY_KERNEL, reps=reps)
        rec["copy_us"] = ms * 1e3
        out["single"].append(rec)
        s.close()
        del s
        torch.cuda.empty_cache()
    probs, u0s = batch_problems(pk, torch.float32)
    bs = pk.BatchSolver(probs)
    u0 = bs.pack_u0(u0s)
    taus = [0.5] * len(probs)   # fixed steps: no power iterations (the pass timings do not depend on them)
    grids = bs.tune(u0, tau_u=taus, tau_phi=taus)
    bs.solve(u0, tau_u=taus, tau_phi=taus, eps=0.0, max_iter=2, check_every=2)
    dof = sum(p.nx * p.nt for p in probs)
    rec = {"problems": len(probs), "dof": dof, "grids": grids, "kernels": {}}
    for kid, (name, words) in BATCH_WORDS.items():
        ms = bs.time_kernel(kid, reps=reps)
        gbs = words * 4 * dof / (ms * 1e-3) / 1e9
        rec["kernels"][name] = {"us_per_launch": ms * 1e3, "algorithmic_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
        log(f"batch f32 ({len(probs)} problems, {dof} DOF): {name}: {ms * 1e3:.1f} us/launch, {gbs:.0f} GB/s "
            f"({gbs / HBM_PEAK_GBS:.2f})")
    out["batch"] = rec
    print(json.dumps(out), flush=True)


def traffic_table3(pk):
    """The traffic example of Section 4.3 (f(u) = u - u^2 on [0, 2), piecewise-constant density, 256 x 32,
    T = 1, upwind finite differences (BE, BDF2) and the DG P1 nodal upwind scheme (BE), tau = 0.4, c = 1,
    tolerance 1e-3) through the three variants, in the columns of Table 3: iterations, world time
    (iterations in sequence) and work in units of N_x (iterations x levels)."""
    import numpy as np
    import torch
    import synthetic as syn
    u0 = torch.tensor(syn.traffic_u0(256, 2.0), dtype=torch.float64, device="cuda")
    out = {}
    # DG P1 nodes x_c -/+ h/4 of the cells [2j/N, 2(j+1)/N)
    xn = (np.arange(256) + 0.5) * (2.0 / 256)
    u0_dg = torch.tensor(np.stack([syn.traffic_u0_at(xn - 0.5 / 256), syn.traffic_u0_at(xn + 0.5 / 256)]),
                         dtype=torch.float64, device="cuda")
    for key, space, tm in (("be", "fd_upwind", "be"), ("bdf2", "fd_upwind", "bdf2"), ("dg_p1_be", "dg_p1_upwind", "be")):
        s = pk.Solver(pk.Problem(nx=256, nt=32, length=2.0, t_final=1.0, alpha=-1.0, beta=1.0, time=tm,
                                 space=space, precond_c=1.0))
        x0 = u0_dg if space == "dg_p1_upwind" else u0
        kw = dict(tau_u=0.4, tau_phi=0.4, eps=1e-3, max_iter=20000)
        v = s.solve(x0, check_every=64, **kw)
        rf = s.solve_refined(x0, nt_start=8, coarse_max_iter=1000, coarse_eps=1e-300, check_every=64, **kw)
        os_ = s.solve_onestep(x0, **kw)
        lv = rf.stats["level_iters"]
        out[key] = {
            "vanilla": {"iterations": v.stats["iters"], "world_time": v.stats["iters"],
                        "work_N": v.stats["iters"] * 33, "status": v.status},
            "mesh_refinement": {"iterations": lv, "world_time": sum(lv),
                                "work_N": sum(n * (m + 1) for n, m in zip(lv, (8, 16, 32))), "status": rf.status},
            "one_step": {"iterations": os_.stats["iters"], "world_time": os_.stats["iters"],
                         "work_N": 2 * os_.stats["iters"], "status": os_.status},
        }
        log(f"traffic example ({key}): vanilla {v.stats['iters']}, refinement {lv}, "
            f"one-step {os_.stats['iters']} iterations")
    out["paper"] = {"vanilla": [4573, 4573, 150909], "mesh_refinement": [[1000, 1000, 3601], 5601, 144833],
                    "one_step": [8627, 8627, 17254]}
    return out


def variant_comparison(pk, solver, prob, u0, tau, vanilla, checks):
    """Algorithms 1, 2 and 3 on the single workload (FP64, 1e-8); `vanilla` = (iterations, seconds)."""
    import torch
    out = {"algorithm_1": {"iterations": vanilla[0], "world_time": vanilla[0],
                           "work_N": vanilla[0] * (NT + 1), "seconds": vanilla[1], "status": 0}}
    # Algorithm 2 from N_t0 = 1; every level to 1e-8 (the first call builds the coarse plans)
    kw = dict(nt_start=1, coarse_eps=EPS, coarse_max_iter=200000, eps=EPS, max_iter=200000, check_every=128)
    solver.solve_refined(u0, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = solver.solve_refined(u0, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lv = r.stats["level_iters"]
    checks["mesh_refinement"] = r.u.double().cpu().numpy()
    nts = [1 << k for k in range(len(lv))]
    out["mesh_refinement"] = {"iterations": lv, "world_time": sum(lv),
                              "work_N": sum(n * (m + 1) for n, m in zip(lv, nts)), "seconds": wall,
                              "status": r.status}
    log(f"Algorithm 2: status {r.status}, iterations per level {lv}, {wall:.3f} s")
    # Algorithm 3, step residual 1e-8
    solver.solve_onestep(u0, eps=EPS, max_iter=20000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = solver.solve_onestep(u0, eps=EPS, max_iter=20000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _, _, res = solver.residual(r.u, r.phi, want_fields=False)
    n = r.stats["iters"]
    checks["one_step"] = r.u.double().cpu().numpy()
    out["one_step"] = {"iterations": n, "world_time": n, "work_N": 2 * n, "seconds": wall, "status": r.status,
                       "space_time_residual": list(res), "steps": NT,
                       "us_per_iteration": r.stats["seconds"] / n * 1e6}
    log(f"Algorithm 3: status {r.status}, {n} iterations ({min(r.stats['step_iters'])}.."
        f"{max(r.stats['step_iters'])} per step), {wall:.3f} s, space-time residual {res[0]:.2e} / {res[1]:.2e}")
    # the same two with the full-symbol preconditioner (the Gram of the linear-flux Jacobian)
    fp = pk.Problem(nx=NX, nt=NT, t_final=T_FINAL, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                    dtype=prob.dtype, precond_kind="full")
    fs = pk.Solver(fp)
    first = fs.solve(u0, eps=EPS, max_iter=200000, check_every=128)
    tf = first.stats["tau_u"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fs.solve(u0, tau_u=tf, tau_phi=tf, eps=EPS, max_iter=200000, check_every=128)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n = r.stats["iters"]
    checks["algorithm_1_full_symbol"] = r.u.double().cpu().numpy()
    cms = fs.time_kernel(1, reps=50)
    out["algorithm_1_full_symbol"] = {"iterations": n, "world_time": n, "work_N": n * (NT + 1), "seconds": wall,
                                      "status": r.status, "precond_c": r.stats["precond_c"],
                                      "us_per_iteration": wall / n * 1e6, "column_pass_us": cms * 1e3}
    log(f"Algorithm 1, full symbol: status {r.status}, {n} iterations, {wall:.3f} s "
        f"({wall / n * 1e6:.1f} us/iteration, column pass {cms * 1e3:.1f} us), c = {r.stats['precond_c']:.4f}")
    fs.solve_onestep(u0, eps=EPS, max_iter=20000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fs.solve_onestep(u0, eps=EPS, max_iter=20000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _, _, res = fs.residual(r.u, r.phi, want_fields=False)
    n = r.stats["iters"]
    checks["one_step_full_symbol"] = r.u.double().cpu().numpy()
    out["one_step_full_symbol"] = {"iterations": n, "world_time": n, "work_N": 2 * n, "seconds": wall,
                                   "status": r.status, "space_time_residual": list(res),
                                   "us_per_iteration": r.stats["seconds"] / n * 1e6}
    log(f"Algorithm 3, full symbol: status {r.status}, {n} iterations, {wall:.3f} s, "
        f"space-time residual {res[0]:.2e} / {res[1]:.2e}")
    if prob.dtype == torch.float64:
        # Algorithm 1 with the Gram preconditioner's spectral pass in float (u, phi, residuals, norms FP64)
        mp = pk.Problem(nx=NX, nt=NT, t_final=T_FINAL, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                        dtype=torch.float64, precond_kind="gram_f32")
        ms = pk.Solver(mp)
        ms.solve(u0, tau_u=tau, tau_phi=tau, eps=EPS, max_iter=200000, check_every=128)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ms.solve(u0, tau_u=tau, tau_phi=tau, eps=EPS, max_iter=200000, check_every=128)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        n = r.stats["iters"]
        checks["algorithm_1_gram_f32"] = r.u.double().cpu().numpy()
        kus = {name: ms.time_kernel(kid, reps=50) * 1e3 for kid, (name, _) in KERNELS_FUSED.items()}
        out["algorithm_1_gram_f32"] = {"iterations": n, "world_time": n, "work_N": n * (NT + 1), "seconds": wall,
                                       "status": r.status, "res_primal": r.stats["res_primal"],
                                       "res_dual": r.stats["res_dual"], "us_per_iteration": wall / n * 1e6,
                                       "kernel_us": kus}
        log(f"Algorithm 1, float spectral pass: status {r.status}, {n} iterations, {wall:.3f} s "
            f"({wall / n * 1e6:.1f} us/iteration; " + ", ".join(f"{k[:1]} {v:.1f} us" for k, v in kus.items()) + ")")
    return out


def batch_onestep_time_to_residual(pk, dev):
    """FP64, every problem of the batch workload by the batched one-step solver (Algorithm 3), step
    residual 1e-8."""
    import torch
    probs, u0s = batch_problems(pk, torch.float64)
    bs = pk.BatchSolver(probs)
    u0 = bs.pack_u0(u0s)
    bs.solve_onestep(u0, eps=EPS, max_iter=20000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = bs.solve_onestep(u0, eps=EPS, max_iter=20000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    slice_its = sum(p.nx * s["iters"] for p, s in zip(probs, r.stats))
    res = {"problems": len(probs), "dtype": "f64", "eps_step": EPS, "seconds": wall,
           "converged": sum(s["status"] == 0 for s in r.stats), "diverged": sum(s["status"] == 2 for s in r.stats),
           "max_iterations": max(s["iters"] for s in r.stats), "slice_dof_iterations_per_s": slice_its / wall}
    log(f"batched one-step (FP64, all {len(probs)} problems, step residual 1e-8): {wall:.3f} s, "
        f"{res['converged']} converged, {res['diverged']} diverged")
    return res


def batch_time_to_residual(pk, count, dev):
    """FP64, eps 1e-8: the first `count` problems of the batch workload solved together against one
    solve per problem (same step sizes); diverging problems stop at detection in both."""
    import torch
    probs, u0s = batch_problems(pk, torch.float64, count)
    bs = pk.BatchSolver(probs)
    u0 = bs.pack_u0(u0s)
    first = bs.solve(u0, eps=0.0, max_iter=2, check_every=2)
    taus = [s["tau_u"] for s in first.stats]
    bs.tune(u0, tau_u=taus, tau_phi=taus)
    kw = dict(eps=EPS, max_iter=40000, check_every=64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = bs.solve(u0, tau_u=taus, tau_phi=taus, **kw)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    singles = [pk.Solver(p) for p in probs]
    u0d = [torch.tensor(x, dtype=torch.float64, device=dev) for x in u0s]
    for i, s in enumerate(singles):
        s.solve(u0d[i], tau_u=taus[i], tau_phi=taus[i], eps=0.0, max_iter=2, check_every=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for i, s in enumerate(singles):
        rr = s.solve(u0d[i], tau_u=taus[i], tau_phi=taus[i], **kw)
        its.append((rr.stats["status"], rr.stats["iters"]))
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    same = all((st["status"], st["iters"]) == it for st, it in zip(r.stats, its))
    res = {"problems": count, "dtype": "f64", "eps": EPS, "batched_s": wall_b, "one_solve_per_problem_s": wall_s,
           "speedup": wall_s / wall_b, "converged": sum(s["status"] == 0 for s in r.stats),
           "diverged": sum(s["status"] == 2 for s in r.stats), "max_iters": max(s["iters"] for s in r.stats),
           "same_n_star_as_single": same}
    log(f"time to residual 1e-8 (FP64, {count} problems): batched {wall_b:.2f} s, one solve per problem "
        f"{wall_s:.2f} s, {res['converged']} converged, {res['diverged']} diverged, n* identical: {same}")
    return res


DG_NX, DG_NT, DG_ITERS = 4096, 512, 2000
DG_KERNELS = {   # kernel id: (name, algorithmic words per DOF; DOF = 3 coefficients x cells x levels)
    7: ("A: inverse FFT + dual step", 4),
    4: ("DG primal step + dual residual", 4),
    0: ("DG residual + forward FFT", 2),
    1: ("DG column solve (per-mode eigenbasis, banded Cholesky in t)", 2),
}


DG_CPU_NT = 64


def dg_cpu_baseline(sample_iters: int):
    """FP64 oracle Algorithm 1 with the DG P2 discretisation on a bounded sample of the workload: all
    4096 cells, the first DG_CPU_NT levels (same h_t = 3 h_x), `sample_iters` iterations (the oracle's
    dense per-mode solves make one full-size iteration take minutes)."""
    import numpy as np

    import synthetic as syn
    from oracle import dg as odg
    from oracle import pdhg as opdhg
    from oracle.problem import Problem as OProblem, default_constants
    u0 = odg.p2_project(lambda x: syn.fourier_u0_at(SEED, x), DG_NX)
    op = default_constants(OProblem(nx=DG_NX, nt=DG_CPU_NT, t_final=3.0 * DG_CPU_NT / DG_NX, alpha=0.5, beta=0.0,
                                    space="dg_p2_llf", time="be"), u0)
    c0, t0 = time.process_time(), time.perf_counter()
    opdhg.run(op, u0, 0.6, 0.6, eps=0.0, max_iter=sample_iters)
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    return {"value": 3 * DG_NX * DG_CPU_NT * sample_iters / wall, "unit": "DOF-iterations/s",
            "cores": host_cores(), "concurrency": cpu / wall, "kind": "oracle",
            "sample": f"{sample_iters} iterations of the FP64 NumPy/SciPy oracle (Algorithm 1, DG P2) on the "
                      f"workload's {DG_NX} cells and first {DG_CPU_NT} levels (h_t = 3 h_x); {wall:.1f} s wall, "
                      f"host has {os.cpu_count()} CPUs ({cpu_model()})"}


def run_dg(args):
    """Burgers with DG P2 (Legendre, local Lax-Friedrichs), 4096 cells x 512 levels, h_t = 3 h_x,
    backward Euler, seeded Fourier u0 projected on P2; FP32 by default, fixed iteration budget."""
    import torch

    import paper_2207_07234_amd as pk
    import synthetic as syn
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    dtype = torch.float32 if args.dtype in (None, "f32") else torch.float64
    esz = 4 if dtype == torch.float32 else 8
    T = 3.0 * DG_NT / DG_NX
    prob = pk.Problem(nx=DG_NX, nt=DG_NT, t_final=T, alpha=0.5, beta=0.0, time="be", space="dg_p2_llf",
                      dtype=dtype)
    solver = pk.Solver(prob)
    u0 = torch.tensor(syn.fourier_u0_legendre(SEED, DG_NX), dtype=dtype, device=dev)
    u = torch.empty((DG_NT + 1, 3, DG_NX), dtype=dtype, device=dev)
    phi = torch.empty((DG_NT, 3, DG_NX), dtype=dtype, device=dev)
    ws = torch.empty(solver.workspace_bytes, dtype=torch.uint8, device=dev)
    iters = args.dg_iters
    kw = dict(u=u, phi=phi, workspace=ws, check_every=128, eps=args.dg_eps, max_iter=iters)
    first = solver.solve(u0, **kw)
    tau = first.stats["tau_u"]
    log(f"DG warm-up: nu_max {first.stats['nu_max']:.4f} tau {tau:.4f} Rp {first.stats['res_primal']:.3e}")
    for _ in range(max(0, args.warmup - 1)):
        solver.solve(u0, tau_u=tau, tau_phi=tau, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    for k in range(args.steps):
        r = solver.solve(u0, tau_u=tau, tau_phi=tau, **kw)
        done += r.stats["iters"]
        log(f"DG step {k}: status {r.status} iters {r.stats['iters']} Rp {r.stats['res_primal']:.3e} "
            f"Rd {r.stats['res_dual']:.3e} loop {r.stats['seconds']*1e3:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dof = 3 * DG_NX * DG_NT
    value = dof * done / wall
    iters = r.stats["iters"]
    kern = {}
    for kid, (name, words) in DG_KERNELS.items():
        ms = solver.time_kernel(kid, reps=30)
        kern[kid] = (name, words, ms, words * esz * dof / (ms * 1e-3) / 1e9)
        log(f"DG kernel {kid} {name}: {ms*1e3:.1f} us/launch, {kern[kid][3]:.0f} GB/s algorithmic")
    dom = max(kern, key=lambda k: kern[k][2])
    name, words, ms, gbs = kern[dom]
    out = {
        "metric": METRIC, "value": value, "unit": "DOF-iterations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if dtype == torch.float32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"Burgers, DG P2 Legendre with local Lax-Friedrichs flux, backward Euler, "
                               f"{DG_NX} cells x {DG_NT} levels, h_t = 3 h_x (T = {T}), seeded Fourier u0 projected "
                               f"on P2, {iters} iterations per solve",
                   "cells": DG_NX, "nt": DG_NT, "dof": dof, "iterations_per_solve": iters, "tau": tau,
                   "res_primal": r.stats["res_primal"], "res_dual": r.stats["res_dual"],
                   "us_per_iteration_wall": wall / done * 1e6, "eps": args.dg_eps,
                   "time_to_residual_s": wall / args.steps if args.dg_eps > 0 else None, "status": r.status,
                   "kernel_sum_us_per_iteration": sum(v[2] for v in kern.values()) * 1e3},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "DG " + name,
                     "bytes_per_launch": words * esz * dof, "ms_per_launch": ms},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = dg_cpu_baseline(args.dg_cpu_iters)
    print(json.dumps(out), flush=True)


def run_adjoint(args):
    """Differentiable workload: viscous Burgers (gamma = 1e-3), 2048 x 512, T = 0.5, backward Euler,
    Lax-Friedrichs flux with centred diffusion, loss h_x ||u^{N_t} - target||^2 with the target from
    seed + 1.  The forward solve (FP32: to its rounding floor, 1000 iterations without a new best
    ||A(u)||; FP64: residual 1e-8), then the adjoint march for d loss / d u0, timed with HIP events."""
    import torch

    import paper_2207_07234_amd as pk
    import synthetic as syn
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    dtype = torch.float32 if args.dtype in (None, "f32") else torch.float64
    esz = 4 if dtype == torch.float32 else 8
    nx, nt = NX, NT
    prob = pk.Problem(nx=nx, nt=nt, t_final=T_FINAL, alpha=0.5, beta=0.0, gamma=1e-3, time="be", space="fd_lf",
                      dtype=dtype, precond_gamma_hat=1e-3)
    solver = pk.Solver(prob)
    u0 = torch.tensor(syn.fourier_u0(SEED, nx), dtype=dtype, device=dev)
    tgt = torch.tensor(syn.fourier_u0(SEED + 1, nx), dtype=dtype, device=dev)
    eps, max_iter = 1e-8, 200000
    stall = 1000 if esz == 4 else 0   # FP32: to its rounding floor
    first = solver.solve(u0, eps=eps, max_iter=max_iter, check_every=128, stall_iters=stall)
    tau = first.stats["tau_u"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = solver.solve(u0, tau_u=tau, tau_phi=tau, eps=eps, max_iter=max_iter, check_every=128,
                         stall_iters=stall)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / args.steps
    n = r.stats["iters"]
    log(f"forward: status {r.status}, {n} iterations, {fwd:.3f} s, Rp {r.stats['res_primal']:.3e} "
        f"Rd {r.stats['res_dual']:.3e}")
    g = torch.zeros((nt + 1, nx), dtype=dtype, device=dev)
    g[-1] = (2.0 / nx) * (r.u[-1] - tgt)
    grad = solver.adjoint_solve(r.u, g)
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        grad = solver.adjoint_solve(r.u, g)
    e1.record()
    torch.cuda.synchronize()
    adj_ms = e0.elapsed_time(e1) / reps
    adj_bytes = (2 * (nt + 1) * nx + nx) * esz
    adj_gbs = adj_bytes / (adj_ms * 1e-3) / 1e9
    log(f"adjoint march: {adj_ms * 1e3:.1f} us ({adj_ms * 1e3 / nt:.2f} us per level), {adj_gbs:.1f} GB/s; "
        f"|grad|max {float(grad.abs().max()):.3e}")
    out = {
        "metric": METRIC, "value": nx * nt * n / fwd, "unit": "DOF-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": (fwd + adj_ms * 1e-3) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if esz == 4 else "f64", "data": "synthetic",
        "config": {"workload": f"differentiable viscous Burgers (gamma 1e-3), FD Lax-Friedrichs + centred "
                               f"diffusion, backward Euler, {nx}x{nt}, T={T_FINAL}, loss h_x|u(T)-target|^2, "
                               f"seeds {SEED}/{SEED + 1}",
                   "forward_iterations": n, "forward_s": fwd, "forward_status": r.status,
                   "res_primal": r.stats["res_primal"], "res_dual": r.stats["res_dual"], "eps": eps,
                   "adjoint_ms": adj_ms, "adjoint_us_per_level": adj_ms * 1e3 / nt,
                   "backward_share": adj_ms * 1e-3 / (fwd + adj_ms * 1e-3)},
        "roofline": {"bound": "hbm", "achieved": adj_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": adj_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "adjoint march (N_t sequential periodic tridiagonal solves in one workgroup)",
                     "bytes_per_launch": adj_bytes, "ms_per_launch": adj_ms},
    }
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ the other workloads (variants)
def dg_summary(pk, checks):
    """DG P2 workload (Burgers, Legendre P2 with local Lax-Friedrichs, 4096 cells x 512 levels, h_t = 3 h_x,
    backward Euler).  FP32 to its rounding floor (500 iterations without a new best ||A(u)||) and FP64 to
    residual 1e-8: time to residual, DOF-iterations/s and the passes' event times against the roofline."""
    import torch
    import synthetic as syn
    T = 3.0 * DG_NT / DG_NX
    dof = 3 * DG_NX * DG_NT
    out = {"workload": f"Burgers, DG P2 Legendre, local Lax-Friedrichs, backward Euler, {DG_NX} cells x {DG_NT} "
                       f"levels, h_t = 3 h_x (T = {T})", "dof": dof}
    for dt, key in ((torch.float32, "f32"), (torch.float64, "f64")):
        esz = 4 if dt == torch.float32 else 8
        s = pk.Solver(pk.Problem(nx=DG_NX, nt=DG_NT, t_final=T, alpha=0.5, beta=0.0, time="be", space="dg_p2_llf",
                                 dtype=dt))
        u0 = torch.tensor(syn.fourier_u0_legendre(SEED, DG_NX), dtype=dt, device="cuda")
        kw = dict(eps=EPS, max_iter=100000, check_every=128, stall_iters=500 if esz == 4 else 0)
        first = s.solve(u0, **kw)
        tau = first.stats["tau_u"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve(u0, tau_u=tau, tau_phi=tau, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        n = r.stats["iters"]
        kern = {}
        for kid, (name, words) in DG_KERNELS.items():
            ms = s.time_kernel(kid, reps=30)
            gbs = words * esz * dof / (ms * 1e-3) / 1e9
            kern[name] = {"us_per_launch": ms * 1e3, "algorithmic_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
        dom = max(kern, key=lambda k: kern[k]["us_per_launch"])   # of the loop body's passes
        checks["dg_" + key] = r.u.double().cpu().numpy()
        # the implicit adjoint at this solution (terminal loss |u^{N_t}|^2 h_x): one block-tridiagonal
        # cyclic reduction per level, in one workgroup
        g = torch.zeros_like(r.u)
        g[-1] = 2.0 * (1.0 / DG_NX) * r.u[-1]
        s.adjoint_solve(r.u, g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.adjoint_solve(r.u, g)
        torch.cuda.synchronize()
        adj_ms = (time.perf_counter() - t0) * 1e3
        if esz == 4:   # the residual with its per-cell products on the matrix cores, beside the VALU residual
            r_valu = s.time_kernel(5, reps=30)
            r_mfma = s.time_kernel(9, reps=30)
            kern["residual (unfused), VALU"] = {"us_per_launch": r_valu * 1e3}
            kern["residual (unfused), per-cell products on MFMA"] = {"us_per_launch": r_mfma * 1e3}
            log(f"DG P2 f32 unfused residual: VALU {r_valu * 1e3:.1f} us, MFMA products {r_mfma * 1e3:.1f} us")
        out[key] = {"status": r.status, "iterations": n, "seconds": wall, "dof_iterations_per_s": dof * n / wall,
                    "us_per_iteration": wall / n * 1e6, "res_primal": r.stats["res_primal"],
                    "res_dual": r.stats["res_dual"], "tau": tau, "kernels": kern, "dominant": dom,
                    "dominant_frac": kern[dom]["frac"], "fp64_error": None, "adjoint_ms": adj_ms,
                    "stop": "residual 1e-8" if esz == 8 else "500 iterations without a new best ||A(u)||"}
        log(f"DG P2 {key}: status {r.status}, {n} iterations, {wall:.3f} s, {dof * n / wall:.3e} DOF-it/s; "
            f"dominant {dom} {kern[dom]['us_per_launch']:.1f} us ({kern[dom]['frac']:.2f} of peak); "
            f"adjoint march {adj_ms:.1f} ms")
        s.close()
        del s
        torch.cuda.empty_cache()
    return out


def batch_summary(pk, checks, sample=6):
    """The 256-problem batch (Burgers, BDF2, LF, T = 0.5, nx in {256..4096}, nt in {64..512}):
    * FP32 throughput at a fixed budget of BATCH_ITERS iterations, batched against one solve per problem;
    * FP64 time to residual 1e-8 over all 256 problems with Algorithm 1 (a diverging problem stops at
      detection and returns its last good checkpoint; counts reported), batched against one solve per
      problem;
    * FP64 time to step residual 1e-8 over all 256 problems with Algorithm 3 (one-step), batched (one
      launch) against one solve per problem.
    Converged problems of a sample go to the oracle check."""
    import torch
    dev = torch.device("cuda", 0)
    out = {}
    # ---- FP32 throughput
    probs, u0s = batch_problems(pk, torch.float32)
    bs = pk.BatchSolver(probs)
    u0 = bs.pack_u0(u0s)
    first = bs.solve(u0, eps=0.0, max_iter=2, check_every=2)
    taus = [st["tau_u"] for st in first.stats]
    grids = bs.tune(u0, tau_u=taus, tau_phi=taus)
    bs.solve(u0, tau_u=taus, tau_phi=taus, eps=0.0, max_iter=BATCH_ITERS, check_every=50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = bs.solve(u0, tau_u=taus, tau_phi=taus, eps=0.0, max_iter=BATCH_ITERS, check_every=50)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    dofit_b = sum(p.nx * p.nt * st["iters"] for p, st in zip(probs, r.stats))
    dof = sum(p.nx * p.nt for p in probs)
    kern = {}
    for kid, (name, words) in BATCH_WORDS.items():
        ms = bs.time_kernel(kid, reps=10)
        gbs = words * 4 * dof / (ms * 1e-3) / 1e9
        kern[name] = {"us_per_launch": ms * 1e3, "algorithmic_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
    dom = max(kern, key=lambda k: kern[k]["us_per_launch"])
    singles = [pk.Solver(p) for p in probs]
    u0d = [torch.tensor(x, dtype=torch.float32, device=dev) for x in u0s]
    for i, s in enumerate(singles):
        s.solve(u0d[i], tau_u=taus[i], tau_phi=taus[i], eps=0.0, max_iter=2, check_every=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dofit_s = 0
    for i, s in enumerate(singles):
        rr = s.solve(u0d[i], tau_u=taus[i], tau_phi=taus[i], eps=0.0, max_iter=BATCH_ITERS, check_every=50)
        dofit_s += probs[i].nx * probs[i].nt * rr.stats["iters"]
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    out["f32_fixed_budget"] = {
        "iterations": BATCH_ITERS, "problems": len(probs), "dof": dof, "grids": grids,
        "batched_s": wall_b, "batched_dof_iterations_per_s": dofit_b / wall_b,
        "one_solve_per_problem_s": wall_s, "one_solve_per_problem_dof_iterations_per_s": dofit_s / wall_s,
        "diverged": sum(st["status"] == 2 for st in r.stats), "kernels": kern, "dominant": dom,
        "dominant_frac": kern[dom]["frac"]}
    log(f"batch FP32, {BATCH_ITERS} iterations: batched {wall_b * 1e3:.1f} ms ({dofit_b / wall_b:.3e} DOF-it/s), "
        f"one solve per problem {wall_s * 1e3:.1f} ms; dominant {dom} {kern[dom]['frac']:.2f} of peak")
    del singles, u0d, bs
    torch.cuda.empty_cache()
    # ---- FP64 time to residual, Algorithm 1 and Algorithm 3, all problems
    probs, u0s = batch_problems(pk, torch.float64)
    bs = pk.BatchSolver(probs)
    u0 = bs.pack_u0(u0s)
    first = bs.solve(u0, eps=0.0, max_iter=2, check_every=2)
    taus = [st["tau_u"] for st in first.stats]
    bs.tune(u0, tau_u=taus, tau_phi=taus)
    kw = dict(eps=EPS, max_iter=40000, check_every=64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = bs.solve(u0, tau_u=taus, tau_phi=taus, **kw)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    singles = [pk.Solver(p) for p in probs]
    u0d = [torch.tensor(x, dtype=torch.float64, device=dev) for x in u0s]
    for i, s in enumerate(singles):
        s.solve(u0d[i], tau_u=taus[i], tau_phi=taus[i], eps=0.0, max_iter=2, check_every=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    single_stats = []
    for i, s in enumerate(singles):
        rr = s.solve(u0d[i], tau_u=taus[i], tau_phi=taus[i], **kw)
        single_stats.append((rr.stats["status"], rr.stats["iters"]))
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    conv = [i for i, st in enumerate(r.stats) if st["status"] == 0]
    pick = conv[:: max(1, len(conv) // sample)][:sample]
    checks["batch_alg1"] = {i: (probs[i].nx, probs[i].nt, u0s[i], r.views_u[i].double().cpu().numpy())
                            for i in pick}
    out["f64_algorithm_1_to_1e-8"] = {
        "problems": len(probs), "converged": len(conv), "diverged": sum(st["status"] == 2 for st in r.stats),
        "max_iter_reached": sum(st["status"] == 1 for st in r.stats),
        "batched_s": wall_b, "one_solve_per_problem_s": wall_s, "speedup": wall_s / wall_b,
        "same_status_and_n_star_as_single": all((st["status"], st["iters"]) == ss
                                                for st, ss in zip(r.stats, single_stats)),
        "differing_from_single": [(i, probs[i].nx, probs[i].nt, (st["status"], st["iters"]), ss)
                                  for i, (st, ss) in enumerate(zip(r.stats, single_stats))
                                  if (st["status"], st["iters"]) != ss][:12],
        "max_n_star": max(st["iters"] for st in r.stats),
        "converged_dof_iterations": sum(probs[i].nx * probs[i].nt * r.stats[i]["iters"] for i in conv),
        "fp64_error": None}
    log(f"batch FP64 Algorithm 1 to 1e-8: batched {wall_b:.2f} s, one solve per problem {wall_s:.2f} s; "
        f"{len(conv)} converged, {out['f64_algorithm_1_to_1e-8']['diverged']} diverged")
    # Algorithm 3
    bs.solve_onestep(u0, eps=EPS, max_iter=20000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = bs.solve_onestep(u0, eps=EPS, max_iter=20000)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    for i, s in enumerate(singles):
        s.solve_onestep(u0d[i], eps=EPS, max_iter=2)   # step sizes (power iteration) outside the timing
    taus1 = [st["tau_u"] for st in r.stats]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok_single = 0
    for i, s in enumerate(singles):
        rr = s.solve_onestep(u0d[i], tau_u=taus1[i], tau_phi=taus1[i], eps=EPS, max_iter=20000)
        ok_single += rr.status == 0
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    conv = [i for i, st in enumerate(r.stats) if st["status"] == 0]
    pick = list(range(0, len(probs), max(1, len(probs) // sample)))[:sample]
    checks["batch_alg3"] = {i: (probs[i].nx, probs[i].nt, u0s[i], r.views_u[i].double().cpu().numpy())
                            for i in pick}
    slice_its = sum(p.nx * st["iters"] for p, st in zip(probs, r.stats))
    out["f64_algorithm_3_to_1e-8"] = {
        "problems": len(probs), "converged": len(conv), "converged_single": ok_single,
        "diverged": sum(st["status"] == 2 for st in r.stats), "batched_s": wall_b,
        "one_solve_per_problem_s": wall_s, "speedup": wall_s / wall_b,
        "slice_dof_iterations_per_s": slice_its / wall_b, "fp64_error": None}
    log(f"batch FP64 Algorithm 3 to step residual 1e-8: batched {wall_b:.3f} s, one solve per problem "
        f"{wall_s:.3f} s; {len(conv)} converged")
    return out


def adjoint_summary(pk, checks):
    """Differentiable workload: viscous Burgers (gamma = 1e-3), 2048 x 512, T = 0.5, BE, LF + centred
    diffusion, loss h_x ||u^{N_t} - target||^2 (target from seed + 1).  Forward in FP32 (to its rounding
    floor: 1000 iterations without a new best) and FP64 (residual 1e-8), then the adjoint march for
    d loss / d u0; the gradients go to the oracle check."""
    import torch
    import synthetic as syn
    out = {"workload": f"viscous Burgers (gamma 1e-3), FD LF + centred diffusion, BE, {NX}x{NT}, T={T_FINAL}, "
                       f"loss h_x |u(T) - target|^2, seeds {SEED}/{SEED + 1}"}
    for dt, key in ((torch.float32, "f32"), (torch.float64, "f64")):
        esz = 4 if dt == torch.float32 else 8
        s = pk.Solver(pk.Problem(nx=NX, nt=NT, t_final=T_FINAL, alpha=0.5, beta=0.0, gamma=1e-3, time="be",
                                 space="fd_lf", dtype=dt, precond_gamma_hat=1e-3))
        u0 = torch.tensor(syn.fourier_u0(SEED, NX), dtype=dt, device="cuda")
        tgt = torch.tensor(syn.fourier_u0(SEED + 1, NX), dtype=dt, device="cuda")
        kw = dict(eps=EPS, max_iter=200000, check_every=128, stall_iters=1000 if esz == 4 else 0)
        first = s.solve(u0, **kw)
        tau = first.stats["tau_u"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.solve(u0, tau_u=tau, tau_phi=tau, **kw)
        torch.cuda.synchronize()
        fwd = time.perf_counter() - t0
        g = torch.zeros((NT + 1, NX), dtype=dt, device="cuda")
        g[-1] = (2.0 / NX) * (r.u[-1] - tgt)
        grad = s.adjoint_solve(r.u, g)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            grad = s.adjoint_solve(r.u, g)
        e1.record()
        torch.cuda.synchronize()
        adj_ms = e0.elapsed_time(e1) / 10
        adj_bytes = (2 * (NT + 1) * NX + NX) * esz
        n = r.stats["iters"]
        checks["adjoint_" + key] = grad.double().cpu().numpy()
        out[key] = {"forward_status": r.status, "forward_iterations": n, "forward_s": fwd,
                    "dof_iterations_per_s": NX * NT * n / fwd, "res_primal": r.stats["res_primal"],
                    "adjoint_ms": adj_ms, "adjoint_GBs": adj_bytes / (adj_ms * 1e-3) / 1e9,
                    "differentiable_solve_s": fwd + adj_ms * 1e-3, "gradient_fp64_rel_error": None}
        log(f"differentiable {key}: forward status {r.status}, {n} iterations, {fwd:.3f} s; adjoint {adj_ms:.2f} ms")
        s.close()
    return out


def onestep_us_sweep(pk):
    """Algorithm 3 microseconds per iteration against N_x (FP64, BDF2 Burgers, 8 steps of a fixed 200
    iterations each, h_t = 2 h_x): the one-workgroup march is latency-bound."""
    import torch
    import synthetic as syn
    out = {}
    for nx in (256, 512, 2048, 4096):
        s = pk.Solver(pk.Problem(nx=nx, nt=8, t_final=16.0 / nx, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                                 dtype=torch.float64))
        u0 = torch.tensor(syn.fourier_u0(SEED, nx), dtype=torch.float64, device="cuda")
        s.solve_onestep(u0, tau_u=0.5, tau_phi=0.5, eps=0.0, max_iter=200)
        r = s.solve_onestep(u0, tau_u=0.5, tau_phi=0.5, eps=0.0, max_iter=200)
        out[str(nx)] = r.stats["seconds"] / r.stats["iters"] * 1e6
        s.close()
    log("one-step us per iteration (FP64): " + ", ".join(f"{k}: {v:.1f}" for k, v in out.items()))
    return out


def oracle_checks(checks, variants, headline_nw):
    """The cpu_baseline leg's oracle references: the Newton march of each workload's implicit scheme and
    the adjoint gradient, and the max-norm FP64 error of every GPU result against them."""
    import numpy as np

    import synthetic as syn
    from oracle import adjoint as oadj
    from oracle import dg as odg
    from oracle import newton as onewton
    from oracle.problem import Problem as OProblem, default_constants

    def err(a, ref):
        return float(np.max(np.abs(a - ref)))

    if headline_nw is not None:
        for key, target in (("burgers_f32", ("fp32_stop_rule",)), ("mesh_refinement", ("mesh_refinement",)),
                            ("one_step", ("one_step",)), ("algorithm_1_full_symbol", ("algorithm_1_full_symbol",)),
                            ("one_step_full_symbol", ("one_step_full_symbol",)),
                            ("algorithm_1_gram_f32", ("algorithm_1_gram_f32",))):
            if key in checks and target[0] in variants:
                variants[target[0]]["fp64_error"] = err(checks[key], headline_nw)
    if "dg_f64" in checks and "dg_p2" in variants:
        t0 = time.perf_counter()
        u0 = odg.p2_project(lambda x: syn.fourier_u0_at(SEED, x), DG_NX)
        op = default_constants(OProblem(nx=DG_NX, nt=DG_NT, t_final=3.0 * DG_NT / DG_NX, alpha=0.5, beta=0.0,
                                        space="dg_p2_llf", time="be"), u0)
        nw = onewton.march(op, u0)
        for key in ("f32", "f64"):
            variants["dg_p2"][key]["fp64_error"] = err(checks["dg_" + key], nw)
        log(f"oracle DG Newton march {time.perf_counter() - t0:.1f} s: errors "
            f"{variants['dg_p2']['f32']['fp64_error']:.2e} (FP32), {variants['dg_p2']['f64']['fp64_error']:.2e} (FP64)")
    if "batch_256" in variants:
        for ck, vk in (("batch_alg1", "f64_algorithm_1_to_1e-8"), ("batch_alg3", "f64_algorithm_3_to_1e-8")):
            worst = 0.0
            for i, (nx, nt, u0, u) in checks.get(ck, {}).items():
                op = default_constants(OProblem(nx=nx, nt=nt, t_final=T_FINAL, alpha=0.5, beta=0.0, space="fd_lf",
                                                time="bdf2"), u0)
                worst = max(worst, err(u, onewton.march(op, u0)))
            variants["batch_256"][vk]["fp64_error"] = worst
            variants["batch_256"][vk]["fp64_error_sample"] = sorted(checks.get(ck, {}))
    if "adjoint_f64" in checks and "differentiable" in variants:
        t0 = time.perf_counter()
        u0, tgt = syn.fourier_u0(SEED, NX), syn.fourier_u0(SEED + 1, NX)
        op = default_constants(OProblem(nx=NX, nt=NT, t_final=T_FINAL, alpha=0.5, beta=0.0, gamma=1e-3,
                                        space="fd_lf", time="be"), u0)
        nw = onewton.march(op, u0)
        gref = oadj.gradient_u0(op, nw, oadj.terminal_loss_grad(op, nw, tgt))
        for key in ("f32", "f64"):
            variants["differentiable"][key]["gradient_fp64_rel_error"] = \
                err(checks["adjoint_" + key], gref) / float(np.max(np.abs(gref)))
        log(f"oracle adjoint gradient {time.perf_counter() - t0:.1f} s")



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--fixed-iters", type=int, default=0,
                    help="run exactly this many iterations per solve instead of solving to 1e-8 (profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the Algorithm 2 / Algorithm 3 comparison")
    ap.add_argument("--dtype", choices=["f64", "f32"], default=None,
                    help="compute type (default f64 for the single workload, f32 for the batch)")
    ap.add_argument("--variant", type=int, default=0, help="0 auto (fused), 1 unfused, 2 fused")
    ap.add_argument("--workload", choices=["burgers", "batch", "dg", "adjoint", "kernels"], default="burgers",
                    help="kernels: event-time the passes of the large single problems and of the 256-problem "
                         "batch only (profiler driver)")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--dg-iters", type=int, default=DG_ITERS)
    ap.add_argument("--dg-cpu-iters", type=int, default=2)
    ap.add_argument("--dg-eps", type=float, default=0.0,
                    help="DG workload: solve to this residual (max --dg-iters iterations) instead of a fixed count")
    ap.add_argument("--batch-iters", type=int, default=BATCH_ITERS)
    ap.add_argument("--ttr-problems", type=int, default=32,
                    help="batch workload: FP64 time-to-residual comparison on this many problems (0 = skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is design-only",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "kernels":
        run_kernels(args)
        return
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "adjoint":
        return run_adjoint(args)
    if args.workload == "dg":
        run_dg(args)
        return
    if args.dtype is None:
        args.dtype = "f64"

    import torch

    import paper_2207_07234_amd as pk
    import synthetic as syn

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    esz = 8 if dtype == torch.float64 else 4
    prob = pk.Problem(nx=NX, nt=NT, t_final=T_FINAL, alpha=0.5, beta=0.0, time="bdf2", space="fd_lf",
                      dtype=dtype)
    solver = pk.Solver(prob)
    u0 = torch.tensor(syn.fourier_u0(SEED, NX), dtype=dtype, device=dev)
    u = torch.empty((NT + 1, NX), dtype=dtype, device=dev)
    phi = torch.empty((NT, NX), dtype=dtype, device=dev)
    ws = torch.empty(solver.workspace_bytes, dtype=torch.uint8, device=dev)
    eps = EPS if dtype == torch.float64 else 0.0
    max_iter = 200000 if dtype == torch.float64 else 5000
    if args.fixed_iters > 0:
        eps, max_iter = 0.0, args.fixed_iters

    # warm-up: the first solve runs the power iteration; later solves reuse its step sizes
    kw = dict(u=u, phi=phi, workspace=ws, check_every=128, variant=args.variant)
    first = solver.solve(u0, eps=eps, max_iter=max_iter, **kw)
    tau = first.stats["tau_u"]
    log(f"warm-up solve: status {first.status} iters {first.stats['iters']} nu_max {first.stats['nu_max']:.6f} "
        f"tau {tau:.6f} Rp {first.stats['res_primal']:.3e} Rd {first.stats['res_dual']:.3e}")
    for _ in range(max(0, args.warmup - 1)):
        solver.solve(u0, tau_u=tau, tau_phi=tau, eps=eps, max_iter=max_iter, **kw)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    stats = None
    for k in range(args.steps):
        r = solver.solve(u0, tau_u=tau, tau_phi=tau, eps=eps, max_iter=max_iter, **kw)
        iters.append(r.stats["iters"])
        stats = r.stats
        log(f"step {k}: status {r.status} iters {r.stats['iters']} loop {r.stats['seconds']*1e3:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    dof = NX * NT
    value = dof * sum(iters) / wall
    u_final = u.double().cpu().numpy() if eps > 0 else None   # converged solution, for the oracle check

    # per-kernel device time (HIP events on the solve's stream), buffers of the last solve
    kern = {}
    table = KERNELS_FUSED if stats["variant"] == 2 else KERNELS_UNFUSED
    for kid, (name, words) in table.items():
        ms = solver.time_kernel(kid, reps=50)
        kern[kid] = (name, words, ms, words * esz * dof / (ms * 1e-3) / 1e9)
        log(f"kernel {kid} {name}: {ms*1e3:.1f} us/launch, {kern[kid][3]:.0f} GB/s algorithmic")
    dom = max(kern, key=lambda k: kern[k][2])
    name, words, ms, gbs = kern[dom]
    iter_us = sum(v[2] for v in kern.values()) * 1e3
    copy_ms = solver.time_kernel(COPY_KERNEL, reps=50)
    copy_bytes = 2 * esz * dof
    log(f"plain copy of {dof} elements: {copy_ms*1e3:.1f} us, {copy_bytes / (copy_ms * 1e-3) / 1e9:.0f} GB/s")
    traffic = counter_traffic(args.dtype, stats["variant"], dom, copy_bytes)
    roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": traffic, "traffic_GBs": traffic / (ms * 1e-3) / 1e9 if traffic else None, "kernel": name,
            "bytes_per_launch": words * esz * dof, "ms_per_launch": ms,
            "copy_GBs": copy_bytes / (copy_ms * 1e-3) / 1e9}

    variants = None
    checks = {}   # GPU results for the oracle check of the cpu_baseline leg
    if eps > 0 and not args.no_variants:
        variants = variant_comparison(pk, solver, prob, u0, tau, (iters[-1], ms_per_step / 1e3), checks)
        variants["traffic_table3"] = traffic_table3(pk)
        variants["advection_cfl4_64x32"] = advection_cfl4(pk)
        variants["fp32_stop_rule"] = fp32_run(pk, checks)
        variants["large_single"] = large_single_sweep(pk)
        variants["one_step_us_per_iteration_f64"] = onestep_us_sweep(pk)
        variants["dg_p2"] = dg_summary(pk, checks)
        variants["batch_256"] = batch_summary(pk, checks)
        variants["differentiable"] = adjoint_summary(pk, checks)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"inviscid Burgers, FD Lax-Friedrichs, BDF2, {NX}x{NT}, T={T_FINAL}, seeded Fourier u0",
            "nx": NX, "nt": NT, "eps": eps, "seed": SEED, "iterations_per_solve": iters[-1],
            "time_to_residual_s": ms_per_step / 1e3 if eps > 0 else None,
            "res_primal": stats["res_primal"], "res_dual": stats["res_dual"], "tau": tau,
            "kernel_sum_us_per_iteration": iter_us, "variant": stats["variant"],
            "us_per_iteration_wall": wall / sum(iters) * 1e6,
            "effective_GBs_all_kernels": sum(w for _, w, _, _ in kern.values()) * esz * dof * sum(iters) / wall / 1e9,
            "variants": variants,
        },
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], err, nw = cpu_baseline(args.cpu_iters, u_final, gpu_iters=iters[-1] if eps > 0 else None)
        out["config"]["error_vs_oracle"] = err
        if variants is not None:
            oracle_checks(checks, variants, nw)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
