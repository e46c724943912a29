#!/usr/bin/env python
"""Benchmark of the ETD / embedded-boundary / level-set hot path on one MI355X.

Default workload (ellipsoid192, the largest single-GPU free-boundary
configuration): 3D free boundary on a 192^3 grid over [-10,10]^3, initial
domain the prolate spheroid with semi-axes (3,2,2) (exact signed distance),
u0 ~ U[0.2,0.8] inside (seed 0), beta = 1, mu = 1, logistic f = u(1-u),
ETD2RK with h = 0.01 and adaptive Krylov tolerance 1e-10, level-set
advection by the extended Stefan speed each step and reinitialisation every
5 steps; 50 steps make the whole configuration.

A step is one call of etd_step: level-set sweeps, geometry rebuild and the
two phi-combinations of ETD2RK.  `value` counts box nodes: n^3 times steps
per second (inputs resident in HBM when the clock starts);
`unknown_steps_per_s` counts the computational points (the ODE unknowns)
instead.  The roofline object reports the stencil-Krylov loop (the
persistent Krylov kernel) against the 8 TB/s HBM peak, with algorithmic
bytes counted by the kernel itself and time from HIP events on the stream it
runs on; `roofline_scale` reports the same kernel, measured in the same
process, on the two bandwidth-scale frozen domains (disk4097: 4097^2 disk,
11.6 M unknowns; sphere385: 385^3 ball, 25 M unknowns), where the loop is
bound by HBM rather than by synchronisation latency.  The CPU baseline is
the oracle (plain NumPy/SciPy, test infrastructure) on the first step of
the same workload.

Other workloads (not the headline line): --workload star512 (512^2 star,
200 steps), batch64 (64 random stars advanced by the batched entry points;
value = sum of n^2 over the instances times steps per second), sphere96 (one
gradient of the 96^3 frozen-domain loss: 40 forward steps, checkpointed
backward with the discrete adjoint; value = n^3 times 40 per second of the
whole gradient), batch64_frozen (graph-replayed batched steps), and the
bandwidth-scale frozen-domain runs disk4097 and sphere385 on their own.

Usage: python bench.py [--gpus 1] [--steps 50] [--warmup 5] [--workload ellipsoid192]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs (calibrated on a plain copy; see profiles/), keyed by the
# workload and a hash of the kernel sources they were taken on.  A changed
# kernel has no entry, and its traffic is reported as null.
MEASURED_TRAFFIC = {
    ("ellipsoid192", "909992ad4a5993c4"): 132.94e6,
    ("star512", "909992ad4a5993c4"): 14.86e6,
    ("disk4097", "909992ad4a5993c4"): 24.88e9,
    ("sphere385", "909992ad4a5993c4"): 33.98e9,
}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha1()
    here = os.path.dirname(os.path.abspath(__file__))
    for f in ("paper_2209_15095_amd/csrc/krylov.hip", "paper_2209_15095_amd/csrc/device_common.h"):
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, steps: int, scheme: str):
    """Time the oracle on the first `steps` steps of the same workload (host
    cores), the pieces of each step in the order of
    oracle.freeboundary.free_boundary_step / multistep_step, with a progress
    line after each."""
    import numpy as np

    from oracle.etd import etd_step, logistic
    from oracle.freeboundary import levelset_advance as o_levelset_advance
    from oracle.freeboundary import multistep_step
    from oracle.geometry import Grid
    from oracle.operator import build_operator

    g = Grid(w.grid.dim, tuple(w.grid.n), tuple(w.grid.lo), tuple(w.grid.hi))
    f, _ = logistic(w.a, w.b)
    rho, u, fp = w.rho0.copy(), w.u0.copy(), np.zeros_like(w.u0)
    t0 = time.perf_counter()
    for m in range(steps):
        reinit = (m + 1) % w.reinit_every == 0
        if scheme == "etd2":
            rho, u, fp, _ = multistep_step(g, rho, u, fp, w.h, w.beta, w.mu, w.a, w.b, first=(m == 0),
                                           reinit=reinit, frozen=w.frozen, method="krylov")
            log(f"[bench] cpu baseline: step {m + 1} done ({time.perf_counter() - t0:.1f} s)")
            continue
        if not w.frozen:
            rho, u, _ = o_levelset_advance(g, rho, u, w.h, w.mu, reinit)
            log(f"[bench] cpu baseline: step {m + 1} level set done ({time.perf_counter() - t0:.1f} s)")
        op = build_operator(g, rho, w.beta)
        U = etd_step(op.A, w.h, op.gather(u), f, scheme, method="krylov")
        u = op.scatter(U)
        log(f"[bench] cpu baseline: step {m + 1} ETD done ({time.perf_counter() - t0:.1f} s)")
    dt = time.perf_counter() - t0
    npts = int(np.prod(w.grid.n[: w.grid.dim]))
    return {"value": npts * steps / dt, "unit": "grid-point steps/s", "cores": 1,
            "host_cpus": os.cpu_count(), "kind": "oracle",
            "sample": f"first {steps} of {w.steps} steps of {w.name} ({'frozen' if w.frozen else 'free-boundary'} "
                      f"{scheme.upper()}, level set included), single-threaded NumPy/SciPy, Krylov route for the "
                      f"phi-combinations",
            "seconds": dt}


def roofline_obj(prof, kernel, alg_key="alg_bytes"):
    kern_s = prof["krylov_ms"] * 1e-3
    achieved = prof[alg_key] / kern_s / 1e9 if kern_s > 0 else 0.0
    return {
        "bound": "hbm",
        "kernel": kernel,
        "achieved": achieved,
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": achieved / PEAK_HBM_GBS,
        "alg_bytes_per_launch": prof[alg_key] / max(prof["krylov_launches"], 1),
        "avg_launch_ms": prof["krylov_ms"] / max(prof["krylov_launches"], 1),
    }


def cpu_baseline_batch(ws, steps: int, count: int):
    """Oracle on the first `count` instances for `steps` steps."""
    import numpy as np

    from oracle.freeboundary import free_boundary_step
    from oracle.geometry import Grid

    pts = 0
    t0 = time.perf_counter()
    for w in ws[:count]:
        g = Grid(w.grid.dim, tuple(w.grid.n), tuple(w.grid.lo), tuple(w.grid.hi))
        rho, u = w.rho0.copy(), w.u0.copy()
        for m in range(steps):
            rho, u, _ = free_boundary_step(g, rho, u, w.h, w.beta, w.mu, w.a, w.b, scheme=w.scheme,
                                           reinit=(m + 1) % w.reinit_every == 0, method="krylov")
        pts += int(np.prod(w.grid.n[: w.grid.dim])) * steps
    dt = time.perf_counter() - t0
    return {"value": pts / dt, "unit": "grid-point steps/s", "cores": 1, "host_cpus": os.cpu_count(),
            "kind": "oracle", "seconds": dt,
            "sample": f"first {steps} steps of the first {count} instances, single-threaded NumPy/SciPy"}


def bench_batch(args):
    """The 64 free-boundary instances of batch64: the block and tile schedule
    chosen by the autotuner, then ETD2RK free-boundary steps (reinitialising
    every 5) replayed from recorded HIP graphs whose launch sizes are found
    on the device (the value), with the same steps taken eagerly (one host
    synchronisation per level set and per geometry build) timed beside it."""
    import numpy as np
    import torch

    from paper_2209_15095_amd import inputs
    from paper_2209_15095_amd.api import Batch

    ws = inputs.batch64()
    h = ws[0].h
    every = ws[0].reinit_every
    pts = sum(int(np.prod(w.grid.n[:2])) for w in ws)
    log(f"[bench] batch64: {len(ws)} instances, {pts} grid points, steps {args.steps}")
    b = Batch([w.grid for w in ws], [dict(beta=w.beta, a=w.a, b=w.b, mu=w.mu) for w in ws])
    rho0 = [torch.from_numpy(w.rho0).cuda() for w in ws]
    u0 = [torch.from_numpy(w.u0).cuda() for w in ws]
    rhos = [r.clone() for r in rho0]
    us = [u.clone() for u in u0]

    def reset():
        for r, r0 in zip(rhos, rho0):
            r.copy_(r0)
        for u, v0 in zip(us, u0):
            u.copy_(v0)
        b.geometry_build(rhos)

    def run(n):
        for m in range(n):
            b.step("etd2rk", h, us, rhos, reinit=(m + 1) % every == 0)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    b.geometry_build(rhos)
    tune = b.autotune("etd2rk", h, us, trials=3)
    log(f"[bench] autotune: limit {tune['limit']}, stage_min {tune['stage_min']}")
    run(args.warmup)
    b.sync()
    reset()
    b.profile_enable(True)
    b.profile_read(reset=True)
    t_eager = timed(lambda: run(args.steps))
    b.sync()
    prof = b.profile_read(reset=True)
    # graph replays: recorded on the first call (warm-up), then timed from
    # the initial state
    reset()
    b.graph_free_steps("etd2rk", h, us, rhos, reinit_every=every, step0=0, nsteps=max(args.warmup, 1))
    b.sync()
    reset()
    wall = timed(lambda: b.graph_free_steps("etd2rk", h, us, rhos, reinit_every=every, step0=0,
                                            nsteps=args.steps))
    b.sync()
    b.close()
    out = {
        "metric": "grid-point ETD steps/s at Krylov tol 1e-10",
        "value": pts * args.steps / wall,
        "unit": "grid-point steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / max(args.steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch64", "instances": len(ws), "grid_points": pts,
                   "scheme": "etd2rk", "h": h, "mu": ws[0].mu, "free_boundary": True,
                   "reinit_every": every, "krylov_tol": 1e-10, "graph_replay": True},
        "eager_ms_per_step": 1e3 * t_eager / max(args.steps, 1),
        "autotune": {"group_limit": tune["limit"], "stage_min": tune["stage_min"],
                     "ms_per_launch": {f"{k[0]}/{k[1]}": v for k, v in tune["ms"].items()}},
        "unknown_steps_per_s": prof["n_unknowns"] * args.steps / wall,
        "eager_breakdown_ms_per_step": {k: prof[k + "_ms"] / max(args.steps, 1)
                                        for k in ("krylov", "levelset", "geometry")},
        "roofline": roofline_obj(prof, "krylov_group_kernel<2> (batched persistent ETD2RK step, eager steps)"),
    }
    out["roofline"]["traffic"] = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: oracle on 4 instances x 2 steps")
        out["cpu_baseline"] = cpu_baseline_batch(ws, 2, 4)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    import numpy as np
    import torch

    from paper_2209_15095_amd import inputs
    from paper_2209_15095_amd.api import Context, ETDSolve

    w = inputs.sphere96()
    steps, every = w.steps, w.extra["checkpoint_every"]
    npts = int(np.prod(w.grid.n[:3]))
    ctx = Context.from_grid(w.grid, beta=w.beta, a=w.a, b=w.b, mu=w.mu, tol=1e-10)
    ctx.geometry_build(torch.from_numpy(w.rho0).cuda())
    u0 = torch.from_numpy(w.u0).cuda()

    def grad_once():
        u = u0.clone().requires_grad_(True)
        bt = torch.tensor([w.beta], dtype=torch.float64, device="cuda", requires_grad=True)
        uT = ETDSolve.apply(u, bt, ctx, w.h, steps, every)
        (uT * uT).sum().backward()
        return u.grad, bt.grad

    reps = max(1, args.steps // steps)
    log(f"[bench] sphere96 gradient: {steps} steps, checkpoints every {every}, {reps} repetitions")
    for _ in range(max(1, args.warmup // 5)):
        grad_once()
    ctx.sync()
    ctx.profile_enable(True)
    ctx.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        grad_once()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.close()
    out = {
        "metric": "grid-point ETD steps/s at Krylov tol 1e-10 (gradient: forward + adjoint)",
        "value": npts * steps * reps / wall,
        "unit": "grid-point steps/s",
        "n_gpus": 1, "steps": steps * reps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / (steps * reps),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "sphere96", "grid": list(w.grid.n[:3]), "scheme": "etd2rk", "h": w.h,
                   "steps": steps, "checkpoint_every": every, "free_boundary": False, "krylov_tol": 1e-10},
        "ms_per_gradient": 1e3 * wall / reps,
        "roofline": roofline_obj(prof, "krylov_kernel<3> (forward steps, recomputation, adjoint steps)"),
        "cpu_baseline": None,
    }
    out["roofline"]["traffic"] = None
    print(json.dumps(out), flush=True)


def bench_batch_graph(args):
    """The 64 instances of batch64 with their domains frozen at the initial
    shapes: block schedule chosen by the autotuner, steps replayed from a
    recorded HIP graph (one graph launch per step), eager steps timed
    beside it."""
    import numpy as np
    import torch

    from paper_2209_15095_amd import inputs
    from paper_2209_15095_amd.api import Batch

    ws = inputs.batch64()
    h = ws[0].h
    pts = sum(int(np.prod(w.grid.n[:2])) for w in ws)
    log(f"[bench] batch64_frozen: {len(ws)} instances, {pts} grid points, steps {args.steps}")
    b = Batch([w.grid for w in ws], [dict(beta=w.beta, a=w.a, b=w.b, mu=0.0) for w in ws])
    rhos = [torch.from_numpy(w.rho0).cuda() for w in ws]
    u0 = [torch.from_numpy(w.u0).cuda() for w in ws]
    us = [u.clone() for u in u0]
    b.geometry_build(rhos)
    tune = b.autotune("etd2rk", h, us, trials=3)
    log(f"[bench] autotune: {tune}")

    def reset():
        for u, v in zip(us, u0):
            u.copy_(v)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    for _ in range(args.warmup):
        b.step("etd2rk", h, us)
    reset()
    t_eager = timed(lambda: [b.step("etd2rk", h, us) for _ in range(args.steps)])
    b.sync()
    reset()
    b.graph_steps("etd2rk", h, us, max(args.warmup, 1))
    reset()
    b.profile_enable(True)
    b.profile_read(reset=True)
    wall = timed(lambda: b.graph_steps("etd2rk", h, us, args.steps))
    b.sync()
    prof = b.profile_read()
    b.close()
    out = {
        "metric": "grid-point ETD steps/s at Krylov tol 1e-10",
        "value": pts * args.steps / wall,
        "unit": "grid-point steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / max(args.steps, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch64_frozen", "instances": len(ws), "grid_points": pts,
                   "scheme": "etd2rk", "h": h, "free_boundary": False, "krylov_tol": 1e-10,
                   "graph_replay": True},
        "eager_ms_per_step": 1e3 * t_eager / max(args.steps, 1),
        "autotune": {"group_limit": tune["limit"], "stage_min": tune["stage_min"],
                     "ms_per_launch": {f"{k[0]}/{k[1]}": v for k, v in tune["ms"].items()}},
        "unknown_steps_per_s": prof["n_unknowns"] * args.steps / wall,
        "roofline": roofline_obj(prof, "krylov_group_kernel<2> (graph-replayed step: gather, Krylov, scatter)"),
        "cpu_baseline": None,
    }
    out["roofline"]["traffic"] = None
    # one timed pair spans all graph launches: per-step figures
    out["roofline"]["alg_bytes_per_launch"] = prof["alg_bytes"] / max(args.steps, 1)
    out["roofline"]["avg_launch_ms"] = prof["krylov_ms"] / max(args.steps, 1)
    print(json.dumps(out), flush=True)


def run_single(w, scheme, steps, warmup):
    """Warm-up steps, then `steps` timed steps of workload w from its initial
    state on one context.  Returns (wall seconds, profile, last stats)."""
    import torch

    from paper_2209_15095_amd.api import Context

    ctx = Context.from_grid(w.grid, beta=w.beta, a=w.a, b=w.b, mu=w.mu, tol=1e-10)
    try:
        rho0 = torch.from_numpy(w.rho0).cuda()
        u0 = torch.from_numpy(w.u0).cuda()
        rho = rho0.clone()
        u = u0.clone()
        f_prev = torch.zeros_like(u) if scheme == "etd2" else None

        def run(nsteps):
            for m in range(nsteps):
                reinit = (m + 1) % w.reinit_every == 0
                r = None if w.frozen else rho
                if scheme == "etd2":
                    ctx.multistep_step(w.h, u, f_prev, first=(m == 0), rho=r, reinit=reinit)
                else:
                    ctx.etd_step(scheme, w.h, u, rho=r, reinit=reinit)

        ctx.geometry_build(rho)
        run(warmup)
        ctx.sync()
        # timed run from the initial state
        rho.copy_(rho0)
        u.copy_(u0)
        ctx.geometry_build(rho)
        ctx.profile_enable(True)
        ctx.profile_read(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ctx.sync()
        prof = ctx.profile_read()
        st = ctx.stats()
    finally:
        ctx.close()
    del rho0, u0, rho, u, f_prev
    return wall, prof, st


def krylov_roofline(w, scheme, prof):
    """Roofline object of the persistent Krylov kernel from a profile."""
    kern_s = prof["krylov_ms"] * 1e-3
    achieved = prof["alg_bytes"] / kern_s / 1e9 if kern_s > 0 else 0.0
    return {
        "bound": "hbm",
        "kernel": f"krylov_kernel<{w.grid.dim}> (persistent Lanczos phi-combination / {scheme.upper()} step)",
        "achieved": achieved,
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": achieved / PEAK_HBM_GBS,
        "traffic": MEASURED_TRAFFIC.get((w.name, kernel_source_hash())) if scheme == w.scheme else None,
        "traffic_unit": "bytes per launch",
        "alg_bytes_per_launch": prof["alg_bytes"] / max(prof["krylov_launches"], 1),
        "avg_launch_ms": prof["krylov_ms"] / max(prof["krylov_launches"], 1),
    }


def roofline_scale(steps: int = 2):
    """The Krylov kernel on the bandwidth-scale frozen domains (one warm-up
    step, then `steps` timed steps each)."""
    from paper_2209_15095_amd import inputs

    out = {}
    for name in ("disk4097", "sphere385"):
        w = inputs.WORKLOADS[name]()
        log(f"[bench] roofline scale: {name} ({steps} ETD2RK steps)")
        wall, prof, st = run_single(w, "etd2rk", steps, 1)
        r = krylov_roofline(w, "etd2rk", prof)
        r["n_unknowns"] = prof["n_unknowns"]
        r["ms_per_step"] = 1e3 * wall / steps
        r["m_last"] = st["m_last"]
        out[name] = r
        del w
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: the workload's own count)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ellipsoid192")
    ap.add_argument("--scheme", default=None, choices=["etd1", "etd2", "etd2rk", "etd3rk", "etd4rk"],
                    help="time-stepping scheme (default: the workload's); etd2 is ETD2 multistep")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-scale", action="store_true", help="skip the bandwidth-scale roofline runs")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="MiB: run 3 plain device copies of this size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              f"see DESIGN.md for how the path would shard", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2209_15095_amd import inputs

    if args.workload == "batch64":
        args.steps = args.steps or 100
        return bench_batch(args)
    if args.workload == "batch64_frozen":
        args.steps = args.steps or 100
        return bench_batch_graph(args)
    if args.workload == "sphere96":
        args.steps = args.steps or 40
        return bench_adjoint(args)
    if args.copy_probe > 0:
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = inputs.WORKLOADS[args.workload]()
    steps = args.steps or w.steps
    npts = int(np.prod(w.grid.n[: w.grid.dim]))
    scheme = args.scheme or w.scheme
    log(f"[bench] workload {w.name} grid {w.grid.n[:w.grid.dim]} steps {steps} warmup {args.warmup}")
    wall, prof, st = run_single(w, scheme, steps, args.warmup)
    log(f"[bench] {w.name}: {1e3 * wall / steps:.3f} ms/step")
    n_unknowns = prof["n_unknowns"]
    out = {
        "metric": "grid-point ETD steps/s at Krylov tol 1e-10",
        "value": npts * steps / wall,
        "unit": "grid-point steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "grid": list(w.grid.n[: w.grid.dim]),
            "box": [list(w.grid.lo[: w.grid.dim]), list(w.grid.hi[: w.grid.dim])],
            "scheme": scheme,
            "h": w.h,
            "beta": w.beta,
            "mu": w.mu,
            "free_boundary": not w.frozen,
            "reinit_every": w.reinit_every,
            "krylov_tol": 1e-10,
        },
        "value_counts": "box nodes (n^d) per step; unknown_steps_per_s counts computational points",
        # the unknowns of the last geometry (the domain grows over the run)
        "unknown_steps_per_s": n_unknowns * steps / wall,
        "n_unknowns_final": n_unknowns,
        "breakdown_ms_per_step": {
            "krylov": prof["krylov_ms"] / steps,
            "levelset": prof["levelset_ms"] / steps,
            "geometry": prof["geometry_ms"] / steps,
        },
        "krylov_device_ms_per_step": {
            "whole": prof["krylov_device_ms"] / steps,
            "in_grid_sync": prof["krylov_sync_ms"] / steps,
            "in_expm": prof["krylov_expm_ms"] / steps,
            "in_passes": prof["krylov_pass_ms"] / steps,
            "in_prologue": prof["krylov_prologue_ms"] / steps,
            "after_syncs": prof["krylov_gap_ms"] / steps,
            "other_control": (prof["krylov_device_ms"] - prof["krylov_sync_ms"] - prof["krylov_expm_ms"]
                              - prof["krylov_pass_ms"] - prof["krylov_prologue_ms"]
                              - prof["krylov_gap_ms"]) / steps,
            "syncs": prof["krylov_syncs"] / steps,
            "expms": prof["krylov_expms"] / steps,
        },
        "last_krylov_stats": st,
        "roofline": krylov_roofline(w, scheme, prof),
    }
    if not args.no_scale and w.name == "ellipsoid192" and scheme == w.scheme:
        out["roofline_scale"] = roofline_scale()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline and args.cpu_steps > 0:
        log(f"[bench] cpu baseline: oracle on {args.cpu_steps} step(s)")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, scheme)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
