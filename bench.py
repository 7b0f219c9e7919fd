"""Throughput of the TDGL step (Landau + gradient + Poisson PCG + hex8-FEM PCG
+ predictor-corrector) on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

Prints one JSON line: cell-steps/s over K timed steps (inputs resident in
HBM, warm-started solves), the roofline position of the kernel class that
takes the most time (algorithmic bytes per launch / mean launch duration,
HIP events on the library's stream over the timed region), and the FP64
CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TDGL cell-steps/s incl. Poisson+FEM solves; HBM GB/s vs peak; adjoint/fwd ratio"
WARM_START_NAMES = {0: "zero", 1: "previous solution", 2: "extrapolated from earlier solutions"}
HBM_PEAK_GBS = 8000.0

# Algorithmic (compulsory) HBM bytes per node of one launch of each kernel
# class, FP64 state (stencil neighbours counted once as cached re-reads).
#   poisson_setup  P, V (48) + phi (8) read; r, p (16) written
#   poisson_a      r, p_old, x (24) read; p_new, x (16) written
#   poisson_b      p, r (16) read; r (8) written
#   fem_setup      P, V (48) + u (24) read; r, p (48) written
#   fem_a          r, p_old, x (72) read; p_new, x (48) written   (rows k >= 1)
#   fem_b          p, r (48) read; r (24) written                 (rows k >= 1)
#   force          P, V (48) + phi (8) + u (24) read; P, V (48) written
#   mg_u0          FEM multigrid on the solver grid, one residual of the first
#                  sweep (b (24) read, out (24) written) and one last sweep
#                  that forms x from b and the next level's correction
#                  (b (24) + correction (3: level 1 has about 1/8 of the
#                  nodes) read, out (24) written) per V-cycle: 49.5 on
#                  average                                        (rows k >= 1)
#   mg_phi0        the same for the Poisson operator: (16 + 17) / 2 = 16.5
#   finish         x, p read, x written (Poisson 24, FEM 72 per node)
# The Poisson classes run over the potential grid (the film plus, with the
# open top, the air planes), the others over the film.
BYTES_PER_NODE_FP64 = {
    "poisson_setup": 72, "poisson_a": 40, "poisson_b": 24, "fem_setup": 120, "fem_a": 120, "fem_b": 72,
    "force": 128, "mg_u0": 49.5, "mg_phi0": 16.5,
}


# HBM bytes per working launch measured with rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (fetch counts scaled by 2.0, writes by 1.0, from a 1 GiB copy)
# for the current kernels (mg_u0: the mean of its two kernels, the first
# sweep's residual (244.5 MB) and the correction with the last sweep
# (232.8 MB), which run equally often); summary and commands in
# profiles/mg_u0_fp64_lateral_256x256x64.md.  Keyed by workload, precision
# and kernel class; anything else reports null.
MEASURED_TRAFFIC = {
    ("lateral_256x256x64", "fp64", "mg_u0"): 238.6e6,
    ("lateral_256x256x64", "fp64", "fem_a"): 606.1e6,
}


def nodes_per_launch(cls, cfg):
    if cls in ("fem_a", "fem_b", "mg_u0"):
        return cfg.nodes - cfg.nx * cfg.ny
    if cls.startswith("poisson") or cls == "mg_phi0":
        return cfg.nx * cfg.ny * cfg.phi_planes
    return cfg.nodes


def cpu_baseline(w, side=64):
    """The FP64 oracle as it stands, on a bounded sample: one time step (its
    Poisson and FEM solves run to the workload's tolerance by Jacobi CG,
    warm-started from the previous solutions, the paper's warm start; then
    the force and the update) on a side x side x nz slab of the same workload
    after an untimed or_set_state; the time per cell is that of the slab."""
    from oracle.pf_oracle import Oracle
    from paper_1202_6116_amd.workloads import centred_strips, domain_polarisation

    cfg = w.cfg
    sx, sy = min(cfg.nx, side), min(cfg.ny, side)
    scfg = cfg.replace(nx=sx, ny=sy, electrodes=centred_strips(sx, sy) if cfg.electrodes else [],
                       warm_start=1, precision="fp64", precond="jacobi")
    o = Oracle(scfg)
    P = domain_polarisation(scfg, w.seed)
    V, phi, u, _ = o.set_state(P)
    t0 = time.perf_counter()
    st = o.step(P, V, phi, u, 1)
    t_sample = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": scfg.nodes / t_sample, "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
        "sample": (f"one predictor-corrector step of the FP64 oracle (Jacobi CG to tol {cfg.tol_phi:g}/{cfg.tol_u:g}, "
                   f"warm start from the previous solutions: Poisson {st['iters_phi']} it, FEM {st['iters_u']} it) "
                   f"on a {sx}x{sy}x{cfg.nz} slab of the workload, {t_sample:.1f} s; cells/s of the slab"),
        "seconds_sample": round(t_sample, 2),
    }


def adjoint_leg(pf, torch, workloads, initial_polarisation, warm_start, precond):
    """Forward (50 steps, checkpoints every 10) and backward of the adjoint
    case, after one untimed pass of both; returns timings and the gradient."""
    from paper_1202_6116_amd.autograd import tdgl_steps
    w = workloads()["adjoint_128x128x32"]
    cfg = w.cfg.replace(warm_start=warm_start, precond=precond)
    ctx = pf.Context(cfg, "cuda:0")
    P0 = torch.from_numpy(initial_polarisation(w)).to("cuda:0")
    x0, x1, y0, y1, z0, z1 = w.region
    wgt = torch.zeros((3,) + cfg.shape, dtype=torch.float64, device="cuda:0")
    wgt[2, z0:z1, y0:y1, x0:x1] = 1.0 / ((x1 - x0) * (y1 - y0) * (z1 - z0))
    for rep in range(2):  # the first pass is an untimed warm-up; both do the same work
        volts = torch.tensor([e.volts for e in cfg.electrodes], dtype=torch.float64, requires_grad=True)
        a1 = torch.tensor(cfg.a1, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        PN = tdgl_steps(P0, volts, a1, ctx, w.steps, w.checkpoint_every)
        J = (PN * wgt).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    return {"workload": w.name, "steps": w.steps, "checkpoint_every": w.checkpoint_every,
            "forward_s": round(t1 - t0, 3), "backward_s": round(t2 - t1, 3),
            "adjoint_fwd_ratio": round((t2 - t1) / (t1 - t0), 3),
            "dJ_dV": [float(v) for v in volts.grad], "dJ_da1": float(a1.grad)}


def micron_leg(pf, torch, workloads, initial_polarisation, warm_start, precond, steps=5, adj_steps=3, warmup=1):
    """The micron-scale film (1024x1024x96, FP32 sweeps with FP64 refinement):
    forward throughput over `steps` steps, then a differentiable run of
    `adj_steps` steps (one checkpoint segment) and its backward; peak device
    memory of the whole leg.  J is the mean Pz of the film."""
    from paper_1202_6116_amd.autograd import tdgl_steps
    w = workloads()["micron_1024x1024x96_fp32"]
    cfg = w.cfg.replace(warm_start=warm_start, precond=precond)
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    ctx = pf.Context(cfg, "cuda:0")
    P0 = torch.from_numpy(initial_polarisation(w)).to("cuda:0").to(ctx.state_dtype)
    print(f"micron leg: workspace {ctx.ws.numel() / 2**30:.1f} GiB", file=sys.stderr, flush=True)
    ctx.set_state(P0)
    ctx.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ctx.step(steps)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / steps
    print(f"micron leg: forward {1e3 * fwd:.1f} ms/step", file=sys.stderr, flush=True)
    volts = torch.tensor([e.volts for e in cfg.electrodes], dtype=torch.float64, requires_grad=True)
    a1 = torch.tensor(cfg.a1, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    PN = tdgl_steps(P0, volts, a1, ctx, adj_steps, adj_steps)
    J = PN[2].double().mean()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"micron leg: differentiable forward {t1 - t0:.1f} s", file=sys.stderr, flush=True)
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"micron leg: adjoint {t2 - t1:.1f} s", file=sys.stderr, flush=True)
    return {"workload": w.name, "cells": cfg.nodes, "steps": steps, "adjoint_steps": adj_steps,
            "ms_per_step": round(1e3 * fwd, 2), "cell_steps_per_s": cfg.nodes / fwd,
            "cg_iters_per_step": {"phi": st["iters_phi"] / max(1, st["solves_phi"]),
                                  "u": st["iters_u"] / max(1, st["solves_u"])},
            "differentiable_forward_s": round(t1 - t0, 3), "backward_s": round(t2 - t1, 3),
            "adjoint_fwd_ratio": round((t2 - t1) / (t1 - t0), 3),
            "peak_device_GiB": round(torch.cuda.max_memory_allocated() / 2**30, 2),
            "dJ_dV": [float(v) for v in volts.grad], "dJ_da1": float(a1.grad)}


def precision_leg(pf, torch, workloads, initial_polarisation, warm_start, precond, steps=10, warmup=10):
    """The 512x512x128 lateral film for a few steps in FP32 sweeps with FP64
    refinement and in plain FP64 from the same start; returns both step times
    and the per-field relative difference after the steps, and the same for
    plain FP64 with looser solver tolerances (the FP64 path at the final-P
    accuracy that FP32 + refinement reaches)."""
    w = workloads()["lateral_512x512x128_fp32"]
    res = {"workload": w.name, "steps": steps, "warmup": warmup}
    states = {}
    runs = [("fp32_refine", "fp32_refine", None), ("fp64", "fp64", None),
            ("fp64_tol_1e-07", "fp64", 1e-7), ("fp64_tol_1e-06", "fp64", 1e-6)]
    for name, prec, tol in runs:
        cfg = w.cfg.replace(precision=prec, warm_start=warm_start, precond=precond)
        if tol is not None:
            cfg = cfg.replace(tol_phi=tol, tol_u=tol)
        ctx = pf.Context(cfg, "cuda:0")
        P0 = torch.from_numpy(initial_polarisation(w)).to("cuda:0").to(ctx.state_dtype)
        ctx.set_state(P0)
        ctx.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.step(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res[name] = {"ms_per_step": round(1e3 * dt, 2), "cell_steps_per_s": cfg.nodes / dt,
                     "cg_iters_per_step": {"phi": st["iters_phi"] / max(1, st["solves_phi"]),
                                           "u": st["iters_u"] / max(1, st["solves_u"])}}
        P, V, phi, u, _ = ctx.get_state()
        states[name] = [t.double() for t in (P, V, phi, u)]
        del ctx
        torch.cuda.empty_cache()
    res["speedup_fp32_refine_vs_fp64"] = round(res["fp64"]["ms_per_step"] / res["fp32_refine"]["ms_per_step"], 3)
    def rel_diff(run):
        return {field: float((a - b).abs().max() / b.abs().max())
                for field, a, b in zip(("P", "V", "phi", "u"), states[run], states["fp64"])}

    res["rel_diff_vs_fp64"] = rel_diff("fp32_refine")
    for name, _, tol in runs[2:]:
        res[name]["rel_diff_vs_fp64"] = rel_diff(name)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="lateral_256x256x64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--warm-start", type=int, default=2, choices=(0, 1, 2),
                    help="initial guess of each solve: 0 zero, 1 previous solution, 2 extrapolated from the "
                         "last solutions (default 2)")
    ap.add_argument("--extrap-order", type=int, default=None,
                    help="with --warm-start 2: number of earlier solutions the polynomial goes through "
                         "(0..8; default: the workload's)")
    ap.add_argument("--precond", choices=("jacobi", "mg"), default="mg",
                    help="preconditioner of the FEM solves: mg (multigrid V-cycle, default) or jacobi (the paper's)")
    ap.add_argument("--nonlocal-every", type=int, default=None,
                    help="refresh phi and u every k steps (default: the workload's, every step)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="time the steps without per-launch events (the roofline is then omitted)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward timing leg")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP32+refinement vs FP64 leg")
    ap.add_argument("--micron", action="store_true",
                    help="also run the 1024x1024x96 FP32 film: forward throughput, adjoint/forward ratio, peak memory")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy a 1 GiB device buffer 4 times (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only (--gpus 1); the step is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1202_6116_amd import pf
    from paper_1202_6116_amd.workloads import initial_polarisation, workloads

    w = workloads()[args.workload]
    if args.warm_start != w.cfg.warm_start:
        w.cfg = w.cfg.replace(warm_start=args.warm_start)
    if args.extrap_order is not None:
        w.cfg = w.cfg.replace(extrap_order=args.extrap_order)
    if args.nonlocal_every is not None:
        w.cfg = w.cfg.replace(nonlocal_every=args.nonlocal_every)
    w.cfg = w.cfg.replace(precond=args.precond)
    cfg = w.cfg
    dev = torch.device("cuda:0")
    ctx = pf.Context(cfg, "cuda:0")
    P0 = torch.from_numpy(initial_polarisation(w)).to(device=dev, dtype=ctx.state_dtype)
    ctx.set_state(P0)
    if args.warmup:
        ctx.step(args.warmup)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)

    def timed_steps(nsteps, per_launch_events):
        ctx.timing(per_launch_events)       # reset the accumulators; per-launch events on/off
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        st = ctx.step(nsteps)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = ctx.timing(False)
        return max(wall, e0.elapsed_time(e1) / 1e3), st, kt

    def progress(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    # throughput: K steps, no per-launch events
    progress(f"{w.name}: warmup done, timing {args.steps} steps")
    secs, stats, _ = timed_steps(args.steps, False)
    progress(f"{w.name}: {1e3 * secs / args.steps:.1f} ms/step")
    value = cfg.nodes * args.steps / secs

    it_phi = stats["iters_phi"] / max(1, stats["solves_phi"])
    it_u = stats["iters_u"] / max(1, stats["solves_u"])
    out = {
        "metric": METRIC, "value": value, "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * secs / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if cfg.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": [cfg.nx, cfg.ny, cfg.nz], "cells": cfg.nodes,
                   "integrator": cfg.integrator, "tol_phi": cfg.tol_phi, "tol_u": cfg.tol_u,
                   "electrodes": len(cfg.electrodes), "init": w.init, "seed": w.seed,
                   "initial_guess": WARM_START_NAMES[int(cfg.warm_start)],
                   "extrap_order": cfg.extrap_order if cfg.warm_start == 2 else None,
                   "nonlocal_every": max(1, cfg.nonlocal_every), "fem_precond": cfg.precond,
                   "precision": cfg.precision},
        "cg_iters_per_step": {"phi": round(it_phi, 2), "u": round(it_u, 2)},
    }
    if not args.no_kernel_timing:
        # roofline: a second timed region with HIP events around every launch
        # on the library's stream; mean duration of the class taking the most time
        ksteps = max(1, min(args.steps, 10))
        ksecs, _, kt = timed_steps(ksteps, True)
        per = {k: {"ms": round(v[0], 3), "launches": v[1]} for k, v in kt.items() if v[1]}
        dom = max((k for k in BYTES_PER_NODE_FP64 if kt[k][1]), key=lambda k: kt[k][0])
        ms, n = kt[dom]
        avg_s = ms / n / 1e3
        scale = 0.5 if cfg.precision != "fp64" else 1.0
        nbytes = int(BYTES_PER_NODE_FP64[dom] * nodes_per_launch(dom, cfg) * scale)
        achieved = nbytes / avg_s / 1e9
        tot_bytes = scale * sum(BYTES_PER_NODE_FP64[k] * nodes_per_launch(k, cfg) * kt[k][1]
                                for k in BYTES_PER_NODE_FP64)
        tot_ms = sum(v[0] for v in kt.values())
        out["roofline"] = {
            "bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": MEASURED_TRAFFIC.get((w.name, cfg.precision, dom)),
            "bytes_per_launch": nbytes, "avg_launch_us": round(avg_s * 1e6, 2),
            "step_alg_GBps": round(tot_bytes / (tot_ms / 1e3) / 1e9, 1),
            "timed_steps": ksteps, "ms_per_step_with_events": round(1e3 * ksecs / ksteps, 2),
        }
        out["kernel_ms"] = per
    del ctx
    torch.cuda.empty_cache()
    if not args.no_adjoint:
        progress("adjoint leg")
        out["adjoint"] = adjoint_leg(pf, torch, workloads, initial_polarisation, args.warm_start, args.precond)
    if not args.no_precision:
        progress("precision leg")
        out["precision"] = precision_leg(pf, torch, workloads, initial_polarisation, args.warm_start, args.precond)
    if args.micron:
        progress("micron leg")
        try:
            out["micron"] = micron_leg(pf, torch, workloads, initial_polarisation, args.warm_start, args.precond)
        except Exception as e:  # an optional leg: report, keep the main line
            out["micron"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        progress("oracle baseline")
        try:
            out["cpu_baseline"] = cpu_baseline(w)
        except Exception as e:  # the oracle is test infrastructure; report, don't fail the bench
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each": src.numel() * 8, "copies": 4}), flush=True)


if __name__ == "__main__":
    main()
