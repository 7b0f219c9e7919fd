"""Throughput of the TDGL step (Landau + gradient + Poisson PCG + hex8-FEM PCG
+ predictor-corrector) on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-legs] ...

Prints one JSON line.  The headline is the micron-scale film
(1024x1024x96 nodes, FP64, four strip electrodes): cell-steps/s over K
timed steps after W untimed ones, inputs resident in HBM, warm-started
solves.  Alongside it:
  step_roofline  the timed steps' algorithmic HBM bytes (every launch's
                 compulsory reads and writes, counted by the library) over
                 their wall time, against the 8 TB/s peak and the 0.60 target;
  roofline       the kernel class that takes the most time in a second run
                 with HIP events around every launch: its algorithmic bytes
                 per launch over its mean launch duration;
  legs           the 256x256x64 lateral film; the same film as the headline
                 with the Jacobi-preconditioned CG the paper's solver names;
                 precision (FP32 sweeps + FP64 refinement against plain FP64
                 at several tolerances, final-state error against the FP64
                 run); the micron film exactly as the adjoint case asks (100
                 FP32 steps, adjoint with checkpoints every 20); the
                 128x128x32 adjoint case;
  cpu_baseline   the FP64 CPU oracle timed on a bounded sample.
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
WARM_START_NAMES = {0: "zero", 1: "previous solution", 2: "extrapolated from earlier solutions",
                    3: "extrapolated from earlier solutions, order chosen per refresh"}
HBM_PEAK_GBS = 8000.0
# highest extrapolation order of the adaptive warm start (the orders that
# predict best fall from ~8 early in a switching run to ~4 late in it)
ADAPTIVE_MAX_ORDER = 8
TARGET_FRAC = 0.60

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and then
# WRITE_SIZE (KiB per dispatch, scaled by what the same counters read for a
# device-to-device copy of known size), keyed by workload, precision and
# kernel class (the mean over the class's kernels, weighted by launches);
# commands and figures in profiles/.  Anything else reports null.
MEASURED_TRAFFIC = {
    ("micron_1024x1024x96", "fp64", "mg_u0"): 5.143e9,
    ("micron_1024x1024x96_fp32", "fp32_refine", "mg_u0"): 1.918e9,
    ("lateral_512x512x128_fp32", "fp32_refine", "mg_u0"): 0.560e9,
    ("lateral_512x512x128_fp32", "fp32_refine", "mg"): 0.906e9,
}


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def class_table(kt):
    """Per kernel class: time, launches, algorithmic bytes and their rate."""
    out = {}
    for k, (ms, n, nb) in kt.items():
        if not n:
            continue
        row = {"ms": round(ms, 3), "launches": n, "alg_GB": round(nb / 1e9, 3)}
        if ms > 0:
            row["alg_GBps"] = round(nb / (ms / 1e3) / 1e9, 1)
            row["frac"] = round(nb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
        out[k] = row
    return out


def timed_steps(torch, ctx, nsteps, mode):
    """nsteps steps with the library's accounting `mode`; returns the wall
    time (the larger of host clock and stream events), the step statistics
    and the per-class accounting."""
    stream = torch.cuda.current_stream(ctx.device)
    ctx.timing(mode)                    # resets the accumulators
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


def iters(st):
    return {"phi": round(st["iters_phi"] / max(1, st["solves_phi"]), 2),
            "u": round(st["iters_u"] / max(1, st["solves_u"]), 2)}


def measure(pf, torch, w, steps, warmup, events_steps):
    """Sets up the workload, runs `warmup` steps, times `steps` steps with
    byte accounting (solves concurrent), then `events_steps` more with
    per-launch events (solves sequential).  Returns (result dict, context)."""
    from paper_1202_6116_amd.workloads import initial_polarisation
    cfg = w.cfg
    ctx = pf.Context(cfg, "cuda:0")
    P0 = torch.from_numpy(initial_polarisation(w)).to(device="cuda:0", dtype=ctx.state_dtype)
    ctx.set_state(P0)
    del P0
    if warmup:
        ctx.step(warmup)
    torch.cuda.synchronize()
    secs, st, kt = timed_steps(torch, ctx, steps, pf.PF_TIMING_BYTES)
    step_bytes = sum(v[2] for v in kt.values())
    res = {
        "ms_per_step": 1e3 * secs / steps, "cell_steps_per_s": cfg.nodes * steps / secs,
        "cg_iters_per_step": iters(st),
        "step_roofline": {
            "bound": "hbm", "achieved": round(step_bytes / secs / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(step_bytes / secs / 1e9 / HBM_PEAK_GBS, 4), "target_frac": TARGET_FRAC,
            "alg_GB_per_step": round(step_bytes / steps / 1e9, 3), "steps": steps,
        },
    }
    if events_steps:
        esecs, _, ekt = timed_steps(torch, ctx, events_steps, pf.PF_TIMING_EVENTS)
        table = class_table(ekt)
        dom = max(table, key=lambda k: table[k]["ms"])
        ms, n, nb = ekt[dom]
        avg_s = ms / n / 1e3
        achieved = nb / n / avg_s / 1e9
        res["roofline"] = {
            "bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": MEASURED_TRAFFIC.get((w.name, cfg.precision, dom)),
            "bytes_per_launch": int(nb / n), "avg_launch_us": round(avg_s * 1e6, 2),
            "share_of_evented_time": round(ms / sum(v["ms"] for v in table.values()), 3),
            "timed_steps": events_steps, "ms_per_step_with_events": round(1e3 * esecs / events_steps, 2),
        }
        res["kernel_classes"] = table
    return res, ctx


def config_of(w):
    cfg = w.cfg
    return {"workload": w.name, "grid": [cfg.nx, cfg.ny, cfg.nz], "cells": cfg.nodes, "integrator": cfg.integrator,
            "tol_phi": cfg.tol_phi, "tol_u": cfg.tol_u, "electrodes": len(cfg.electrodes), "init": w.init,
            "seed": w.seed, "initial_guess": WARM_START_NAMES[int(cfg.warm_start)],
            "extrap_order": cfg.extrap_order if cfg.warm_start >= 2 else None,
            "nonlocal_every": max(1, cfg.nonlocal_every), "precond": cfg.precond, "precision": cfg.precision}


def cpu_baseline(w, side=48, steps=6, warmup=2):
    """The FP64 oracle as it stands, on a bounded sample: `steps` time steps
    (Poisson and FEM solves to the workload's tolerance by Jacobi CG, the
    oracle's warm start: extrapolated earlier solutions; then the force and
    the update) on a side x side x nz slab of the same workload, after an
    untimed or_set_state and `warmup` untimed steps (so that the
    extrapolation has earlier solutions, as in the GPU's timed window: the
    oracle keeps its solution history within one call, so the sample is the
    time of warmup + steps steps less that of the warmup steps alone, from
    the same state); the time per cell is that of the slab."""
    from oracle.pf_oracle import Oracle
    from paper_1202_6116_amd.workloads import Electrode, domain_polarisation

    cfg = w.cfg
    sx, sy = min(cfg.nx, side), min(cfg.ny, side)
    # two strips 16 nodes wide at +-2 V centred at sx/4 and 3 sx/4, full length in y
    strips = [Electrode(sx // 4 - 8, sx // 4 + 8, 0, sy, 2.0), Electrode(3 * sx // 4 - 8, 3 * sx // 4 + 8, 0, sy, -2.0)]
    # the oracle's own warm starts: the previous solution or its extrapolation
    # of fixed order (order 4 when the GPU run chooses the order per refresh)
    ws = min(int(cfg.warm_start), 2)
    scfg = cfg.replace(nx=sx, ny=sy, electrodes=strips if cfg.electrodes else [], precision="fp64",
                       precond="jacobi", warm_start=ws,
                       extrap_order=4 if int(cfg.warm_start) == 3 else cfg.extrap_order)
    o = Oracle(scfg)
    P = domain_polarisation(scfg, w.seed)
    V, phi, u, _ = o.set_state(P)
    t_warm = 0.0
    if warmup:
        copies = [a.copy() for a in (P, V, phi, u)]
        t0 = time.perf_counter()
        sw = o.step(*copies, warmup)
        t_warm = time.perf_counter() - t0
    t0 = time.perf_counter()
    st = o.step(P, V, phi, u, warmup + steps)
    t_sample = time.perf_counter() - t0 - t_warm
    if warmup:
        st = {k: st[k] - sw[k] for k in ("iters_phi", "iters_u")}
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": scfg.nodes * steps / t_sample, "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
        "sample": (f"{steps} predictor-corrector steps of the FP64 oracle (Jacobi CG to tol {cfg.tol_phi:g}/"
                   f"{cfg.tol_u:g}, warm start {WARM_START_NAMES[int(scfg.warm_start)]}"
                   f"{f' of order {scfg.extrap_order}' if scfg.warm_start == 2 else ''}: Poisson "
                   f"{st['iters_phi']} it, FEM {st['iters_u']} it in all) on a {sx}x{sy}x{cfg.nz} slab of the "
                   f"workload with two strips at sx/4 and 3sx/4, after an untimed set_state and {warmup} untimed "
                   f"steps, {t_sample:.1f} s; cells/s of the slab"),
        "seconds_sample": round(t_sample, 2),
    }


def adjoint_leg(pf, torch, w):
    """Forward (50 steps, checkpoints every 10) and backward of the 128x128x32
    adjoint case, after one untimed pass of both; timings and the gradient."""
    from paper_1202_6116_amd.autograd import tdgl_steps
    from paper_1202_6116_amd.workloads import initial_polarisation
    cfg = w.cfg
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


def micron_adjoint_leg(pf, torch, w):
    """The micron film as the adjoint case asks: a differentiable run of
    w.steps (100) FP32 + refinement steps with checkpoints every
    w.checkpoint_every (20), then the adjoint of J = mean Pz of the film;
    forward and backward times, their ratio and the peak device memory."""
    from paper_1202_6116_amd.autograd import tdgl_steps
    from paper_1202_6116_amd.workloads import initial_polarisation
    cfg = w.cfg
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    ctx = pf.Context(cfg, "cuda:0")
    P0 = torch.from_numpy(initial_polarisation(w)).to("cuda:0").to(ctx.state_dtype)
    progress(f"{w.name}: workspace {ctx.ws.numel() / 2**30:.1f} GiB")
    volts = torch.tensor([e.volts for e in cfg.electrodes], dtype=torch.float64, requires_grad=True)
    a1 = torch.tensor(cfg.a1, dtype=torch.float64, requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    PN = tdgl_steps(P0, volts, a1, ctx, w.steps, w.checkpoint_every)
    J = PN[2].double().mean()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    progress(f"{w.name}: forward of {w.steps} steps {t1 - t0:.1f} s")
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    progress(f"{w.name}: adjoint {t2 - t1:.1f} s")
    out = {"workload": w.name, "cells": cfg.nodes, "steps": w.steps, "checkpoint_every": w.checkpoint_every,
           "forward_s": round(t1 - t0, 3), "forward_cell_steps_per_s": cfg.nodes * w.steps / (t1 - t0),
           "backward_s": round(t2 - t1, 3), "adjoint_fwd_ratio": round((t2 - t1) / (t1 - t0), 3),
           "peak_device_GiB": round(torch.cuda.max_memory_allocated() / 2**30, 2),
           "workspace_GiB": round(ctx.ws.numel() / 2**30, 2),
           "J": float(J.detach()), "dJ_dV": [float(v) for v in volts.grad], "dJ_da1": float(a1.grad)}
    del ctx, PN, J, P0
    torch.cuda.empty_cache()
    return out


def ablation_leg(pf, torch, w, steps=20, warmup=5):
    """The paper's two solver-time ablations on one film, each from the same
    start, `steps` steps timed after `warmup`: the initial guess of the solves
    (zero, the previous step's solution as the paper does, the extrapolation
    of earlier solutions of order 4 and of the order chosen per refresh),
    and the non-local fields refreshed every step or
    every 5 steps with the paper's guess; with the paper's solver (Jacobi
    PCG) and with the multigrid one."""
    from paper_1202_6116_amd.workloads import initial_polarisation
    runs = {}
    for precond in ("jacobi", "mg"):
        for name, kw in (("zero_guess", dict(warm_start=0)), ("previous_solution", dict(warm_start=1)),
                         ("extrapolated", dict(warm_start=2, extrap_order=4)),
                         ("extrapolated_adaptive", dict(warm_start=3, extrap_order=ADAPTIVE_MAX_ORDER)),
                         ("previous_solution_nonlocal_every_5", dict(warm_start=1, nonlocal_every=5))):
            cfg = w.cfg.replace(precond=precond, **kw)
            ctx = pf.Context(cfg, "cuda:0")
            ctx.set_state(torch.from_numpy(initial_polarisation(w)).to(device="cuda:0", dtype=ctx.state_dtype))
            ctx.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.step(steps)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            runs[f"{precond}/{name}"] = {"ms_per_step": round(1e3 * secs / steps, 3), "cg_iters_per_solve": iters(st),
                                        "solves_per_step": round((st["solves_phi"] + st["solves_u"]) / steps, 2)}
            del ctx
    out = {"workload": w.name, "steps": steps, "warmup": warmup, "runs": runs}
    for precond in ("jacobi", "mg"):
        r = {k.split("/", 1)[1]: v["ms_per_step"] for k, v in runs.items() if k.startswith(precond + "/")}
        out[f"{precond}_previous_vs_zero_guess_speedup"] = round(r["zero_guess"] / r["previous_solution"], 2)
        out[f"{precond}_extrapolated_vs_previous_speedup"] = round(r["previous_solution"] / r["extrapolated"], 2)
        out[f"{precond}_adaptive_vs_extrapolated_speedup"] = round(r["extrapolated"] / r["extrapolated_adaptive"], 2)
        out[f"{precond}_nonlocal_every_5_speedup"] = round(
            r["previous_solution"] / r["previous_solution_nonlocal_every_5"], 2)
    torch.cuda.empty_cache()
    return out


def precision_leg(pf, torch, w, steps=10, warmup=5,
                  runs=(("fp64", 1e-9), ("fp64", 1e-7), ("fp64", 1e-6), ("fp64", 1e-5),
                        ("fp32_refine", 1e-9), ("fp32_refine", 1e-7), ("fp32_refine", 1e-6),
                        ("fp32_solves", 1e-9), ("fp32_solves", 1e-7), ("fp32_solves", 1e-6))):
    """One film from the same start in plain FP64, in FP32 sweeps with FP64
    refinement (FP32 state), and with only the solves in FP32 sweeps with
    FP64 refinement (FP64 state), each at several solver tolerances: step
    time over `steps` steps after `warmup`, and the largest difference of
    each field after the run from the FP64 run at tolerance 1e-9, relative
    to that field's largest magnitude (final-P accuracy against cost)."""
    from paper_1202_6116_amd.workloads import initial_polarisation
    res = {"workload": w.name, "steps": steps, "warmup": warmup, "runs": {}}
    ref = None
    for prec, tol in runs:
        cfg = w.cfg.replace(precision=prec, tol_phi=tol, tol_u=tol)
        ctx = pf.Context(cfg, "cuda:0")
        P0 = torch.from_numpy(initial_polarisation(w)).to("cuda:0").to(ctx.state_dtype)
        ctx.set_state(P0)
        del P0
        ctx.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.step(steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        name = f"{prec}_tol_{tol:g}"
        row = {"ms_per_step": round(1e3 * dt, 2), "cell_steps_per_s": cfg.nodes / dt, "cg_iters_per_step": iters(st)}
        state = [t.double() for t in ctx.get_state()[:4]]
        del ctx
        if ref is None:
            ref = state
        else:
            row["rel_diff_vs_fp64_tol_1e-9"] = {
                f: float((a - b).abs().max() / b.abs().max()) for f, a, b in zip(("P", "V", "phi", "u"), state, ref)}
        del state
        torch.cuda.empty_cache()
        res["runs"][name] = row
        progress(f"precision: {name} {row['ms_per_step']} ms/step")
    return res


def main():
    from paper_1202_6116_amd.workloads import workloads as all_workloads
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="micron_1024x1024x96", choices=sorted(all_workloads()))
    ap.add_argument("--warm-start", type=int, default=3, choices=(0, 1, 2, 3),
                    help="initial guess of each solve: 0 zero, 1 previous solution, 2 extrapolated from the "
                         "last solutions, 3 extrapolated with the order chosen per refresh (default 3)")
    ap.add_argument("--extrap-order", type=int, default=None,
                    help="with --warm-start 2 or 3: number of earlier solutions the polynomial goes through, "
                         "for 3 the highest order tried (0..8; default: the workload's for 2, "
                         f"{ADAPTIVE_MAX_ORDER} for 3)")
    ap.add_argument("--precond", choices=("jacobi", "mg"), default="mg",
                    help="preconditioner of both solves: mg (multigrid V-cycle, default) or jacobi (the oracle's)")
    ap.add_argument("--nonlocal-every", type=int, default=None,
                    help="refresh phi and u every k steps (default: the workload's, every step)")
    ap.add_argument("--event-steps", type=int, default=10,
                    help="steps of the per-launch event run that picks the roofline kernel (0: skip)")
    ap.add_argument("--no-legs", action="store_true", help="only the headline (and the CPU baseline)")
    ap.add_argument("--no-lateral", action="store_true", help="skip the 256x256x64 leg")
    ap.add_argument("--no-jacobi", action="store_true", help="skip the Jacobi-PCG leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 128x128x32 adjoint leg")
    ap.add_argument("--no-micron-adjoint", action="store_true", help="skip the 100-step micron adjoint leg")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP32+refinement vs FP64 leg")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the initial-guess and non-local-every-5 ablations on the 256x256x64 film")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy a 1 GiB device buffer 4 times (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only (--gpus 1); the step is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1202_6116_amd import pf

    W = all_workloads()

    def prepared(name, **kw):
        w = W[name]
        cfg = w.cfg.replace(warm_start=args.warm_start, precond=args.precond)
        if args.extrap_order is not None:
            cfg = cfg.replace(extrap_order=args.extrap_order)
        elif args.warm_start == 3:
            cfg = cfg.replace(extrap_order=ADAPTIVE_MAX_ORDER)
        if args.nonlocal_every is not None:
            cfg = cfg.replace(nonlocal_every=args.nonlocal_every)
        w.cfg = cfg.replace(**kw)
        return w

    w = prepared(args.workload)
    progress(f"{w.name}: {args.warmup} warmup steps, then {args.steps} timed")
    head, ctx = measure(pf, torch, w, args.steps, args.warmup, args.event_steps)
    progress(f"{w.name}: {head['ms_per_step']:.1f} ms/step")
    del ctx
    torch.cuda.empty_cache()
    cfg = w.cfg
    out = {
        "metric": METRIC, "value": head["cell_steps_per_s"], "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"fp64": "f64"}.get(cfg.precision, "f32+f64"),
        "data": "synthetic", "config": config_of(w),
    }
    out.update({k: v for k, v in head.items() if k not in ("ms_per_step", "cell_steps_per_s")})
    legs = {}
    if not args.no_legs:
        if not args.no_lateral and w.name != "lateral_256x256x64":
            lw = prepared("lateral_256x256x64")
            progress(f"leg {lw.name}")
            r, c = measure(pf, torch, lw, args.steps, args.warmup, args.event_steps)
            del c
            r.pop("kernel_classes", None)
            legs["lateral"] = {"config": config_of(lw), **r}
        if not args.no_jacobi and args.precond != "jacobi":
            # the paper's solver with the order-4 extrapolation: the adaptive
            # order scores the rough part of the error, which Jacobi-PCG removes
            # fastest, and is slower there
            jw = prepared(args.workload, precond="jacobi", warm_start=2, extrap_order=4)
            progress(f"leg {jw.name} jacobi")
            r, c = measure(pf, torch, jw, 3, 2, 2)
            del c
            torch.cuda.empty_cache()
            legs["jacobi"] = {"config": config_of(jw), **r}
        if not args.no_ablation:
            progress("leg ablations")
            legs["ablations"] = ablation_leg(pf, torch, prepared("lateral_256x256x64"))
        if not args.no_precision:
            progress("leg precision")
            legs["precision"] = precision_leg(pf, torch, prepared("micron_1024x1024x96"))
        if not args.no_micron_adjoint:
            progress("leg micron adjoint")
            try:
                # extrapolation up to order 4: the adjoint's rings of psi and du
                # hold extrap_order solutions each, and the run keeps 100 steps
                # of checkpoints besides
                legs["micron_adjoint"] = micron_adjoint_leg(
                    pf, torch, prepared("micron_1024x1024x96_fp32", extrap_order=4))
            except Exception as e:  # a leg: report, keep the headline
                legs["micron_adjoint"] = {"error": repr(e)}
        if not args.no_adjoint:
            progress("leg adjoint")
            legs["adjoint"] = adjoint_leg(pf, torch, prepared("adjoint_128x128x32"))
    if legs:
        out["legs"] = legs
    if not args.no_cpu_baseline:
        progress("oracle baseline")
        try:
            out["cpu_baseline"] = cpu_baseline(w)
        except Exception as e:  # the oracle is test infrastructure; report, don't fail the bench
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each": src.numel() * 8, "copies": 4}), flush=True)


if __name__ == "__main__":
    main()
