"""Writes the FP64 oracle's states of the 512x512x128 lateral-switching film
(sampled columns) for the full-size parity test of the FP32 + refinement path,
or (--workload lateral_256x256x64) those of the 256x256x64 film of the FP64
benchmark leg.

    OMP_NUM_THREADS=8 python tests/golden/make_lateral_512_oracle.py [--steps 1 2 3 4]
    OMP_NUM_THREADS=8 python tests/golden/make_lateral_512_oracle.py --workload lateral_256x256x64 --steps 1 2

Calls only the oracle (oracle/pf_oracle.py) and the seeded input generator.
The film is the one the benchmark's precision leg runs: 512x512x128 nodes,
two centred strip electrodes at +-2 V on the top ghost plane, the seeded
+-<111> domain start (seed 3), predictor-corrector (Eq. 19), both solves to
a relative residual of 1e-9 (Jacobi-preconditioned CG, warm-started by
extrapolating the earlier solutions within each call of the oracle's step).

After or_set_state (the initial rate V0 = F(P0) and its two cold solves) and
after each chunk of steps, the state (P, V, phi, u) is sampled on the
columns x = 8 + 32a, y = 16 + 64b (all z) and written to
lateral_<nx>x<ny>x<nz>_oracle_step<n>.npz together with each field's largest
magnitude over the whole film (the scale the relative errors are quoted
against) and the solver's iteration counts.  The oracle's CG takes about
three seconds per FEM iteration and its FEM right-hand side about two
minutes at this size on eight host cores, so the whole prefix takes hours.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.pf_oracle import Oracle  # noqa: E402
from paper_1202_6116_amd.workloads import initial_polarisation, workloads  # noqa: E402

WORKLOADS = ("lateral_512x512x128_fp32", "lateral_256x256x64")
XS = YS = None
WORKLOAD = PREFIX = None


def sample(a):
    """Columns (XS x YS, every z) of a field shaped (..., nz, ny, nx)."""
    return np.ascontiguousarray(a[..., :, YS, :][..., XS])


def write(step, P, V, phi, u, stats, seconds):
    out = os.path.join(HERE, f"{PREFIX}_oracle_step{step}.npz")
    tmp = out + ".tmp.npz"
    np.savez_compressed(
        tmp, P=sample(P), V=sample(V), phi=sample(phi), u=sample(u), xs=XS, ys=YS,
        scale=np.array([np.abs(P).max(), np.abs(V).max(), np.abs(phi).max(), np.abs(u).max()]),
        step=np.array(step), meta=np.array(json.dumps({"workload": WORKLOAD, "stats": stats,
                                                        "seconds": round(seconds, 1)})))
    os.replace(tmp, out)
    print(f"wrote {out} ({seconds:.0f} s)", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, nargs="*", default=[1, 2, 3, 4],
                    help="chunks of steps; a snapshot is written after each")
    ap.add_argument("--workload", default=WORKLOADS[0], choices=WORKLOADS)
    args = ap.parse_args()
    global XS, YS, WORKLOAD, PREFIX
    WORKLOAD = args.workload
    w = workloads()[WORKLOAD]
    nz, ny, nx = w.cfg.shape
    PREFIX = f"lateral_{nx}x{ny}x{nz}"
    XS = np.arange(8, nx, 32)
    YS = np.arange(16, ny, 64)
    cfg = w.cfg.replace(precision="fp64", precond="jacobi", warm_start=2, maxit=50000)
    o = Oracle(cfg)
    P = initial_polarisation(w)
    t0 = time.time()
    V, phi, u, st = o.set_state(P)
    print(f"set_state: {st}", flush=True)
    write(0, P, V, phi, u, [st], time.time() - t0)
    done, stats = 0, [st]
    for n in args.steps:
        s = o.step(P, V, phi, u, n, done)
        done += n
        stats.append(s)
        print(f"steps {done}: {s}", flush=True)
        write(done, P, V, phi, u, stats, time.time() - t0)


if __name__ == "__main__":
    main()
