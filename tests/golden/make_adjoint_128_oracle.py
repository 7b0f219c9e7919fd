"""Writes the FP64 oracle's gradient of the 128x128x32 adjoint case over a
prefix of its trajectory, for the full-size adjoint parity test.

    OMP_NUM_THREADS=8 python tests/golden/make_adjoint_128_oracle.py [--steps 10]

Calls only the oracle (oracle/pf_oracle.py) and the seeded input generator.
The case is the benchmark's adjoint film: 128x128x32 nodes, strips [16, 32)
at +2 V and [96, 112) at -2 V, the seeded +-<111> domain start (seed 4),
predictor-corrector (Eq. 19), forward solves to 1e-12 (the preset's
tolerance), adjoint solves to 1e-13; J is the mean of Pz over x, y in
[48, 80), k in [24, 32) after `steps` steps.  The oracle's discrete adjoint
(every state stored, no checkpoints) gives dJ/dV_1, dJ/dV_2, dJ/da1 and
dJ/dP0; the file keeps J, dtheta and dJ/dP0 on the columns x = 4 + 8a,
y = 4 + 8b (all planes) with the largest magnitude of dJ/dP0 over the film.
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

WORKLOAD = "adjoint_128x128x32"
XS = np.arange(4, 128, 8)
YS = np.arange(4, 128, 8)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10)
    args = ap.parse_args()
    w = workloads()[WORKLOAD]
    cfg = w.cfg.replace(precision="fp64", precond="jacobi", warm_start=2, maxit=50000)
    x0, x1, y0, y1, z0, z1 = w.region
    wgt = np.zeros((3,) + cfg.shape)
    wgt[2, z0:z1, y0:y1, x0:x1] = 1.0 / ((x1 - x0) * (y1 - y0) * (z1 - z0))
    t0 = time.time()
    J, dth, dP = Oracle(cfg).gradient(initial_polarisation(w), args.steps, wgt, tol=1e-13)
    seconds = time.time() - t0
    out = os.path.join(HERE, f"adjoint_128x128x32_oracle_steps{args.steps}.npz")
    np.savez_compressed(out, J=np.array(J), dtheta=dth, dP0=np.ascontiguousarray(dP[:, :, YS, :][..., XS]),
                        dP0_scale=np.array(np.abs(dP).max()), xs=XS, ys=YS, steps=np.array(args.steps),
                        meta=np.array(json.dumps({"workload": WORKLOAD, "seconds": round(seconds, 1)})))
    print(f"wrote {out}: J {J!r}, dtheta {dth.tolist()}, {seconds:.0f} s", flush=True)


if __name__ == "__main__":
    main()
