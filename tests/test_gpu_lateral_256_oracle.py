"""The 256x256x64 lateral-switching film (the FP64 benchmark leg) at full size
against the FP64 oracle's own run of it: the oracle's states after set-up and
after the first steps, sampled on columns, were written by
tests/golden/make_lateral_512_oracle.py --workload lateral_256x256x64 (which
calls only the oracle); here the GPU path runs the same film from the same
seeded start in the launch configuration of the benchmark leg (multigrid CG,
warm starts extrapolated with the order chosen per refresh) and its states
are compared on the same columns, per field, relative to the field's largest
magnitude over the whole film.

Bars: FP64 and FP32 solves with an FP64 state, 1e-6: both sides solve to a
relative residual of 1e-9 with different preconditioners and initial
guesses (multigrid and extrapolation here, Jacobi and the oracle's
extrapolation there), so two correct solves may differ by up to kappa * 1e-9
with kappa the condition number (up to ~1e3 for these operators), and the
differences propagate into P through dt * F.  FP32 sweeps with FP64
refinement, 1e-4 (the FP32 tolerance of the path's specification)."""
import glob
import json
import os
import re

import numpy as np
import pytest
import torch

from paper_1202_6116_amd.workloads import initial_polarisation, workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
PREFIX = "lateral_256x256x64"


def snapshots():
    out = []
    for f in glob.glob(os.path.join(GOLDEN, f"{PREFIX}_oracle_step*.npz")):
        out.append(int(re.search(r"step(\d+)\.npz$", f).group(1)))
    return sorted(out)


@pytest.fixture(scope="module")
def pf():
    from paper_1202_6116_amd import pf as m
    return m


def sample(t, xs, ys):
    """Columns (xs x ys, every z) of a (..., nz, ny, nx) device field."""
    xs_t = torch.as_tensor(xs, device=t.device)
    ys_t = torch.as_tensor(ys, device=t.device)
    return t.index_select(-2, ys_t).index_select(-1, xs_t).double().cpu().numpy()


BARS = {"fp64": 1e-6, "fp32_solves": 1e-6, "fp32_refine": 1e-4}


@pytest.mark.skipif(not snapshots(), reason="the oracle's samples of the 256x256x64 film are not in tests/golden")
@pytest.mark.parametrize("precision", ["fp64", "fp32_solves", "fp32_refine"])
def test_lateral_256_film_matches_oracle_on_sampled_columns(pf, precision):
    w = workloads()["lateral_256x256x64"]
    cfg = w.cfg.replace(precision=precision, precond="mg", warm_start=3, extrap_order=8)
    steps = snapshots()
    print(f"case: lateral 256x256x64 {precision} vs oracle, snapshots {steps}", flush=True)
    ctx = pf.Context(cfg)
    ctx.set_state(torch.from_numpy(initial_polarisation(w)).to("cuda:0").to(ctx.state_dtype))
    done = 0
    worst = {}
    for n in steps:
        if n > done:
            st = ctx.step(n - done)
            assert st["status"] == 0
            done = n
        ref = np.load(os.path.join(GOLDEN, f"{PREFIX}_oracle_step{n}.npz"))
        meta = json.loads(str(ref["meta"]))
        assert meta["workload"] == w.name
        xs, ys = ref["xs"], ref["ys"]
        P, V, phi, u, step = ctx.get_state()
        assert step == n
        errs = {}
        for k, (name, field) in enumerate((("P", P), ("V", V), ("phi", phi), ("u", u))):
            got = sample(field, xs, ys)
            errs[name] = float(np.abs(got - ref[name]).max() / ref["scale"][k])
            worst[name] = max(worst.get(name, 0.0), errs[name])
        print(f"step {n}: relative errors vs the FP64 oracle {errs}", flush=True)
        for name, e in errs.items():
            assert e < BARS[precision], (n, name, e)
    print(f"{precision}: largest relative errors over the snapshots {worst}", flush=True)
