"""GPU test of pf_init_static, the context whose workspace is the library's
static device array (for callers that cannot allocate device memory),
against a context on a caller-owned workspace, through the C ABI."""
import numpy as np
import pytest
import torch

from paper_1202_6116_amd.workloads import PFConfig, Electrode, domain_polarisation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pf():
    from paper_1202_6116_amd import pf as m
    return m


def run(pf, cfg, P0, static):
    ctx = pf.Context(cfg, static_workspace=static)
    ctx.set_state(torch.from_numpy(P0).to("cuda:0").to(ctx.state_dtype))
    st = ctx.step(4)
    out = [t.clone() for t in ctx.get_state()[:4]]
    energy = ctx.energy()
    ctx.close()
    return out, st, energy


def test_static_workspace_context_matches_caller_workspace(pf):
    """Two static contexts in a row, the second on a smaller film (the
    array keeps the first one's contents), and an FP32 one: each gives the
    bits of a context on a torch-owned workspace (its solves run one after
    the other, and its V-cycles launch their coarse part kernel by kernel
    where the other replays a captured graph: neither changes the results),
    and making one takes no torch memory."""
    cases = [
        PFConfig(nx=64, ny=48, nz=10, precond="mg", warm_start=2, tol_phi=1e-11, tol_u=1e-11,
                 electrodes=[Electrode(6, 18, 0, 48, 2.0), Electrode(38, 50, 0, 48, -2.0)]),
        PFConfig(nx=40, ny=16, nz=6, precond="jacobi", warm_start=1, tol_phi=1e-11, tol_u=1e-11,
                 electrodes=[Electrode(4, 12, 0, 16, 1.0)]),
        PFConfig(nx=32, ny=32, nz=8, precond="mg", precision="fp32_refine", warm_start=2, tol_phi=1e-9,
                 tol_u=1e-9, electrodes=[Electrode(4, 12, 0, 32, 1.0), Electrode(20, 28, 0, 32, -1.0)]),
    ]
    for t, cfg in enumerate(cases):
        print(f"case: static workspace {cfg.nx}x{cfg.ny}x{cfg.nz} {cfg.precond} {cfg.precision}", flush=True)
        P0 = domain_polarisation(cfg, 60 + t, block=4, std=0.1)
        ref, st_ref, e_ref = run(pf, cfg, P0, False)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        ctx = pf.Context(cfg, static_workspace=True)
        assert torch.cuda.memory_allocated() == before
        # one static context per GPU at a time
        with pytest.raises(pf.PFError) as err:
            pf.Context(cfg, static_workspace=True)
        assert err.value.status == pf.PF_ESTATE
        ctx.close()
        got, st, e = run(pf, cfg, P0, True)
        assert st["iters_phi"] == st_ref["iters_phi"] and st["iters_u"] == st_ref["iters_u"]
        for a, b in zip(got, ref):
            assert torch.isfinite(a).all()
            assert torch.equal(a, b)
        assert np.array_equal(np.array(e), np.array(e_ref))
