"""GPU tests of an FP32 + refinement context with the multigrid
preconditioner whose buffers also serve FP64 solves (the adjoint's and the
energy's): forward steps after those solves, and a checkpointed adjoint with
several recomputed segments against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

from paper_1202_6116_amd.workloads import PFConfig, Electrode, domain_polarisation

pytestmark = pytest.mark.gpu


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def dev(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0").to(dtype)


def host(t):
    return t.detach().double().cpu().numpy()


@pytest.fixture(scope="module")
def pf():
    from paper_1202_6116_amd import pf as m
    return m


def cfg_for(top):
    # 64 x 32 x 8: three multigrid levels, so the restriction from a coarse
    # level (whose top plane is fixed with the metal top) runs
    kw = dict(nx=64, ny=32, nz=8, precision="fp32_refine", precond="mg", warm_start=2, tol_phi=1e-10,
              tol_u=1e-10, dt=0.05, Q11=0.5, Q12=-0.15, Q44=0.2,
              electrodes=[Electrode(4, 14, 0, 32, 1.0), Electrode(36, 46, 0, 32, -1.0)])
    if top == "open":
        kw.update(top="open", n_air=3, eps_b=10.0, eps_air=1.0)
    return PFConfig(**kw)


@pytest.mark.parametrize("top", ["metal", "open"])
def test_fp32_forward_after_fp64_solves_is_unchanged(pf, top):
    """An adjoint step and an energy evaluation run FP64 solves in the
    multigrid buffers that the FP32 solves use; the forward steps after them
    give the bits of a context that never ran them."""
    cfg = cfg_for(top)
    print(f"case: fp32 mg forward after fp64 solves, {top} top", flush=True)
    P0 = domain_polarisation(cfg, 91, block=4, std=0.1)
    out = []
    for with_adjoint in (False, True):
        ctx = pf.Context(cfg)
        ctx.set_state(dev(P0, torch.float32))
        ctx.step(2)
        cp = ctx.get_state()
        if with_adjoint:
            lamP = dev(np.full((3,) + cfg.shape, 1e-3), torch.float32)
            lamV = torch.zeros_like(lamP)
            dth = [0.0] * (len(cfg.electrodes) + 1)
            ctx.adjoint_step(cp[0], cp[1], lamP, lamV, dth)
            ctx.energy()
        ctx.restore_state(*cp)
        ctx.step(3)
        out.append([t.clone() for t in ctx.get_state()[:4]])
        del ctx
    for a, b in zip(*out):
        assert torch.isfinite(a).all()
        assert torch.equal(a, b)


def test_fp32_mg_adjoint_with_recomputed_segments_matches_oracle(pf, oracle_mod):
    """Checkpointed adjoint of an FP32 + refinement multigrid context over
    three segments (two recomputed after adjoint steps) against the FP64
    oracle's gradient; the bar is the FP32 adjoint's, 1e-6 relative."""
    from paper_1202_6116_amd.autograd import tdgl_steps
    cfg = cfg_for("metal")
    print("case: fp32 mg adjoint, 3 segments", flush=True)
    nsteps = 6
    P0 = domain_polarisation(cfg, 92, block=4, std=0.2).astype(np.float32).astype(np.float64)
    wgt = np.zeros((3,) + cfg.shape)
    wgt[2, 4:, 8:20, 20:40] = 1.0 / (4 * 12 * 20)
    ocfg = cfg.replace(precision="fp64", precond="jacobi", tol_phi=1e-12, tol_u=1e-12)
    J_ref, dth_ref, dP_ref = oracle_mod.Oracle(ocfg).gradient(P0, nsteps, wgt)
    ctx = pf.Context(cfg)
    P0t = dev(P0, torch.float32).requires_grad_(True)
    volts = torch.tensor([e.volts for e in cfg.electrodes], dtype=torch.float64, requires_grad=True)
    a1 = torch.tensor(cfg.a1, dtype=torch.float64, requires_grad=True)
    PN = tdgl_steps(P0t, volts, a1, ctx, nsteps, checkpoint_every=2)
    J = (PN.double() * dev(wgt)).sum()
    J.backward()
    g = np.concatenate([volts.grad.cpu().numpy(), [a1.grad.item()]])
    errs = (abs(float(J.detach()) - J_ref) / abs(J_ref), rel(g, dth_ref), rel(host(P0t.grad), dP_ref))
    print("fp32 mg adjoint: J, dtheta, dJ/dP0 relative errors", errs, flush=True)
    assert errs[0] < 1e-6 and errs[1] < 1e-6 and errs[2] < 1e-6
