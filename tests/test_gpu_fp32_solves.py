"""GPU tests of PF_FP32_SOLVES (double state, force and update; the solves
in float sweeps with double refinement) against the FP64 oracle, through
the C ABI.  Refined to the FP64 parity tolerance the solves leave no trace
of the float sweeps, so the FP64 bar applies."""
import numpy as np
import pytest
import torch

from paper_1202_6116_amd.workloads import PFConfig, Electrode, domain_polarisation

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


def cfg_for(precond, **kw):
    base = dict(nx=64, ny=32, nz=8, precision="fp32_solves", precond=precond, tol_phi=1e-13, tol_u=1e-13,
                phi_bottom=0.1, electrodes=[Electrode(4, 14, 0, 32, 2.0), Electrode(36, 46, 3, 29, -1.5)])
    base.update(kw)
    return PFConfig(**base)


@pytest.mark.parametrize("precond", ["jacobi", "mg"])
def test_fp32_solves_reach_fp64_accuracy(pf, oracle_mod, precond):
    cfg = cfg_for(precond)
    print(f"case: fp32_solves solves {precond}", flush=True)
    P = domain_polarisation(cfg, 81, block=4)
    o = oracle_mod.Oracle(cfg)
    ctx = pf.Context(cfg)
    assert ctx.state_dtype == torch.float64
    phi, st = ctx.solve_phi(dev(P))
    assert st["status"] == 0 and st["relres"] <= 1e-13 and st["outer"] >= 1
    assert rel(host(phi), o.solve_phi(P)[0]) < TOL
    u, st = ctx.solve_u(dev(P))
    assert st["status"] == 0 and st["relres"] <= 1e-13 and st["outer"] >= 1
    assert rel(host(u), o.solve_u(P)[0]) < TOL


@pytest.mark.parametrize("precond,integrator,ws", [("mg", "pc", 2), ("jacobi", "pc", 1), ("mg", "euler", 1)])
def test_fp32_solves_trajectory_matches_oracle(pf, oracle_mod, precond, integrator, ws):
    """Eight steps against the FP64 oracle, every field at the FP64 bar
    (the state stays double, unlike PF_FP32_REFINE's)."""
    cfg = cfg_for(precond, integrator=integrator, warm_start=ws)
    print(f"case: fp32_solves trajectory {precond} {integrator} ws={ws}", flush=True)
    P0 = domain_polarisation(cfg, 82, block=4)
    o = oracle_mod.Oracle(cfg)
    P = P0.copy()
    V, phi, u, _ = o.set_state(P)
    o.step(P, V, phi, u, 8)
    ctx = pf.Context(cfg)
    ctx.set_state(dev(P0))
    st = ctx.step(8)
    assert st["status"] == 0
    Pg, Vg, phig, ug, _ = ctx.get_state()
    errs = {"P": rel(host(Pg), P), "phi": rel(host(phig), phi), "u": rel(host(ug), u)}
    if integrator == "pc":
        errs["V"] = rel(host(Vg), V)
    print("fp32_solves errors vs fp64 oracle:", errs, flush=True)
    for k, v in errs.items():
        assert v < TOL, (k, v)


def test_fp32_solves_adjoint_matches_oracle(pf, oracle_mod):
    """The adjoint of a PF_FP32_SOLVES context runs the FP64 adjoint (double
    state) on the trajectory its refined solves produced."""
    from paper_1202_6116_amd.autograd import tdgl_steps
    cfg = PFConfig(nx=20, ny=9, nz=5, tol_phi=1e-13, tol_u=1e-13, dt=0.05, precision="fp32_solves",
                   Q11=0.5, Q12=-0.15, Q44=0.2,
                   electrodes=[Electrode(2, 6, 0, 9, 1.0), Electrode(12, 16, 0, 9, -1.0)])
    print("case: fp32_solves adjoint", flush=True)
    nsteps = 6
    P0 = domain_polarisation(cfg, 83, block=3, std=0.2)
    wgt = np.zeros((3,) + cfg.shape)
    wgt[2, 2:, 2:6, 3:10] = 1.0 / 3 / 4 / 7
    J_ref, dth_ref, dP_ref = oracle_mod.Oracle(cfg).gradient(P0, nsteps, wgt)
    ctx = pf.Context(cfg)
    P0t = dev(P0).requires_grad_(True)
    volts = torch.tensor([e.volts for e in cfg.electrodes], dtype=torch.float64, requires_grad=True)
    a1 = torch.tensor(cfg.a1, dtype=torch.float64, requires_grad=True)
    PN = tdgl_steps(P0t, volts, a1, ctx, nsteps, checkpoint_every=4)
    J = (PN * dev(wgt)).sum()
    J.backward()
    assert abs(float(J.detach()) - J_ref) <= TOL * abs(J_ref)
    g = np.concatenate([volts.grad.cpu().numpy(), [a1.grad.item()]])
    errs = (rel(g, dth_ref), rel(host(P0t.grad), dP_ref))
    print("adjoint relative errors (dtheta, dJ/dP0):", errs, flush=True)
    assert errs[0] < TOL and errs[1] < TOL, (g, dth_ref)
