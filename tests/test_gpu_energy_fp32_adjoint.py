"""GPU tests of the free energy, the FP32 + FP64-refinement path and the
discrete adjoint, against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

from paper_1202_6116_amd.workloads import (
    PFConfig, Electrode, TERM_ALL, TERM_LANDAU, TERM_GRAD, TERM_ELEC, TERM_ELAS, workloads, initial_polarisation,
    domain_polarisation, noise_polarisation, random_field,
)

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


def small_cfg(**kw):
    base = dict(nx=70, ny=13, nz=6, tol_phi=1e-13, tol_u=1e-13, phi_bottom=0.1, phi_top=-0.2,
                electrodes=[Electrode(5, 20, 0, 13, 2.0), Electrode(40, 56, 2, 11, -1.5)])
    base.update(kw)
    return PFConfig(**base)


# ---------------------------------------------------------------------------
# Energy
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("terms", [TERM_LANDAU, TERM_GRAD, TERM_ELEC, TERM_ELAS, TERM_ALL])
def test_energy_matches_oracle(pf, oracle_mod, terms):
    cfg = small_cfg(terms=terms, integrator="euler")
    print(f"case: energy terms={terms}", flush=True)
    P = domain_polarisation(cfg, 21, block=4, std=0.1)
    ref = oracle_mod.Oracle(cfg).energy(P, tol=1e-13)
    ctx = pf.Context(cfg)
    ctx.set_state(dev(P))
    e = np.array(ctx.energy())
    scale = np.abs(ref).max()
    assert np.abs(e - ref).max() <= 1e-10 * scale, (e, ref)


def test_energy_decreases_on_gpu_at_zero_bias(pf):
    w = workloads()["film_32x32x8"]
    cfg = w.cfg.replace(integrator="euler")
    ctx = pf.Context(cfg)
    ctx.set_state(dev(noise_polarisation(cfg, 3, std=0.1)))
    prev = ctx.energy()[4]
    for _ in range(10):
        ctx.step(5)
        e = ctx.energy()[4]
        assert e < prev
        prev = e


# ---------------------------------------------------------------------------
# FP32 sweeps + FP64 refinement
# ---------------------------------------------------------------------------

def test_refined_solves_reach_fp64_accuracy(pf, oracle_mod):
    """The FP64 masters of the refined solves satisfy the FP64 tolerance, so
    they agree with the FP64 oracle (given the same, FP32-rounded P) to
    FP64-level accuracy."""
    cfg = small_cfg(precision="fp32_refine", tol_phi=1e-12, tol_u=1e-12)
    print("case: refined solves", flush=True)
    P = domain_polarisation(cfg, 22, block=4).astype(np.float32).astype(np.float64)
    o = oracle_mod.Oracle(cfg.replace(precision="fp64", tol_phi=1e-13, tol_u=1e-13))
    ctx = pf.Context(cfg)
    Pf = dev(P, torch.float32)
    phi, st = ctx.solve_phi(Pf)
    assert st["status"] == 0 and st["relres"] <= 1e-12 and st["outer"] >= 1
    assert rel(host(phi), o.solve_phi(P)[0]) < 1e-9
    u, st = ctx.solve_u(Pf)
    # outer >= 1: the later sweeps form the residual from the stored body force
    assert st["status"] == 0 and st["relres"] <= 1e-12 and st["outer"] >= 1
    assert rel(host(u), o.solve_u(P)[0]) < 1e-9


def test_fp32_trajectory_error_per_field(pf, oracle_mod):
    """FP32 sweeps with FP64 refinement against the FP64 oracle after 20
    steps: relative error per field below 1e-4."""
    cfg = small_cfg(precision="fp32_refine", tol_phi=1e-9, tol_u=1e-9)
    print("case: fp32 trajectory", flush=True)
    P0 = domain_polarisation(cfg, 23, block=4)
    o = oracle_mod.Oracle(cfg.replace(precision="fp64"))
    P = P0.astype(np.float32).astype(np.float64)
    V, phi, u, _ = o.set_state(P)
    o.step(P, V, phi, u, 20)
    ctx = pf.Context(cfg)
    ctx.set_state(dev(P0, torch.float32))
    ctx.step(20)
    Pg, Vg, phig, ug, _ = ctx.get_state()
    errs = {"P": rel(host(Pg), P), "V": rel(host(Vg), V), "phi": rel(host(phig), phi), "u": rel(host(ug), u)}
    print("fp32 errors vs fp64 oracle:", errs, flush=True)
    for k, v in errs.items():
        assert v < 1e-4, (k, v)


# ---------------------------------------------------------------------------
# Adjoint
# ---------------------------------------------------------------------------

def adjoint_cfg(**kw):
    base = dict(nx=20, ny=9, nz=5, tol_phi=1e-13, tol_u=1e-13, dt=0.05,
                electrodes=[Electrode(2, 6, 0, 9, 1.0), Electrode(12, 16, 0, 9, -1.0)],
                Q11=0.5, Q12=-0.15, Q44=0.2)
    base.update(kw)
    return PFConfig(**base)


@pytest.mark.parametrize("integrator,ws", [("pc", 1), ("euler", 1), ("pc", 2)])
def test_adjoint_gradient_matches_oracle(pf, oracle_mod, integrator, ws):
    """warm_start 2 also extrapolates the adjoint solves' initial guesses
    (eight steps fill the rings of order 4)."""
    from paper_1202_6116_amd.autograd import tdgl_steps
    cfg = adjoint_cfg(integrator=integrator, warm_start=ws)
    print(f"case: adjoint {integrator} warm start {ws}", flush=True)
    nsteps = 6 if ws == 1 else 8
    P0 = domain_polarisation(cfg, 31, block=3, std=0.2)
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
    assert abs(float(J.detach()) - J_ref) <= 1e-10 * abs(J_ref)
    g = np.concatenate([volts.grad.cpu().numpy(), [a1.grad.item()]])
    errs = (rel(g, dth_ref), rel(host(P0t.grad), dP_ref))
    print("adjoint relative errors (dtheta, dJ/dP0):", errs, flush=True)
    # both sides solve to a relative residual of 1e-13, so each gradient
    # carries an error of order kappa * 1e-13 (kappa <= 1e3 on these films);
    # measured: 1e-15 .. 1e-14
    assert errs[0] < 1e-10 and errs[1] < 1e-10, (g, dth_ref)


@pytest.mark.parametrize("integrator", ["pc", "euler"])
def test_repeated_backward_is_bitwise_reproducible(pf, integrator):
    """The adjoint warm starts carry within one reverse sweep only: a second
    forward and backward on the same context gives the same gradient bit for
    bit."""
    from paper_1202_6116_amd.autograd import tdgl_steps
    cfg = adjoint_cfg(integrator=integrator, warm_start=2, tol_phi=1e-10, tol_u=1e-10)
    print(f"case: repeated backward {integrator}", flush=True)
    P0 = domain_polarisation(cfg, 33, block=3, std=0.2)
    wgt = dev(np.full((3,) + cfg.shape, 1.0 / (3 * cfg.nx * cfg.ny * cfg.nz)))
    ctx = pf.Context(cfg)
    grads = []
    for _ in range(2):
        P0t = dev(P0).requires_grad_(True)
        volts = torch.tensor([e.volts for e in cfg.electrodes], dtype=torch.float64, requires_grad=True)
        a1 = torch.tensor(cfg.a1, dtype=torch.float64, requires_grad=True)
        PN = tdgl_steps(P0t, volts, a1, ctx, 8, checkpoint_every=3)
        ((PN * PN) * wgt).sum().backward()
        grads.append((host(volts.grad), float(a1.grad), host(P0t.grad)))
    assert np.array_equal(grads[0][0], grads[1][0])
    assert grads[0][1] == grads[1][1]
    assert np.array_equal(grads[0][2], grads[1][2])


def test_fp32_adjoint_gradient_matches_oracle(pf, oracle_mod):
    """The adjoint of an FP32 + refinement context (FP32 state and adjoint
    vectors, FP64 solves) against the FP64 oracle's adjoint gradient: the
    state is rounded to FP32 every step, so the bar is 1e-6 relative
    (measured: 2e-8 for J and the parameters, 1e-7 for dJ/dP0)."""
    from paper_1202_6116_amd.autograd import tdgl_steps
    cfg = adjoint_cfg(precision="fp32_refine", tol_phi=1e-11, tol_u=1e-11)
    print("case: adjoint fp32_refine", flush=True)
    nsteps = 6
    P0 = domain_polarisation(cfg, 32, block=3, std=0.2).astype(np.float32).astype(np.float64)
    wgt = np.zeros((3,) + cfg.shape)
    wgt[2, 2:, 2:6, 3:10] = 1.0 / 3 / 4 / 7
    J_ref, dth_ref, dP_ref = oracle_mod.Oracle(cfg.replace(precision="fp64")).gradient(P0, nsteps, wgt)
    ctx = pf.Context(cfg)
    P0t = dev(P0, torch.float32).requires_grad_(True)
    volts = torch.tensor([e.volts for e in cfg.electrodes], dtype=torch.float64, requires_grad=True)
    a1 = torch.tensor(cfg.a1, dtype=torch.float64, requires_grad=True)
    PN = tdgl_steps(P0t, volts, a1, ctx, nsteps, checkpoint_every=4)
    J = (PN.double() * dev(wgt)).sum()
    J.backward()
    g = np.concatenate([volts.grad.cpu().numpy(), [a1.grad.item()]])
    errs = (abs(float(J.detach()) - J_ref) / abs(J_ref), rel(g, dth_ref), rel(host(P0t.grad), dP_ref))
    print("fp32 adjoint: J, dtheta, dJ/dP0 relative errors", errs, flush=True)
    assert errs[0] < 1e-6 and errs[1] < 1e-6 and errs[2] < 1e-6


def test_adjoint_step_with_forward_displacement(pf):
    """pf_adjoint_step_u, given the displacement each forward step solved
    for, agrees with pf_adjoint_step, which solves for it again (both to
    tolerance 1e-13)."""
    cfg = adjoint_cfg()
    print("case: adjoint step with the forward displacement", flush=True)
    P0 = dev(domain_polarisation(cfg, 33, block=3, std=0.2))
    ctx = pf.Context(cfg)
    ctx.set_state(P0)
    states = []
    for _ in range(6):
        Pn, Vn = [t.clone() for t in ctx.get_state()[:2]]
        ctx.step(1)
        states.append((Pn, Vn, ctx.get_state()[3].clone()))
    rng = np.random.default_rng(5)
    lam0 = dev(rng.normal(size=(3,) + cfg.shape))
    out = []
    # never given, always given, and given on every other step (the solves in
    # between restart the displacement's extrapolation from the given ones)
    for mode in ("none", "all", "mixed"):
        c2 = pf.Context(cfg)
        c2.set_state(P0)
        lamP, lamV = lam0.clone(), torch.zeros_like(lam0)
        dth = [0.0, 0.0, 0.0]
        for t, (Pn, Vn, un) in enumerate(reversed(states)):
            give = mode == "all" or (mode == "mixed" and t % 2 == 0)
            c2.adjoint_step(Pn, Vn, lamP, lamV, dth, un if give else None)
        out.append((host(lamP), host(lamV), np.array(dth)))
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert rel(b, a) < 1e-9


def test_adjoint_full_size_vs_central_differences(pf):
    """The 128x128x32 adjoint case: dJ/dV_1, dJ/dV_2, dJ/da1 of the mean Pz
    over the 32x32x8 box after 50 steps (checkpoint every 10) against
    central differences of the GPU forward (step 1e-6)."""
    from paper_1202_6116_amd.autograd import tdgl_steps
    w = workloads()["adjoint_128x128x32"]
    cfg = w.cfg
    print("case: adjoint_128x128x32", flush=True)
    P0 = dev(initial_polarisation(w))
    x0, x1, y0, y1, z0, z1 = w.region
    wgt = torch.zeros((3,) + cfg.shape, dtype=torch.float64, device="cuda:0")
    wgt[2, z0:z1, y0:y1, x0:x1] = 1.0 / ((x1 - x0) * (y1 - y0) * (z1 - z0))
    ctx = pf.Context(cfg)
    volts = torch.tensor([e.volts for e in cfg.electrodes], dtype=torch.float64, requires_grad=True)
    a1 = torch.tensor(cfg.a1, dtype=torch.float64, requires_grad=True)
    PN = tdgl_steps(P0, volts, a1, ctx, w.steps, w.checkpoint_every)
    J = (PN * wgt).sum()
    J.backward()
    g = [volts.grad[0].item(), volts.grad[1].item(), a1.grad.item()]

    def run(vv, aa):
        ctx.set_params(vv, aa)
        ctx.set_state(P0)
        ctx.step(w.steps)
        return float((ctx.get_state()[0] * wgt).sum())

    d = 1e-6
    base_v = [e.volts for e in cfg.electrodes]
    fd = []
    for e in range(2):
        vp = list(base_v); vp[e] += d
        vm = list(base_v); vm[e] -= d
        fd.append((run(vp, cfg.a1) - run(vm, cfg.a1)) / (2 * d))
    fd.append((run(base_v, cfg.a1 + d) - run(base_v, cfg.a1 - d)) / (2 * d))
    print("adjoint:", g, "central differences:", fd, flush=True)
    for a, b in zip(g, fd):
        assert abs(a - b) <= 1e-5 * max(abs(b), 1e-12) + 1e-9, (g, fd)
