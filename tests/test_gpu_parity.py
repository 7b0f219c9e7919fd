"""GPU (HIP library, through the C ABI) against the FP64 oracle.

FP64 bar: relative error max|gpu - oracle| / max|oracle| <= 1e-10 with both
sides solving to a relative residual of 1e-13 (two correct CG solves differ
by up to about kappa * tol, so the configured tolerances are tightened for
parity).  Grids are chosen to cover several 64 x 4 tiles with ragged edges.
"""
import numpy as np
import pytest
import torch

from paper_1202_6116_amd.workloads import (
    PFConfig, Electrode, TERM_ALL, TERM_LANDAU, TERM_GRAD, TERM_ELEC, TERM_ELAS, workloads, initial_polarisation,
    domain_polarisation, noise_polarisation, random_field,
)

pytestmark = pytest.mark.gpu

TOL = 1e-10


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def pf():
    from paper_1202_6116_amd import pf as m
    return m


def ragged_cfg(**kw):
    base = dict(nx=70, ny=13, nz=6, tol_phi=1e-13, tol_u=1e-13, phi_bottom=0.1, phi_top=-0.2,
                electrodes=[Electrode(5, 20, 0, 13, 2.0), Electrode(40, 56, 2, 11, -1.5)])
    base.update(kw)
    return PFConfig(**base)


def test_poisson_solve_matches_oracle(pf, oracle_mod):
    cfg = ragged_cfg()
    print("case: poisson 70x13x6", flush=True)
    P = domain_polarisation(cfg, 11, block=4)
    ref, it, rr, st = oracle_mod.Oracle(cfg).solve_phi(P)
    ctx = pf.Context(cfg)
    phi, stats = ctx.solve_phi(dev(P))
    assert stats["status"] == 0 and stats["relres"] <= 1e-13
    assert abs(stats["iters"] - it) <= 2
    assert rel(host(phi), ref) < TOL


def test_fem_solve_matches_oracle(pf, oracle_mod):
    cfg = ragged_cfg()
    print("case: fem 70x13x6", flush=True)
    P = domain_polarisation(cfg, 12, block=4)
    ref, it, rr, st = oracle_mod.Oracle(cfg).solve_u(P)
    ctx = pf.Context(cfg)
    u, stats = ctx.solve_u(dev(P))
    assert stats["status"] == 0 and stats["relres"] <= 1e-13
    assert abs(stats["iters"] - it) <= 2
    assert rel(host(u), ref) < TOL
    assert np.all(host(u)[:, 0] == 0)


@pytest.mark.parametrize("terms", [TERM_LANDAU, TERM_GRAD, TERM_ELEC, TERM_ELAS, TERM_ALL])
def test_force_matches_oracle(pf, oracle_mod, terms):
    cfg = ragged_cfg(terms=terms)
    print(f"case: force terms={terms}", flush=True)
    o = oracle_mod.Oracle(cfg)
    P = domain_polarisation(cfg, 13, block=4)
    phi = random_field(cfg.shape, 14)
    u = random_field((3,) + cfg.shape, 15)
    u[:, 0] = 0
    ref = o.force(P, phi, u)
    ctx = pf.Context(cfg)
    F = ctx.force(dev(P), dev(phi), dev(u))
    assert rel(host(F), ref) < 1e-13


@pytest.mark.parametrize("integrator", ["pc", "euler"])
def test_trajectory_matches_oracle_ragged(pf, oracle_mod, integrator):
    cfg = ragged_cfg(integrator=integrator)
    print(f"case: trajectory 70x13x6 {integrator}", flush=True)
    P0 = domain_polarisation(cfg, 16, block=4)
    o = oracle_mod.Oracle(cfg)
    P = P0.copy()
    V, phi, u, _ = o.set_state(P)
    o.step(P, V, phi, u, 10)
    ctx = pf.Context(cfg)
    ctx.set_state(dev(P0))
    stats = ctx.step(10)
    assert stats["status"] == 0 and stats["steps"] == 10
    Pg, Vg, phig, ug, step = ctx.get_state()
    assert step == 10
    assert rel(host(Pg), P) < TOL
    assert rel(host(phig), phi) < TOL
    assert rel(host(ug), u) < TOL
    if integrator == "pc":
        assert rel(host(Vg), V) < TOL


def test_small_film_full_run_matches_oracle(pf, oracle_mod):
    """The 32x32x8 film, 100 predictor-corrector steps (tolerance tightened
    from 1e-10 to 1e-13 for the element-wise comparison)."""
    w = workloads()["film_32x32x8"]
    cfg = w.cfg.replace(tol_phi=1e-13, tol_u=1e-13)
    print("case: film_32x32x8 100 steps", flush=True)
    P0 = initial_polarisation(w)
    o = oracle_mod.Oracle(cfg)
    P = P0.copy()
    V, phi, u, _ = o.set_state(P)
    o.step(P, V, phi, u, w.steps)
    ctx = pf.Context(cfg)
    ctx.set_state(dev(P0))
    ctx.step(w.steps)
    Pg, Vg, phig, ug, _ = ctx.get_state()
    assert rel(host(Pg), P) < TOL
    assert rel(host(Vg), V) < TOL


def test_small_film_at_configured_tolerance(pf, oracle_mod):
    """At the configured CG tolerance 1e-10 the two trajectories are both
    correct solves; they agree to about kappa * tol."""
    w = workloads()["film_32x32x8"]
    cfg = w.cfg
    print("case: film_32x32x8 tol 1e-10", flush=True)
    P0 = initial_polarisation(w)
    o = oracle_mod.Oracle(cfg)
    P = P0.copy()
    V, phi, u, _ = o.set_state(P)
    o.step(P, V, phi, u, 20)
    ctx = pf.Context(cfg)
    ctx.set_state(dev(P0))
    ctx.step(20)
    Pg = host(ctx.get_state()[0])
    assert rel(Pg, P) < 1e-7


def test_zero_polarisation_and_zero_bias(pf):
    """b = 0 on both solves: phi = u = 0 and, with only the Landau term
    vanishing at P = 0, the state stays exactly zero."""
    cfg = PFConfig(nx=16, ny=8, nz=4)
    ctx = pf.Context(cfg)
    P = torch.zeros((3,) + cfg.shape, dtype=torch.float64, device="cuda:0")
    phi, st = ctx.solve_phi(P)
    assert st["iters"] == 0 and float(phi.abs().max()) == 0.0
    u, st = ctx.solve_u(P)
    assert st["iters"] == 0 and float(u.abs().max()) == 0.0
    ctx.set_state(P)
    ctx.step(3)
    assert float(ctx.get_state()[0].abs().max()) == 0.0


def test_minimal_grid(pf, oracle_mod):
    cfg = PFConfig(nx=3, ny=3, nz=3, tol_phi=1e-13, tol_u=1e-13, electrodes=[Electrode(0, 1, 0, 3, 1.0)])
    print("case: 3x3x3", flush=True)
    P0 = noise_polarisation(cfg, 3, std=0.3)
    o = oracle_mod.Oracle(cfg)
    P = P0.copy()
    V, phi, u, _ = o.set_state(P)
    o.step(P, V, phi, u, 5)
    ctx = pf.Context(cfg)
    ctx.set_state(dev(P0))
    ctx.step(5)
    assert rel(host(ctx.get_state()[0]), P) < TOL


def test_iteration_cap_reports_noconv(pf):
    cfg = ragged_cfg(maxit=1)
    ctx = pf.Context(cfg)
    P = dev(domain_polarisation(cfg, 1, block=4))
    phi, st = ctx.solve_phi(P)
    assert st["status"] == pf.PF_ENOCONV and st["iters"] == 1 and st["relres"] > 1e-13


def test_nonfinite_input_is_reported(pf):
    cfg = ragged_cfg()
    ctx = pf.Context(cfg)
    P = domain_polarisation(cfg, 1, block=4)
    P[1, 2, 3, 4] = np.nan
    with pytest.raises(pf.PFError) as ei:
        ctx.solve_phi(dev(P))
    assert ei.value.status == pf.PF_ENONFINITE


def test_bitwise_deterministic_and_resume(pf):
    cfg = ragged_cfg(tol_phi=1e-9, tol_u=1e-9)
    P0 = dev(domain_polarisation(cfg, 5, block=4))
    a = pf.Context(cfg)
    a.set_state(P0)
    a.step(6)
    Pa = a.get_state()[0]
    b = pf.Context(cfg)
    b.set_state(P0)
    b.step(3)
    saved = b.get_state()
    c = pf.Context(cfg)
    c.restore_state(*saved[:4], saved[4])
    c.step(3)
    Pc = c.get_state()[0]
    b.step(3)
    Pb = b.get_state()[0]
    assert torch.equal(Pa, Pb)
    assert torch.equal(Pa, Pc)


def test_sign_symmetry_bitwise(pf):
    els = [Electrode(5, 20, 0, 13, 2.0), Electrode(40, 56, 2, 11, -1.5)]
    cfg = ragged_cfg(phi_bottom=0.0, phi_top=0.0, electrodes=els)
    cfgn = cfg.replace(electrodes=[Electrode(e.x0, e.x1, e.y0, e.y1, -e.volts) for e in els])
    P0 = domain_polarisation(cfg, 7, block=4)
    out = []
    for c, s in ((cfg, 1.0), (cfgn, -1.0)):
        ctx = pf.Context(c)
        ctx.set_state(dev(s * P0))
        ctx.step(4)
        out.append(ctx.get_state())
    assert torch.equal(out[0][0], -out[1][0])
    assert torch.equal(out[0][2], -out[1][2])
    assert torch.equal(out[0][3], out[1][3])


def test_lateral_256_full_size_properties(pf, oracle_mod):
    """The 256x256x64 lateral-switching film in the benchmark's launch
    configuration: the GPU solves satisfy the oracle's own residual test,
    and the GPU force equals the oracle's force evaluated on the GPU's phi
    and u."""
    w = workloads()["lateral_256x256x64"]
    cfg = w.cfg
    print("case: lateral_256x256x64 solves + force", flush=True)
    o = oracle_mod.Oracle(cfg)
    P0 = initial_polarisation(w)
    ctx = pf.Context(cfg)
    Pd = dev(P0)
    phi, st1 = ctx.solve_phi(Pd)
    u, st2 = ctx.solve_u(Pd)
    assert st1["status"] == 0 and st2["status"] == 0
    phi_h, u_h = host(phi), host(u)
    b = o.poisson_rhs(P0)
    r = b - o.poisson_apply(phi_h)
    assert np.linalg.norm(r) <= 1.05 * cfg.tol_phi * np.linalg.norm(b)
    f = o.fem_rhs(P0)
    r = f - o.fem_apply(u_h)
    assert np.linalg.norm(r) <= 1.05 * cfg.tol_u * np.linalg.norm(f)
    F = host(ctx.force(Pd, phi, u))
    ref = o.force(P0, phi_h, u_h)
    assert rel(F, ref) < 1e-12


@pytest.mark.parametrize("order", [0, 2, 5, 8])
def test_extrapolated_warm_start_matches_oracle(pf, oracle_mod, order):
    cfg = ragged_cfg(warm_start=2, extrap_order=order)
    print(f"case: trajectory 70x13x6 extrapolated warm start order {order}", flush=True)
    P0 = domain_polarisation(cfg, 17, block=4)
    o = oracle_mod.Oracle(cfg)
    P = P0.copy()
    V, phi, u, _ = o.set_state(P)
    st_o = o.step(P, V, phi, u, 10)
    ctx = pf.Context(cfg)
    ctx.set_state(dev(P0))
    st_g = ctx.step(10)
    assert abs(st_g["iters_phi"] - st_o["iters_phi"]) <= 10 and abs(st_g["iters_u"] - st_o["iters_u"]) <= 10
    Pg, Vg, phig, ug, _ = ctx.get_state()
    assert rel(host(Pg), P) < TOL
    assert rel(host(phig), phi) < TOL
    assert rel(host(ug), u) < TOL


def test_extrapolation_history_spans_step_calls(pf):
    """The solution history of the extrapolated warm start is kept across
    pf_step calls, so split and single runs agree bitwise; set_state starts
    it afresh."""
    cfg = ragged_cfg(warm_start=2, extrap_order=6, tol_phi=1e-9, tol_u=1e-9)
    P0 = dev(domain_polarisation(cfg, 18, block=4))
    a = pf.Context(cfg)
    a.set_state(P0)
    sa = a.step(12)
    b = pf.Context(cfg)
    b.set_state(P0)
    sb = b.step(5)
    sb2 = b.step(7)
    assert torch.equal(a.get_state()[0], b.get_state()[0])
    assert sa["iters_phi"] == sb["iters_phi"] + sb2["iters_phi"]
    b.set_state(P0)
    sc = b.step(5)
    assert sc["iters_phi"] == sb["iters_phi"] and sc["iters_u"] == sb["iters_u"]


@pytest.mark.parametrize("order,kw", [(1, {}), (4, {}), (8, {}), (8, {"precond": "mg", "precision": "fp32_solves"})])
def test_adaptive_extrapolation_matches_oracle(pf, oracle_mod, order, kw):
    """warm_start 3 chooses the order of each refresh (up to extrap_order)
    by how well each order would have predicted the newest solution from the
    ones before it; only the initial guesses change, so the trajectory
    matches the oracle's (which starts each solve from the previous
    solution) at the parity bar, and the choices depend on the state alone:
    two contexts agree bitwise, a run split over two calls agrees with a
    single one, and set_state starts the history afresh."""
    cfg = ragged_cfg(warm_start=3, extrap_order=order, **kw)
    print(f"case: trajectory 70x13x6 adaptive extrapolation up to order {order} {kw}", flush=True)
    P0 = domain_polarisation(cfg, 19, block=4)
    o = oracle_mod.Oracle(cfg.replace(warm_start=1, precision="fp64", precond="jacobi"))
    P = P0.copy()
    V, phi, u, _ = o.set_state(P)
    o.step(P, V, phi, u, 12)
    a = pf.Context(cfg)
    a.set_state(dev(P0))
    sa = a.step(12)
    Pa, Va, phia, ua, _ = a.get_state()
    assert rel(host(Pa), P) < TOL
    assert rel(host(phia), phi) < TOL
    assert rel(host(ua), u) < TOL
    b = pf.Context(cfg)
    b.set_state(dev(P0))
    sb = b.step(5)
    sb2 = b.step(7)
    for x, y in zip((Pa, Va, phia, ua), b.get_state()[:4]):
        assert torch.equal(x, y)
    assert sa["iters_phi"] == sb["iters_phi"] + sb2["iters_phi"]
    assert sa["iters_u"] == sb["iters_u"] + sb2["iters_u"]
    b.set_state(dev(P0))
    sc = b.step(5)
    assert sc["iters_phi"] == sb["iters_phi"] and sc["iters_u"] == sb["iters_u"]


def test_adaptive_extrapolation_of_order_zero_is_the_previous_solution(pf):
    """With extrap_order 0 there is no order to choose: warm_start 3 gives
    the bits of warm_start 1 (and of warm_start 2 with order 0)."""
    P0 = dev(domain_polarisation(ragged_cfg(), 20, block=4))
    out = []
    for ws in (1, 2, 3):
        ctx = pf.Context(ragged_cfg(warm_start=ws, extrap_order=0))
        ctx.set_state(P0)
        ctx.step(6)
        out.append(ctx.get_state()[:4])
    for other in out[1:]:
        for x, y in zip(out[0], other):
            assert torch.equal(x, y)


@pytest.mark.parametrize("integrator,ws", [("pc", 1), ("euler", 1), ("pc", 2)])
def test_nonlocal_every_k_matches_oracle(pf, oracle_mod, integrator, ws):
    """Non-local fields refreshed every 5 steps (the paper's Fig. 3d
    option): phi and u stay frozen in between while P evolves."""
    cfg = ragged_cfg(integrator=integrator, nonlocal_every=5, warm_start=ws)
    print(f"case: nonlocal_every 5 {integrator} ws={ws}", flush=True)
    P0 = domain_polarisation(cfg, 19, block=4)
    o = oracle_mod.Oracle(cfg)
    P = P0.copy()
    V, phi, u, _ = o.set_state(P)
    st_o = o.step(P, V, phi, u, 13)
    ctx = pf.Context(cfg)
    ctx.set_state(dev(P0))
    st_g = ctx.step(13)
    assert st_g["solves_phi"] == st_o["nsolves_phi"] == 3
    Pg, Vg, phig, ug, _ = ctx.get_state()
    assert rel(host(Pg), P) < TOL
    assert rel(host(phig), phi) < TOL
    assert rel(host(ug), u) < TOL
