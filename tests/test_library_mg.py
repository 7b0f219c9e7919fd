"""Host checks of the multigrid hierarchy of the FEM operator (no GPU):
level sizes, and the Galerkin stencils against P^T A P formed with scipy
from the assembled fine operator (an independent construction: sparse
matrices instead of probing)."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1202_6116_amd import pf
from paper_1202_6116_amd.workloads import PFConfig, axis_rotation


def tap(o):
    return (o % 3 - 1, (o // 3) % 3 - 1, o // 9 - 1)


def fine_operator(cfg):
    """The FEM operator over the unknowns (planes >= 1) from the stencil
    tables, which the host tests check against the oracle's assembly."""
    T = pf.pf_fem_tables(cfg)["K"]
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    N = nx * ny * nz
    rows, cols, vals = [], [], []
    for k in range(1, nz):
        zt = 1 if k == nz - 1 else 0
        for j in range(ny):
            for i in range(nx):
                n = i + nx * (j + ny * k)
                for o in range(27):
                    dx, dy, dz = tap(o)
                    if not 1 <= k + dz < nz:
                        continue
                    m = (i + dx) % nx + nx * ((j + dy) % ny + ny * (k + dz))
                    for c in range(3):
                        for e in range(3):
                            if T[zt, c, e, o] != 0:
                                rows.append(c * N + n); cols.append(e * N + m); vals.append(T[zt, c, e, o])
    return sp.csr_matrix((vals, (rows, cols)), shape=(3 * N, 3 * N))


def prolongation(nf, nc, periodic):
    P = np.zeros((nf, nc))
    if periodic and nc < nf:
        for i in range(nf):
            if i % 2 == 0:
                P[i, i // 2] = 1
            else:
                P[i, (i - 1) // 2] += 0.5
                P[i, ((i + 1) // 2) % nc] += 0.5
        return P
    if periodic:
        return np.eye(nf)
    zc = list(range(0, nf, 2))
    if zc[-1] != nf - 1:
        zc.append(nf - 1)
    assert len(zc) == nc
    for k in range(nf):
        if k in zc:
            P[k, zc.index(k)] = 1
        else:
            a = max(z for z in zc if z < k)
            b = min(z for z in zc if z > k)
            P[k, zc.index(a)] = (b - k) / (b - a)
            P[k, zc.index(b)] = (k - a) / (b - a)
    return P


@pytest.mark.parametrize("shape,rotation", [((16, 8, 6), None), ((16, 12, 5), axis_rotation((1, 2, 3), 0.7)),
                                            ((18, 14, 8), None), ((9, 13, 7), None)])
def test_level1_galerkin_stencils(shape, rotation):
    nx, ny, nz = shape
    cfg = PFConfig(nx=nx, ny=ny, nz=nz, h=0.9)
    if rotation is not None:
        cfg = cfg.replace(rotation=rotation)
    levels = pf.pf_mg_levels(cfg)
    assert levels[0][0] == shape
    (cx, cy, cz), omega = levels[1]
    assert 0 < omega < 1
    A = fine_operator(cfg)
    Pn = np.kron(prolongation(nz, cz, False), np.kron(prolongation(ny, cy, True), prolongation(nx, cx, True)))
    P = sp.block_diag([sp.csr_matrix(Pn)] * 3).tocsr()
    Ac = (P.T @ A @ P).toarray()
    T = pf.pf_mg_table(cfg, 1)
    Nc = cx * cy * cz
    ref = np.zeros_like(T)
    # read the stencil of every coarse row; rows must be translation invariant
    for k in range(1, cz):
        for c in range(3):
            stencils = []
            for j in range(cy):
                for i in range(cx):
                    r = c * Nc + i + cx * (j + cy * k)
                    s = np.zeros((3, 27))
                    for o in range(27):
                        dx, dy, dz = tap(o)
                        if not 1 <= k + dz < cz:
                            continue
                        m = (i + dx) % cx + cx * ((j + dy) % cy + cy * (k + dz))
                        for e in range(3):
                            s[e, o] = Ac[r, e * Nc + m]
                    stencils.append(s)
            ref[k, c] = stencils[0]
            for s in stencils[1:]:
                np.testing.assert_allclose(s, stencils[0], rtol=0, atol=1e-13)
    np.testing.assert_allclose(T, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    # the clamp plane carries nothing
    assert np.abs(T[0]).max() == 0


def test_hierarchy_of_the_benchmark_film():
    cfg = PFConfig(nx=256, ny=256, nz=64)
    assert [d for d, _ in pf.pf_mg_levels(cfg, "phi")] == [(256, 256, 66), (128, 128, 34), (64, 64, 18), (32, 32, 10),
                                                           (16, 16, 6), (8, 8, 4)]
    dims = [d for d, _ in pf.pf_mg_levels(cfg)]
    assert dims == [(256, 256, 64), (128, 128, 33), (64, 64, 17), (32, 32, 9), (16, 16, 5), (8, 8, 3)]


def oracle_poisson_matrix(oracle_mod, cfg):
    o = oracle_mod.Oracle(cfg)
    M = cfg.nx * cfg.ny * cfg.phi_planes
    A = np.zeros((M, M))
    for t in range(M):
        e = np.zeros(M)
        e[t] = 1
        A[:, t] = o.poisson_apply(e.reshape(cfg.phi_shape)).ravel()
    return A


@pytest.mark.parametrize("kw", [dict(), dict(top="open", n_air=3, eps_b=7.0, eps_air=1.5), dict(h=0.8, eps_b=2.0)])
def test_poisson_levels_match_oracle_and_galerkin(oracle_mod, kw):
    """Level 0 of the Poisson hierarchy is the oracle's operator (stored plane
    k is extended plane k + 1; the ghost planes are fixed), and level 1 is
    P^T A P on the extended grid."""
    cfg = PFConfig(nx=16, ny=12, nz=7, **kw)
    A = oracle_poisson_matrix(oracle_mod, cfg)
    levels = pf.pf_mg_levels(cfg, "phi")
    open_top = cfg.top == "open"
    nze = cfg.phi_planes + 1 + (0 if open_top else 1)
    assert levels[0][0] == (16, 12, nze)
    T0 = pf.pf_mg_table(cfg, 0, "phi")[:, 0, 0, :]
    nx, ny, K = cfg.nx, cfg.ny, cfg.phi_planes
    for k in range(K):
        for (j, i) in ((0, 0), (5, 7), (11, 15)):
            n = i + nx * (j + ny * k)
            s = np.zeros(27)
            for o in range(27):
                dx, dy, dz = tap(o)
                if not 0 <= k + dz < K:
                    continue
                s[o] = A[n, (i + dx) % nx + nx * ((j + dy) % ny + ny * (k + dz))]
            ref = T0[k + 1].copy()
            if k == 0:  # the coupling to the bottom ghost plane is not a matrix entry
                ref[[o for o in range(27) if tap(o)[2] == -1]] = 0
            if k == K - 1:
                ref[[o for o in range(27) if tap(o)[2] == 1]] = 0
            np.testing.assert_allclose(s, ref, rtol=0, atol=1e-13)
    assert np.abs(T0[0]).max() == 0 and (open_top or np.abs(T0[-1]).max() == 0)
    # level 1 by scipy on the extended grid
    (cx, cy, cz), _ = levels[1]
    Pz = prolongation(nze, cz, False)
    top_fixed = not open_top
    fine_rows = list(range(1, nze - (1 if top_fixed else 0)))        # extended planes of the unknowns
    coarse_cols = list(range(1, cz - (1 if top_fixed else 0)))
    Pz = Pz[np.ix_(fine_rows, coarse_cols)]
    P = np.kron(Pz, np.kron(prolongation(ny, cy, True), prolongation(nx, cx, True)))
    Ac = P.T @ A @ P
    T1 = pf.pf_mg_table(cfg, 1, "phi")[:, 0, 0, :]
    nzu = len(coarse_cols)
    for kc in range(nzu):
        for (J, I) in ((0, 0), (3, 5)):
            r = I + cx * (J + cy * kc)
            s = np.zeros(27)
            for o in range(27):
                dx, dy, dz = tap(o)
                if not 0 <= kc + dz < nzu:
                    continue
                s[o] = Ac[r, (I + dx) % cx + cx * ((J + dy) % cy + cy * (kc + dz))]
            ref = T1[kc + 1].copy()
            if kc == 0:
                ref[[o for o in range(27) if tap(o)[2] == -1]] = 0
            if kc == nzu - 1:
                ref[[o for o in range(27) if tap(o)[2] == 1]] = 0
            np.testing.assert_allclose(s, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
