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
    dims = [d for d, _ in pf.pf_mg_levels(cfg)]
    assert dims == [(256, 256, 64), (128, 128, 33), (64, 64, 17), (32, 32, 9), (16, 16, 5), (8, 8, 3)]
