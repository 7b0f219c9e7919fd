"""The premise of the full-size GPU checks: the oracle's FEM right-hand
side, FEM operator and force at the inner columns of a window cut out of a
film (with a one-column border, on a small periodic grid) equal the
oracle's results on the whole film."""
import numpy as np

from paper_1202_6116_amd.workloads import Electrode, PFConfig, domain_polarisation, random_field

import test_gpu_full_size as fs


def test_windowed_oracle_equals_whole_film(oracle_mod):
    cfg = PFConfig(nx=64, ny=40, nz=7, electrodes=[Electrode(8, 26, 0, 40, 1.5), Electrode(40, 58, 0, 40, -2.0)],
                   phi_top=0.3, phi_bottom=-0.1)
    o = oracle_mod.Oracle(cfg)
    P = domain_polarisation(cfg, 5, block=4)
    rng = np.random.default_rng(3)
    phi = rng.normal(size=(cfg.phi_planes, cfg.ny, cfg.nx))
    u = rng.normal(size=(3,) + cfg.shape)
    u[:, 0] = 0.0
    f, Ku, F = o.fem_rhs(P), o.fem_apply(u), o.force(P, phi, u)
    for x0, y0, e in fs.windows(cfg):
        els = [Electrode(0, fs.W, 0, fs.W, e.volts)] if e is not None else []
        ow = oracle_mod.Oracle(cfg.replace(nx=fs.W, ny=fs.W, electrodes=els))
        Pw, phiw, uw = fs.cut(P, x0, y0), fs.cut(phi, x0, y0), fs.cut(u, x0, y0)
        for whole, part in ((f, ow.fem_rhs(Pw)), (Ku, ow.fem_apply(uw)), (F, ow.force(Pw, phiw, uw))):
            ref = fs.inner(fs.cut(whole, x0, y0))
            assert np.abs(fs.inner(part) - ref).max() <= 1e-12 * np.abs(ref).max()
