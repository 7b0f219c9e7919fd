"""Problem descriptions and seeded synthetic inputs.

This module is shared by the GPU binding's callers (tests, benchmark) and by
the CPU oracle's tests.  It holds configuration values and random-number
draws only -- none of the method's arithmetic -- so that both sides start
from the same arrays without sharing any code that computes the method.

Fields are numpy float64 arrays shaped (3, nz, ny, nx) (component, then z,
y, x with x fastest), i.e. structure-of-arrays in the paper's natural node
numbering (x fastest, then y, then z; Sec. III.B.2).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# term mask bits (which energy contributions enter the force)
TERM_LANDAU = 1
TERM_GRAD = 2
TERM_ELEC = 4
TERM_ELAS = 8
TERM_ALL = TERM_LANDAU | TERM_GRAD | TERM_ELEC | TERM_ELAS


@dataclass
class Electrode:
    """A rectangle of the top ghost plane held at a fixed potential.

    x0..x1 and y0..y1 are half-open node ranges (Sec. III.C: the applied
    field enters as Dirichlet values where electrodes sit).
    """
    x0: int
    x1: int
    y0: int
    y1: int
    volts: float


@dataclass
class PFConfig:
    """One phase-field problem: grid, coefficients, boundary values, solver.

    Coefficients are in reduced units.  Landau a1, a11, a12 (Eq. 1); gradient
    G (Eq. 2-3); mobility L and time step dt (Eq. 7, 19); permittivity eps_b
    (Eq. 18); cubic stiffness C11, C12, C44 (Eq. 13); electrostriction Q11,
    Q12, Q44 (Eq. 15).
    """
    nx: int = 32
    ny: int = 32
    nz: int = 8
    h: float = 1.0
    a1: float = -1.0
    a11: float = 0.5
    a12: float = 0.3
    G: float = 1.0
    L: float = 1.0
    dt: float = 0.01
    eps_b: float = 1.0
    phi_bottom: float = 0.0
    phi_top: float = 0.0
    electrodes: List[Electrode] = field(default_factory=list)
    C11: float = 1.7
    C12: float = 0.8
    C44: float = 0.5
    Q11: float = 0.05
    Q12: float = -0.015
    Q44: float = 0.02
    integrator: str = "pc"          # "pc" (Eq. 19) or "euler"
    precision: str = "fp64"         # "fp64", "fp32_refine" or "fp32_solves" (FP64 state, FP32 refined solves)
    tol_phi: float = 1e-10
    tol_u: float = 1e-10
    maxit: int = 5000
    warm_start: int = 1             # 0 cold, 1 previous solution, 2 extrapolated from earlier solutions,
                                    # 3 extrapolated with the order chosen per refresh (up to extrap_order)
    extrap_order: int = 4           # warm_start 2, 3: polynomial through up to 1 + this many solutions
    noise_sigma: float = 0.0        # thermal noise: one Euler step adds noise_sigma * sqrt(dt) * N(0, 1)
    noise_seed: int = 0             # key of the counter-based noise generator
    terms: int = TERM_ALL
    nonlocal_every: int = 1         # recompute phi and u every k steps
    top: str = "metal"              # "metal": Dirichlet plane above the film; "open": air layers, Neumann top
    n_air: int = 5                  # open top: air planes of the potential grid above the film
    eps_air: float = 1.0            # open top: permittivity of the air planes
    misfit: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # substrate strain: xx, yy, engineering xy
    rotation: Tuple[float, ...] = (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0)  # crystal-to-grid R, row-major
    precond: str = "jacobi"         # FEM solves: "jacobi" (the paper's) or "mg" (multigrid V-cycle)

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def phi_planes(self) -> int:
        """Planes of the potential grid: the film, plus the air when open."""
        return self.nz + (self.n_air if self.top == "open" else 0)

    @property
    def phi_shape(self) -> Tuple[int, int, int]:
        return (self.phi_planes, self.ny, self.nx)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def replace(self, **kw) -> "PFConfig":
        return dataclasses.replace(self, **kw)


# Magnitude of each component at the <111> minimum of the Landau energy for
# the preset coefficients a1 = -1, a11 = 0.5, a12 = 0.3 (p^2 = 0.625).
DOMAIN_AMPLITUDE = 0.7905694150420949


def centred_strips(nx: int, ny: int) -> List[Electrode]:
    """Two strips 16 nodes wide with a 64-node gap, centred in x, full length
    in y: [nx/2-48, nx/2-32) at +2 and [nx/2+32, nx/2+48) at -2."""
    c = nx // 2
    return [Electrode(c - 48, c - 32, 0, ny, 2.0), Electrode(c + 32, c + 48, 0, ny, -2.0)]


def quarter_strips(nx: int, ny: int) -> List[Electrode]:
    """Four strips 16 nodes wide centred at nx/8, 3nx/8, 5nx/8, 7nx/8,
    alternating +2, -2, +2, -2."""
    out = []
    for t, v in zip((1, 3, 5, 7), (2.0, -2.0, 2.0, -2.0)):
        c = t * nx // 8
        out.append(Electrode(c - 8, c + 8, 0, ny, v))
    return out


@dataclass
class Workload:
    name: str
    cfg: PFConfig
    init: str                 # "noise" or "domains"
    steps: int
    seed: int = 0
    checkpoint_every: int = 0
    # x0, x1, y0, y1, z0, z1 of the objective's averaging box (None: whole grid)
    region: Optional[Tuple[int, int, int, int, int, int]] = None


def workloads() -> dict:
    """The five problem sizes: a small film, the lateral-switching film that
    the throughput figure is quoted on, its mixed-precision big brother, the
    adjoint case and the micron-scale film; and the lateral film with the
    open-circuit top."""
    w = {}
    w["film_32x32x8"] = Workload(
        "film_32x32x8", PFConfig(nx=32, ny=32, nz=8, tol_phi=1e-10, tol_u=1e-10), "noise", 100, seed=1)
    w["lateral_256x256x64"] = Workload(
        "lateral_256x256x64",
        PFConfig(nx=256, ny=256, nz=64, electrodes=centred_strips(256, 256), tol_phi=1e-9, tol_u=1e-9),
        "domains", 500, seed=2)
    w["lateral_512x512x128_fp32"] = Workload(
        "lateral_512x512x128_fp32",
        PFConfig(nx=512, ny=512, nz=128, electrodes=centred_strips(512, 512), tol_phi=1e-9, tol_u=1e-9,
                 precision="fp32_refine"),
        "domains", 200, seed=3)
    w["adjoint_128x128x32"] = Workload(
        "adjoint_128x128x32",
        PFConfig(nx=128, ny=128, nz=32, electrodes=[Electrode(16, 32, 0, 128, 2.0), Electrode(96, 112, 0, 128, -2.0)],
                 tol_phi=1e-12, tol_u=1e-12),
        "domains", 50, seed=4, checkpoint_every=10, region=(48, 80, 48, 80, 24, 32))
    # the micron-scale film in plain FP64 (the precision the paper's PETSc
    # solves run in): the largest film that fits one GPU in FP64
    w["micron_1024x1024x96"] = Workload(
        "micron_1024x1024x96",
        PFConfig(nx=1024, ny=1024, nz=96, electrodes=quarter_strips(1024, 1024), tol_phi=1e-9, tol_u=1e-9),
        "domains", 100, seed=5, checkpoint_every=20, region=None)
    w["micron_1024x1024x96_fp32"] = Workload(
        "micron_1024x1024x96_fp32",
        PFConfig(nx=1024, ny=1024, nz=96, electrodes=quarter_strips(1024, 1024), tol_phi=1e-9, tol_u=1e-9,
                 precision="fp32_refine"),
        "domains", 100, seed=5, checkpoint_every=20, region=None)
    # the lateral film with the open-circuit top of the paper's second
    # switching study: five air planes, film/air permittivities 100 / 1
    w["lateral_open_256x256x64"] = Workload(
        "lateral_open_256x256x64",
        PFConfig(nx=256, ny=256, nz=64, electrodes=centred_strips(256, 256), tol_phi=1e-9, tol_u=1e-9,
                 top="open", n_air=5, eps_b=100.0, eps_air=1.0),
        "domains", 500, seed=6)
    return w


def noise_polarisation(cfg: PFConfig, seed: int, std: float = 0.01) -> np.ndarray:
    """P ~ N(0, std^2) per component and node, numpy PCG64 stream `seed`."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, std, size=(3,) + cfg.shape)


def domain_polarisation(cfg: PFConfig, seed: int, block: int = 8, amplitude: float = DOMAIN_AMPLITUDE,
                        std: float = 0.01) -> np.ndarray:
    """Random +-<111> domains on block^3 cells plus N(0, std^2) noise.

    Per block a variant v in [0, 8) is drawn; bit c of v gives the sign of
    component c.  Draw order: all variants (z, y, x block order), then the
    noise field."""
    rng = np.random.default_rng(seed)
    nbz, nby, nbx = (-(-cfg.nz // block), -(-cfg.ny // block), -(-cfg.nx // block))
    v = rng.integers(0, 8, size=(nbz, nby, nbx))
    noise = rng.normal(0.0, std, size=(3,) + cfg.shape)
    vz = np.repeat(np.repeat(np.repeat(v, block, 0), block, 1), block, 2)[:cfg.nz, :cfg.ny, :cfg.nx]
    P = np.empty((3,) + cfg.shape)
    for c in range(3):
        sign = np.where((vz >> c) & 1, 1.0, -1.0)
        P[c] = amplitude * sign + noise[c]
    return P


def initial_polarisation(w: Workload) -> np.ndarray:
    if w.init == "noise":
        return noise_polarisation(w.cfg, w.seed)
    return domain_polarisation(w.cfg, w.seed)


def axis_rotation(axis, angle: float) -> Tuple[float, ...]:
    """Row-major rotation matrix by `angle` (radians) about the unit vector
    along `axis` (Rodrigues' formula), as a PFConfig.rotation value."""
    k = np.asarray(axis, dtype=float)
    k = k / np.linalg.norm(k)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    R = np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * (K @ K)
    return tuple(float(x) for x in R.ravel())


def random_field(shape: Tuple[int, ...], seed: int, scale: float = 1.0) -> np.ndarray:
    """Uniform(-scale, scale) test field."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=shape)
