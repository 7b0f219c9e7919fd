"""ctypes access to the FP64 CPU oracle in pf_oracle.c.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use this module.  It never imports the GPU
library, and the GPU library never imports it.

Fields are numpy float64 arrays shaped (3, nz, ny, nx) (stress fields:
(6, nz, ny, nx); scalar fields: (nz, ny, nx)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pf_oracle.c")
LIB = os.path.join(HERE, "libpf_oracle.so")

OK, EINVAL, ENOMEM, ENOCONV, ENONFINITE = 0, -1, -2, -4, -5


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class OrParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("h", ctypes.c_double),
        ("a1", ctypes.c_double), ("a11", ctypes.c_double), ("a12", ctypes.c_double),
        ("G", ctypes.c_double), ("L", ctypes.c_double), ("dt", ctypes.c_double),
        ("eps_b", ctypes.c_double), ("phi_bottom", ctypes.c_double), ("phi_top", ctypes.c_double),
        ("C11", ctypes.c_double), ("C12", ctypes.c_double), ("C44", ctypes.c_double),
        ("Q11", ctypes.c_double), ("Q12", ctypes.c_double), ("Q44", ctypes.c_double),
        ("n_el", ctypes.c_int32),
        ("el_box", ctypes.POINTER(ctypes.c_int32)),
        ("el_volts", ctypes.POINTER(ctypes.c_double)),
        ("integrator", ctypes.c_int32),
        ("maxit", ctypes.c_int32),
        ("tol_phi", ctypes.c_double), ("tol_u", ctypes.c_double),
        ("warm_start", ctypes.c_int32),
        ("terms", ctypes.c_uint32),
        ("nonlocal_every", ctypes.c_int32),
        ("extrap_order", ctypes.c_int32),
        ("noise_sigma", ctypes.c_double),
        ("noise_seed", ctypes.c_uint64),
        ("top_bc", ctypes.c_int32),
        ("n_air", ctypes.c_int32),
        ("eps_air", ctypes.c_double),
        ("misfit", ctypes.c_double * 3),
        ("rot", ctypes.c_double * 9),
        ("Cg", ctypes.c_double * 36),
        ("Qv", ctypes.c_double * 54),
    ]


class OrStats(ctypes.Structure):
    _fields_ = [
        ("iters_phi", ctypes.c_int64), ("iters_u", ctypes.c_int64),
        ("last_iters_phi", ctypes.c_int32), ("last_iters_u", ctypes.c_int32),
        ("relres_phi", ctypes.c_double), ("relres_u", ctypes.c_double),
        ("nsolves_phi", ctypes.c_int32), ("nsolves_u", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER(OrParams)
        d = ctypes.POINTER(ctypes.c_double)
        i32 = ctypes.POINTER(ctypes.c_int32)
        sig = {
            "or_element_stiffness": (None, [P, d]),
            "or_fem_apply": (None, [P, d, d, d]),
            "or_fem_assemble_nodewise": (None, [P, d]),
            "or_fem_assemble_elementwise": (None, [P, d]),
            "or_fem_diagonal": (None, [P, d, d]),
            "or_nodal_eigenstrain": (None, [P, d, d]),
            "or_fem_rhs": (ctypes.c_int, [P, d, d]),
            "or_fem_rhs_e0": (None, [P, d, d]),
            "or_stress_gather": (ctypes.c_int, [P, d, d, d]),
            "or_elastic_energy": (ctypes.c_double, [P, d, d]),
            "or_divergence": (None, [P, d, d]),
            "or_efield": (None, [P, d, ctypes.c_int, d]),
            "or_poisson_apply": (None, [P, d, d]),
            "or_poisson_rhs": (None, [P, d, ctypes.c_int, ctypes.c_int, d]),
            "or_laplacian_neumann": (None, [P, d, d]),
            "or_solve_poisson_parts": (ctypes.c_int, [P, d, ctypes.c_int, ctypes.c_int, d, ctypes.c_double,
                                                      ctypes.c_int, i32, d]),
            "or_solve_phi": (ctypes.c_int, [P, d, d, i32, d]),
            "or_solve_u": (ctypes.c_int, [P, d, d, i32, d]),
            "or_force": (ctypes.c_int, [P, d, d, d, d]),
            "or_set_state": (ctypes.c_int, [P, d, d, d, d, ctypes.POINTER(OrStats)]),
            "or_step": (ctypes.c_int, [P, d, d, d, d, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(OrStats)]),
            "or_energy": (ctypes.c_int, [P, d, ctypes.c_double, d]),
            "or_electrode_field": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_double, d]),
            "or_hvp": (ctypes.c_int, [P, d, d, d, ctypes.c_double, d]),
            "or_dtheta_accumulate": (None, [P, d, d, d, d]),
            "or_adjoint_step": (ctypes.c_int, [P, d, d, d, d, d, ctypes.c_double, d]),
            "or_adjoint_initial_rate": (ctypes.c_int, [P, d, d, d, d, ctypes.c_double, d]),
            "or_top_ghost": (ctypes.c_double, [P, ctypes.c_int, ctypes.c_int]),
            "or_extrapolate": (None, [d, d, ctypes.c_int64, ctypes.c_int, ctypes.c_int]),
            "or_philox4x32_10": (None, [ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                        ctypes.POINTER(ctypes.c_uint32)]),
            "or_noise": (None, [P, ctypes.c_int64, d]),
            "or_prepare": (None, [P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


def _check(st, what, allow_noconv=False):
    if st == OK or (allow_noconv and st == ENOCONV):
        return st
    raise OracleError(st, what)


class Oracle:
    """The oracle bound to one problem description (a workloads.PFConfig)."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.lib = lib()
        boxes = np.array([[e.x0, e.x1, e.y0, e.y1] for e in cfg.electrodes], dtype=np.int32).reshape(-1, 4)
        volts = np.array([e.volts for e in cfg.electrodes], dtype=np.float64)
        self._boxes = np.ascontiguousarray(boxes)
        self._volts = np.ascontiguousarray(volts)
        p = OrParams()
        p.nx, p.ny, p.nz = cfg.nx, cfg.ny, cfg.nz
        for f in ("h", "a1", "a11", "a12", "G", "L", "dt", "eps_b", "phi_bottom", "phi_top",
                  "C11", "C12", "C44", "Q11", "Q12", "Q44", "tol_phi", "tol_u"):
            setattr(p, f, float(getattr(cfg, f)))
        p.n_el = len(cfg.electrodes)
        p.el_box = self._boxes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        p.el_volts = self._volts.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.integrator = 0 if cfg.integrator == "pc" else 1
        p.maxit = cfg.maxit
        p.warm_start = int(cfg.warm_start)
        p.terms = cfg.terms
        p.nonlocal_every = cfg.nonlocal_every
        p.extrap_order = cfg.extrap_order
        p.noise_sigma = cfg.noise_sigma
        p.noise_seed = cfg.noise_seed
        p.top_bc = 1 if cfg.top == "open" else 0
        p.n_air = cfg.n_air
        p.eps_air = cfg.eps_air
        p.misfit[:] = [float(x) for x in cfg.misfit]
        p.rot[:] = [float(x) for x in cfg.rotation]
        self.lib.or_prepare(ctypes.byref(p))
        self.p = p
        self.pp = ctypes.byref(p)
        self.N = cfg.nodes
        self.shape = cfg.shape
        self.phi_shape = cfg.phi_shape

    # --- helpers ---------------------------------------------------------
    def _vec(self, ncomp):
        return np.zeros((ncomp,) + self.shape) if ncomp > 1 else np.zeros(self.shape)

    def _phi(self):
        """A field on the potential grid (the film plus the air planes of the
        open top)."""
        return np.zeros(self.phi_shape)

    @staticmethod
    def _c(a):
        return np.ascontiguousarray(a, dtype=np.float64)

    # --- element and FEM operator ---------------------------------------
    def grid_stiffness(self):
        """The 6x6 Voigt stiffness on the grid axes."""
        return np.array(self.p.Cg[:]).reshape(6, 6)

    def element_stiffness(self):
        Ke = np.zeros((24, 24))
        self.lib.or_element_stiffness(self.pp, _ptr(Ke))
        return Ke

    def fem_apply(self, u):
        Ke = self.element_stiffness()
        out = self._vec(3)
        self.lib.or_fem_apply(self.pp, _ptr(Ke), _ptr(self._c(u)), _ptr(out))
        return out

    def fem_assemble(self, method="nodewise"):
        D = 3 * self.N
        K = np.zeros((D, D))
        fn = self.lib.or_fem_assemble_nodewise if method == "nodewise" else self.lib.or_fem_assemble_elementwise
        fn(self.pp, _ptr(K))
        return K

    def fem_diagonal(self):
        out = self._vec(3)
        self.lib.or_fem_diagonal(self.pp, _ptr(self.element_stiffness()), _ptr(out))
        return out

    def nodal_eigenstrain(self, P):
        out = self._vec(6)
        self.lib.or_nodal_eigenstrain(self.pp, _ptr(self._c(P)), _ptr(out))
        return out

    def fem_rhs(self, P):
        out = self._vec(3)
        _check(self.lib.or_fem_rhs(self.pp, _ptr(self._c(P)), _ptr(out)), "fem_rhs")
        return out

    def fem_rhs_e0(self, e0):
        out = self._vec(3)
        self.lib.or_fem_rhs_e0(self.pp, _ptr(self._c(e0)), _ptr(out))
        return out

    def stress_gather(self, P, u):
        out = self._vec(6)
        _check(self.lib.or_stress_gather(self.pp, _ptr(self._c(P)), _ptr(self._c(u)), _ptr(out)), "stress")
        return out

    def elastic_energy(self, P, u):
        return self.lib.or_elastic_energy(self.pp, _ptr(self._c(P)), _ptr(self._c(u)))

    # --- finite differences ----------------------------------------------
    def divergence(self, P):
        out = self._phi()
        self.lib.or_divergence(self.pp, _ptr(self._c(P)), _ptr(out))
        return out

    def efield(self, phi, with_ghosts=True):
        out = self._vec(3)
        self.lib.or_efield(self.pp, _ptr(self._c(phi)), int(with_ghosts), _ptr(out))
        return out

    def poisson_apply(self, phi):
        out = self._phi()
        self.lib.or_poisson_apply(self.pp, _ptr(self._c(phi)), _ptr(out))
        return out

    def poisson_rhs(self, P, with_P=True, with_bc=True):
        out = self._phi()
        self.lib.or_poisson_rhs(self.pp, _ptr(None if P is None else self._c(P)), int(with_P), int(with_bc),
                                _ptr(out))
        return out

    def laplacian(self, P):
        out = self._vec(3)
        self.lib.or_laplacian_neumann(self.pp, _ptr(self._c(P)), _ptr(out))
        return out

    def top_ghost(self, i, j):
        return self.lib.or_top_ghost(self.pp, i, j)

    # --- solves -------------------------------------------------------------
    def solve_poisson_parts(self, P, with_P, with_bc, tol, phi0=None):
        phi = self._phi() if phi0 is None else self._c(phi0).copy()
        it = ctypes.c_int32()
        rr = ctypes.c_double()
        st = self.lib.or_solve_poisson_parts(self.pp, _ptr(None if P is None else self._c(P)), int(with_P),
                                             int(with_bc), _ptr(phi), tol, int(phi0 is not None),
                                             ctypes.byref(it), ctypes.byref(rr))
        _check(st, "poisson", allow_noconv=True)
        return phi, it.value, rr.value, st

    def solve_phi(self, P, phi0=None):
        """Poisson solve with the boundary values; warm-started from phi0 when
        the configuration asks for warm starts."""
        phi = self._phi() if phi0 is None else self._c(phi0).copy()
        it = ctypes.c_int32()
        rr = ctypes.c_double()
        st = self.lib.or_solve_phi(self.pp, _ptr(self._c(P)), _ptr(phi), ctypes.byref(it), ctypes.byref(rr))
        _check(st, "solve_phi", allow_noconv=True)
        return phi, it.value, rr.value, st

    def solve_u(self, P, u0=None):
        u = self._vec(3) if u0 is None else self._c(u0).copy()
        it = ctypes.c_int32()
        rr = ctypes.c_double()
        st = self.lib.or_solve_u(self.pp, _ptr(self._c(P)), _ptr(u), ctypes.byref(it), ctypes.byref(rr))
        _check(st, "solve_u", allow_noconv=True)
        return u, it.value, rr.value, st

    # --- force, stepping, energy ----------------------------------------
    def force(self, P, phi=None, u=None):
        out = self._vec(3)
        st = self.lib.or_force(self.pp, _ptr(self._c(P)), _ptr(None if phi is None else self._c(phi)),
                               _ptr(None if u is None else self._c(u)), _ptr(out))
        _check(st, "force")
        return out

    def set_state(self, P, phi0=None, u0=None):
        """Returns (V0, phi, u, stats) for the state P (V0 = F(P0) for the
        predictor-corrector, zero for Euler)."""
        P = self._c(P)
        V = self._vec(3)
        phi = self._phi() if phi0 is None else self._c(phi0).copy()
        u = self._vec(3) if u0 is None else self._c(u0).copy()
        s = OrStats()
        st = self.lib.or_set_state(self.pp, _ptr(P), _ptr(V), _ptr(phi), _ptr(u), ctypes.byref(s))
        _check(st, "set_state", allow_noconv=True)
        return V, phi, u, s.as_dict()

    @staticmethod
    def philox(ctr, key):
        """Philox4x32-10 of one counter block: 4 words from 4 counter and 2 key words."""
        c = (ctypes.c_uint32 * 4)(*ctr)
        k = (ctypes.c_uint32 * 2)(*key)
        out = (ctypes.c_uint32 * 4)()
        lib().or_philox4x32_10(c, k, out)
        return [int(x) for x in out]

    def noise(self, step):
        """The standard normal variates xi (3, nz, ny, nx) of the thermal
        noise of a step."""
        xi = self._vec(3)
        self.lib.or_noise(self.pp, step, _ptr(xi))
        return xi

    @staticmethod
    def extrapolate(x, hist, m):
        """The warm-start guess from x and the m newest rows of hist (newest
        first), in place; hist shifts and x becomes its newest row."""
        assert x.dtype == np.float64 and hist.dtype == np.float64 and hist.shape[1:] == x.shape
        lib().or_extrapolate(_ptr(x), _ptr(hist), x.size, m, hist.shape[0])

    def step(self, P, V, phi, u, nsteps, step0=0):
        """Advances (P, V, phi, u) in place by nsteps; returns the stats."""
        for a in (P, V, phi, u):
            assert a.dtype == np.float64 and a.flags.c_contiguous
        s = OrStats()
        st = self.lib.or_step(self.pp, _ptr(P), _ptr(V), _ptr(phi), _ptr(u), nsteps, step0, ctypes.byref(s))
        _check(st, "step", allow_noconv=True)
        d = s.as_dict()
        d["status"] = st
        return d

    def energy(self, P, tol=1e-12):
        out = np.zeros(5)
        st = self.lib.or_energy(self.pp, _ptr(self._c(P)), tol, _ptr(out))
        _check(st, "energy", allow_noconv=True)
        return out

    # --- adjoint -----------------------------------------------------------
    def electrode_fields(self, tol=1e-13):
        n = len(self.cfg.electrodes)
        E = np.zeros((max(n, 1), 3) + self.shape)
        for e in range(n):
            _check(self.lib.or_electrode_field(self.pp, e, tol, _ptr(E[e])), "electrode_field", True)
        return E

    def hvp(self, P, u, lam, tol=1e-13):
        out = self._vec(3)
        st = self.lib.or_hvp(self.pp, _ptr(self._c(P)), _ptr(None if u is None else self._c(u)),
                             _ptr(self._c(lam)), tol, _ptr(out))
        _check(st, "hvp", allow_noconv=True)
        return out

    def adjoint_step(self, Pn, Vn, lamP, lamV, Ebasis, dtheta, tol=1e-13):
        st = self.lib.or_adjoint_step(self.pp, _ptr(self._c(Pn)), _ptr(self._c(Vn)), _ptr(lamP), _ptr(lamV),
                                      _ptr(Ebasis), tol, _ptr(dtheta))
        _check(st, "adjoint_step", allow_noconv=True)

    def adjoint_initial_rate(self, P0, lamP, lamV, Ebasis, dtheta, tol=1e-13):
        st = self.lib.or_adjoint_initial_rate(self.pp, _ptr(self._c(P0)), _ptr(lamP), _ptr(lamV), _ptr(Ebasis),
                                              tol, _ptr(dtheta))
        _check(st, "adjoint_initial_rate", allow_noconv=True)

    def gradient(self, P0, nsteps, weight, tol=1e-13):
        """dJ/dtheta, theta = (V_1..V_nel, a1), for J = sum(weight * P_N) after
        nsteps from P0 (zero initial guesses), by the discrete adjoint with
        every state stored.  Returns (J, dtheta, dJ/dP0)."""
        P = self._c(P0).copy()
        V, phi, u, _ = self.set_state(P)
        states = []
        for n in range(nsteps):
            states.append((P.copy(), V.copy()))
            self.step(P, V, phi, u, 1, n)
        J = float(np.sum(weight * P))
        Eb = self.electrode_fields(tol)
        lamP = self._c(weight).copy()
        lamV = self._vec(3)
        dth = np.zeros(len(self.cfg.electrodes) + 1)
        for n in reversed(range(nsteps)):
            self.adjoint_step(states[n][0], states[n][1], lamP, lamV, Eb, dth, tol)
        self.adjoint_initial_rate(self._c(P0), lamP, lamV, Eb, dth, tol)
        return J, dth, lamP
