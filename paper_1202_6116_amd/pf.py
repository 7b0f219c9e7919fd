"""ctypes binding of libpf.so (include/pf.h).

Argument marshalling only: torch supplies device memory and the stream,
every step of the method runs in the library's HIP kernels.  The functions
keep the C names (pf_init, pf_step, pf_solve_phi, pf_solve_u, pf_force,
pf_energy, pf_adjoint_step, ...); `Context` wraps them for convenience.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

from .workloads import PFConfig

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpf.so")

PF_OK, PF_EINVAL, PF_ENOMEM, PF_EHIP, PF_ENOCONV, PF_ENONFINITE, PF_ESTATE = 0, -1, -2, -3, -4, -5, -6
PF_INT_PC, PF_INT_EULER = 0, 1
PF_FP64, PF_FP32_REFINE, PF_FP32_SOLVES = 0, 1, 2
PRECISIONS = {"fp64": PF_FP64, "fp32_refine": PF_FP32_REFINE, "fp32_solves": PF_FP32_SOLVES}
PF_TOP_METAL, PF_TOP_OPEN = 0, 1
PF_PRECOND_JACOBI, PF_PRECOND_MG = 0, 1
PF_TIMING_OFF, PF_TIMING_EVENTS, PF_TIMING_BYTES = 0, 1, 2
KERNEL_CLASSES = ["poisson_setup", "poisson_a", "poisson_b", "fem_setup", "fem_a", "fem_b", "force", "finish",
                  "reduce", "other", "mg", "mg_u0", "mg_phi0"]

# Every symbol declared in include/pf.h.
EXPORTS = [
    "pf_workspace_size", "pf_init", "pf_init_static", "pf_set_state", "pf_restore_state", "pf_get_state", "pf_step",
    "pf_solve_phi", "pf_solve_u", "pf_force", "pf_noise", "pf_energy", "pf_set_params", "pf_adjoint_step",
    "pf_adjoint_step_u",
    "pf_adjoint_initial_rate", "pf_timing", "pf_fem_table_size", "pf_fem_tables", "pf_mg_levels", "pf_mg_table",
    "pf_status_str", "pf_last_error",
    "pf_destroy",
]


class PFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class pf_electrode(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_int32), ("x1", ctypes.c_int32), ("y0", ctypes.c_int32), ("y1", ctypes.c_int32),
                ("volts", ctypes.c_double)]


class pf_config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("h", ctypes.c_double),
        ("a1", ctypes.c_double), ("a11", ctypes.c_double), ("a12", ctypes.c_double),
        ("G", ctypes.c_double), ("L", ctypes.c_double), ("dt", ctypes.c_double),
        ("eps_b", ctypes.c_double), ("phi_bottom", ctypes.c_double), ("phi_top", ctypes.c_double),
        ("n_electrodes", ctypes.c_int32), ("electrodes", ctypes.POINTER(pf_electrode)),
        ("C11", ctypes.c_double), ("C12", ctypes.c_double), ("C44", ctypes.c_double),
        ("Q11", ctypes.c_double), ("Q12", ctypes.c_double), ("Q44", ctypes.c_double),
        ("integrator", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("tol_phi", ctypes.c_double), ("tol_u", ctypes.c_double),
        ("maxit", ctypes.c_int32), ("warm_start", ctypes.c_int32),
        ("terms", ctypes.c_uint32), ("nonlocal_every", ctypes.c_int32),
        ("extrap_order", ctypes.c_int32),
        ("noise_sigma", ctypes.c_double), ("noise_seed", ctypes.c_uint64),
        ("top_bc", ctypes.c_int32), ("n_air", ctypes.c_int32), ("eps_air", ctypes.c_double),
        ("misfit", ctypes.c_double * 3), ("rotation", ctypes.c_double * 9),
        ("precond", ctypes.c_int32),
    ]


class pf_solve_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer", ctypes.c_int32), ("relres", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class pf_step_stats(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int32), ("iters_phi", ctypes.c_int64), ("iters_u", ctypes.c_int64),
        ("last_iters_phi", ctypes.c_int32), ("last_iters_u", ctypes.c_int32),
        ("solves_phi", ctypes.c_int32), ("solves_u", ctypes.c_int32),
        ("relres_phi", ctypes.c_double), ("relres_u", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libpf.so (building it first only if it is absent)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build()
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        cfgp = ctypes.POINTER(pf_config)
        dp = ctypes.POINTER(ctypes.c_double)
        sig = {
            "pf_workspace_size": (ctypes.c_int, [cfgp, ctypes.POINTER(sz)]),
            "pf_init": (ctypes.c_int, [cfgp, vp, sz, vp, ctypes.POINTER(vp)]),
            "pf_init_static": (ctypes.c_int, [cfgp, vp, ctypes.POINTER(vp)]),
            "pf_set_state": (ctypes.c_int, [vp, vp, vp, vp]),
            "pf_restore_state": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.c_int64]),
            "pf_get_state": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int64)]),
            "pf_step": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(pf_step_stats)]),
            "pf_solve_phi": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(pf_solve_stats)]),
            "pf_solve_u": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(pf_solve_stats)]),
            "pf_force": (ctypes.c_int, [vp, vp, vp, vp, vp]),
            "pf_noise": (ctypes.c_int, [vp, ctypes.c_int64, vp]),
            "pf_energy": (ctypes.c_int, [vp, dp]),
            "pf_set_params": (ctypes.c_int, [vp, dp, ctypes.c_double]),
            "pf_adjoint_step": (ctypes.c_int, [vp, vp, vp, vp, vp, dp]),
            "pf_adjoint_step_u": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, dp]),
            "pf_adjoint_initial_rate": (ctypes.c_int, [vp, vp, vp, vp, dp]),
            "pf_timing": (ctypes.c_int, [vp, ctypes.c_int, dp, ctypes.POINTER(ctypes.c_int64), dp]),
            "pf_fem_table_size": (sz, []),
            "pf_fem_tables": (ctypes.c_int, [cfgp, dp, sz]),
            "pf_mg_levels": (ctypes.c_int, [cfgp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32), dp, ctypes.c_int32]),
            "pf_mg_table": (ctypes.c_int, [cfgp, ctypes.c_int32, ctypes.c_int32, dp, sz]),
            "pf_status_str": (ctypes.c_char_p, [ctypes.c_int]),
            "pf_last_error": (ctypes.c_char_p, [vp]),
            "pf_destroy": (None, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def make_config(cfg: PFConfig):
    """pf_config for a PFConfig; returns (struct, keep-alive electrode array)."""
    els = (pf_electrode * max(1, len(cfg.electrodes)))()
    for t, e in enumerate(cfg.electrodes):
        els[t] = pf_electrode(e.x0, e.x1, e.y0, e.y1, float(e.volts))
    c = pf_config()
    c.nx, c.ny, c.nz = cfg.nx, cfg.ny, cfg.nz
    for f in ("h", "a1", "a11", "a12", "G", "L", "dt", "eps_b", "phi_bottom", "phi_top",
              "C11", "C12", "C44", "Q11", "Q12", "Q44", "tol_phi", "tol_u"):
        setattr(c, f, float(getattr(cfg, f)))
    c.n_electrodes = len(cfg.electrodes)
    c.electrodes = ctypes.cast(els, ctypes.POINTER(pf_electrode))
    c.integrator = PF_INT_PC if cfg.integrator == "pc" else PF_INT_EULER
    c.precision = PRECISIONS[cfg.precision]
    c.maxit = cfg.maxit
    c.warm_start = int(cfg.warm_start)
    c.terms = cfg.terms
    c.nonlocal_every = cfg.nonlocal_every
    c.extrap_order = cfg.extrap_order
    c.noise_sigma = cfg.noise_sigma
    c.noise_seed = cfg.noise_seed
    c.top_bc = {"metal": PF_TOP_METAL, "open": PF_TOP_OPEN}[cfg.top]
    c.n_air = cfg.n_air
    c.eps_air = cfg.eps_air
    c.misfit[:] = [float(x) for x in cfg.misfit]
    c.rotation[:] = [float(x) for x in cfg.rotation]
    c.precond = {"jacobi": PF_PRECOND_JACOBI, "mg": PF_PRECOND_MG}[cfg.precond]
    return c, els


def status_str(s: int) -> str:
    return lib().pf_status_str(s).decode()


# --- the C entry points, one Python function each --------------------------

def pf_workspace_size(cfg: PFConfig) -> int:
    c, keep = make_config(cfg)
    n = ctypes.c_size_t()
    st = lib().pf_workspace_size(ctypes.byref(c), ctypes.byref(n))
    if st != PF_OK:
        raise PFError(st, f"pf_workspace_size: {status_str(st)}")
    return n.value


def pf_fem_tables(cfg: PFConfig):
    """The kernels' constant FEM stencil tables (host computation) as a dict
    of float64 numpy arrays K (2,3,3,27), Bf (2,3,6,27), Su (3,6,3,27),
    Ms (3,27)."""
    import numpy as np
    c, keep = make_config(cfg)
    n = lib().pf_fem_table_size()
    out = np.zeros(n)
    st = lib().pf_fem_tables(ctypes.byref(c), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n)
    if st != PF_OK:
        raise PFError(st, f"pf_fem_tables: {status_str(st)}")
    sizes = [("K", (2, 3, 3, 27)), ("Bf", (2, 3, 6, 27)), ("Su", (3, 6, 3, 27)), ("Ms", (3, 27))]
    res, o = {}, 0
    for name, shp in sizes:
        cnt = int(np.prod(shp))
        res[name] = out[o:o + cnt].reshape(shp)
        o += cnt
    return res


def pf_mg_levels(cfg: PFConfig, field: str = "u"):
    """The multigrid levels of the FEM ("u") or Poisson ("phi") operator:
    list of ((nx, ny, nz), omega)."""
    import numpy as np
    c, keep = make_config(cfg)
    n = ctypes.c_int32()
    dims = (ctypes.c_int32 * 48)()
    om = np.zeros(16)
    st = lib().pf_mg_levels(ctypes.byref(c), 1 if field == "u" else 0, ctypes.byref(n), dims,
                            om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 16)
    if st != PF_OK:
        raise PFError(st, f"pf_mg_levels: {status_str(st)}")
    return [((dims[3 * l], dims[3 * l + 1], dims[3 * l + 2]), float(om[l])) for l in range(n.value)]


def pf_mg_table(cfg: PFConfig, level: int, field: str = "u"):
    """Stencils of a multigrid level (0: the operator, >= 1: Galerkin), float64
    (nz, nc, nc, 27) with nc = 3 for "u" and 1 for "phi"."""
    import numpy as np
    c, keep = make_config(cfg)
    nz = pf_mg_levels(cfg, field)[level][0][2]
    nc = 3 if field == "u" else 1
    out = np.zeros(nz * nc * nc * 27)
    st = lib().pf_mg_table(ctypes.byref(c), 1 if field == "u" else 0, level,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size)
    if st != PF_OK:
        raise PFError(st, f"pf_mg_table: {status_str(st)}")
    return out.reshape(nz, nc, nc, 27)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """One library context bound to a configuration, a torch-owned device
    workspace (or, with static_workspace, the library's static one: see
    pf_init_static) and the current torch stream of `device`."""

    def __init__(self, cfg: PFConfig, device: str = "cuda:0", static_workspace: bool = False):
        if not torch.cuda.is_available():
            raise RuntimeError("the phase-field library needs a GPU (torch.cuda is not available)")
        self.cfg = cfg
        self.device = torch.device(device)
        self.L = lib()
        self._cfg_struct, self._els = make_config(cfg)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = ctypes.c_void_p()
        if static_workspace:
            self.ws = None
            with torch.cuda.device(self.device):
                st = self.L.pf_init_static(ctypes.byref(self._cfg_struct), ctypes.c_void_p(self.stream.cuda_stream),
                                           ctypes.byref(self.ctx))
            if st != PF_OK:
                raise PFError(st, f"pf_init_static: {status_str(st)}")
        else:
            nbytes = pf_workspace_size(cfg)
            # over-allocate by 256 B and align the base
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            self._ws_ptr = (base + 255) // 256 * 256
            st = self.L.pf_init(ctypes.byref(self._cfg_struct), ctypes.c_void_p(self._ws_ptr), nbytes,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.ctx))
            if st != PF_OK:
                raise PFError(st, f"pf_init: {status_str(st)}")
        self.state_dtype = torch.float32 if cfg.precision == "fp32_refine" else torch.float64
        self.N = cfg.nodes

    def close(self):
        """Releases the context (pf_destroy); also done when it is collected."""
        if getattr(self, "ctx", None) and self.ctx.value:
            self.L.pf_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- helpers -----------------------------------------------------------
    def _check(self, st: int, what: str, allow_noconv: bool = False) -> int:
        if st == PF_OK or (allow_noconv and st == PF_ENOCONV):
            return st
        msg = self.L.pf_last_error(self.ctx)
        raise PFError(st, f"{what}: {status_str(st)}: {msg.decode() if msg else ''}")

    def _field(self, t: torch.Tensor, ncomp: int, dtype, name: str) -> torch.Tensor:
        """ncomp = 0: a field of the potential grid (phi)."""
        shape = (ncomp,) + self.cfg.shape if ncomp > 1 else (self.cfg.shape if ncomp == 1 else self.cfg.phi_shape)
        if t.device != self.device or t.dtype != dtype or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous {dtype} tensor of shape {shape} on {self.device}, "
                             f"got {t.dtype} {tuple(t.shape)} on {t.device}")
        return t

    def new_field(self, ncomp: int, dtype=None) -> torch.Tensor:
        """ncomp = 0: a field of the potential grid (phi)."""
        shape = (ncomp,) + self.cfg.shape if ncomp > 1 else (self.cfg.shape if ncomp == 1 else self.cfg.phi_shape)
        return torch.zeros(shape, dtype=dtype or self.state_dtype, device=self.device)

    # --- entry points --------------------------------------------------------
    def set_state(self, P: torch.Tensor, phi0: Optional[torch.Tensor] = None, u0: Optional[torch.Tensor] = None):
        self._field(P, 3, self.state_dtype, "P")
        if phi0 is not None:
            self._field(phi0, 0, torch.float64, "phi0")
        if u0 is not None:
            self._field(u0, 3, torch.float64, "u0")
        return self._check(self.L.pf_set_state(self.ctx, _ptr(P), _ptr(phi0), _ptr(u0)), "pf_set_state", True)

    def restore_state(self, P, V, phi, u, step: int):
        self._field(P, 3, self.state_dtype, "P")
        self._field(V, 3, self.state_dtype, "V")
        self._field(phi, 0, torch.float64, "phi")
        self._field(u, 3, torch.float64, "u")
        self._check(self.L.pf_restore_state(self.ctx, _ptr(P), _ptr(V), _ptr(phi), _ptr(u), step),
                    "pf_restore_state")

    def get_state(self):
        P, V = self.new_field(3), self.new_field(3)
        phi, u = self.new_field(0, torch.float64), self.new_field(3, torch.float64)
        step = ctypes.c_int64()
        self._check(self.L.pf_get_state(self.ctx, _ptr(P), _ptr(V), _ptr(phi), _ptr(u), ctypes.byref(step)),
                    "pf_get_state")
        return P, V, phi, u, step.value

    def get_fields(self, *names):
        """Copies of the named state fields ("P", "V", "phi", "u"), in the
        order given (pf_get_state with the other pointers NULL)."""
        made = {}
        for nm in names:
            if nm in ("P", "V"):
                made[nm] = self.new_field(3)
            elif nm == "phi":
                made[nm] = self.new_field(0, torch.float64)
            elif nm == "u":
                made[nm] = self.new_field(3, torch.float64)
            else:
                raise ValueError(f"get_fields: unknown field {nm!r}")
        step = ctypes.c_int64()
        self._check(self.L.pf_get_state(self.ctx, _ptr(made.get("P")), _ptr(made.get("V")), _ptr(made.get("phi")),
                                        _ptr(made.get("u")), ctypes.byref(step)), "pf_get_state")
        return tuple(made[nm] for nm in names)

    def step(self, nsteps: int = 1) -> dict:
        st = pf_step_stats()
        s = self.L.pf_step(self.ctx, nsteps, ctypes.byref(st))
        self._check(s, "pf_step", True)
        d = st.as_dict()
        d["status"] = s
        return d

    def solve_phi(self, P: torch.Tensor, phi: Optional[torch.Tensor] = None):
        self._field(P, 3, self.state_dtype, "P")
        phi = self.new_field(0, torch.float64) if phi is None else self._field(phi, 0, torch.float64, "phi")
        st = pf_solve_stats()
        s = self.L.pf_solve_phi(self.ctx, _ptr(P), _ptr(phi), ctypes.byref(st))
        self._check(s, "pf_solve_phi", True)
        d = st.as_dict()
        d["status"] = s
        return phi, d

    def solve_u(self, P: torch.Tensor, u: Optional[torch.Tensor] = None):
        self._field(P, 3, self.state_dtype, "P")
        u = self.new_field(3, torch.float64) if u is None else self._field(u, 3, torch.float64, "u")
        st = pf_solve_stats()
        s = self.L.pf_solve_u(self.ctx, _ptr(P), _ptr(u), ctypes.byref(st))
        self._check(s, "pf_solve_u", True)
        d = st.as_dict()
        d["status"] = s
        return u, d

    def force(self, P: torch.Tensor, phi: Optional[torch.Tensor], u: Optional[torch.Tensor]) -> torch.Tensor:
        self._field(P, 3, self.state_dtype, "P")
        if phi is not None:
            self._field(phi, 0, torch.float64, "phi")
        if u is not None:
            self._field(u, 3, torch.float64, "u")
        F = self.new_field(3)
        self._check(self.L.pf_force(self.ctx, _ptr(P), _ptr(phi), _ptr(u), _ptr(F)), "pf_force")
        return F

    def noise(self, step: int) -> torch.Tensor:
        """The standard normal variates (3, nz, ny, nx), float64, of the
        thermal noise of step `step`."""
        xi = torch.empty((3,) + self.cfg.shape, dtype=torch.float64, device=self.device)
        self._check(self.L.pf_noise(self.ctx, int(step), _ptr(xi)), "pf_noise")
        return xi

    def timing(self, mode):
        """Returns {class: (ms, launches, algorithmic bytes)} accumulated since
        the last call and sets the accounting mode: False / PF_TIMING_OFF,
        True / PF_TIMING_EVENTS (per-launch events, solves sequential) or
        PF_TIMING_BYTES (launch and byte counts only)."""
        mode = {False: PF_TIMING_OFF, True: PF_TIMING_EVENTS}.get(mode, mode)
        n = len(KERNEL_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        nb = (ctypes.c_double * n)()
        self._check(self.L.pf_timing(self.ctx, int(mode), ms, cnt, nb), "pf_timing")
        return {k: (ms[t], cnt[t], nb[t]) for t, k in enumerate(KERNEL_CLASSES)}

    def energy(self):
        out = (ctypes.c_double * 5)()
        self._check(self.L.pf_energy(self.ctx, out), "pf_energy", True)
        return [out[t] for t in range(5)]

    def set_params(self, volts: Optional[Sequence[float]] = None, a1: Optional[float] = None):
        n = len(self.cfg.electrodes)
        arr = None
        if volts is not None:
            if len(volts) != n:
                raise ValueError(f"expected {n} voltages")
            arr = (ctypes.c_double * max(1, n))(*[float(v) for v in volts])
        a = float(self.cfg.a1 if a1 is None else a1)
        self._check(self.L.pf_set_params(self.ctx, arr, a), "pf_set_params")

    def adjoint_step(self, Pn, Vn, lamP, lamV, dtheta, un=None):
        """One reverse step; un (FP64 3N, optional): the u that forward step n
        solved for, which spares the re-solve at the linearisation point."""
        self._field(Pn, 3, self.state_dtype, "P_n")
        self._field(lamP, 3, self.state_dtype, "lamP")
        self._field(lamV, 3, self.state_dtype, "lamV")
        if Vn is not None:
            self._field(Vn, 3, self.state_dtype, "V_n")
        if un is not None:
            self._field(un, 3, torch.float64, "u_n")
        arr = (ctypes.c_double * len(dtheta))(*dtheta)
        s = self.L.pf_adjoint_step_u(self.ctx, _ptr(Pn), _ptr(Vn), _ptr(un), _ptr(lamP), _ptr(lamV), arr)
        self._check(s, "pf_adjoint_step", True)
        for t in range(len(dtheta)):
            dtheta[t] = arr[t]
        return s

    def adjoint_initial_rate(self, P0, lamP, lamV, dtheta):
        """Folds the initial rate V0 = F(P0) into the adjoints (no-op for Euler)."""
        self._field(P0, 3, self.state_dtype, "P0")
        arr = (ctypes.c_double * len(dtheta))(*dtheta)
        s = self.L.pf_adjoint_initial_rate(self.ctx, _ptr(P0), _ptr(lamP), _ptr(lamV), arr)
        self._check(s, "pf_adjoint_initial_rate", True)
        for t in range(len(dtheta)):
            dtheta[t] = arr[t]
        return s


# Same names as the C ABI, taking a Context.
def pf_init(cfg: PFConfig, device: str = "cuda:0") -> Context:
    return Context(cfg, device)


def pf_set_state(ctx: Context, P, phi0=None, u0=None):
    return ctx.set_state(P, phi0, u0)


def pf_get_state(ctx: Context):
    return ctx.get_state()


def pf_step(ctx: Context, nsteps: int = 1):
    return ctx.step(nsteps)


def pf_solve_phi(ctx: Context, P, phi=None):
    return ctx.solve_phi(P, phi)


def pf_solve_u(ctx: Context, P, u=None):
    return ctx.solve_u(P, u)


def pf_force(ctx: Context, P, phi, u):
    return ctx.force(P, phi, u)


def pf_noise(ctx: Context, step):
    return ctx.noise(step)


def pf_energy(ctx: Context):
    return ctx.energy()


def pf_adjoint_step(ctx: Context, Pn, Vn, lamP, lamV, dtheta):
    return ctx.adjoint_step(Pn, Vn, lamP, lamV, dtheta)
