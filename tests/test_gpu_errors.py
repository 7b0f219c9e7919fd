"""Error behaviour of the C ABI on a live context: each documented failure
returns its status code, leaves a message in pf_last_error, and leaves the
context usable."""
import ctypes
import math

import numpy as np
import pytest
import torch

from paper_1202_6116_amd.workloads import Electrode, PFConfig, domain_polarisation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pf():
    from paper_1202_6116_amd import pf as m
    return m


def cfg(**kw):
    base = dict(nx=20, ny=9, nz=5, electrodes=[Electrode(2, 6, 0, 9, 1.0), Electrode(12, 16, 0, 9, -1.0)])
    base.update(kw)
    return PFConfig(**base)


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def last_error(pf, ctx):
    return pf.lib().pf_last_error(ctx.ctx)


def test_calls_before_a_state_are_rejected(pf):
    print("case: no state", flush=True)
    ctx = pf.Context(cfg())
    L = pf.lib()
    out = (ctypes.c_double * 5)()
    assert L.pf_step(ctx.ctx, 1, None) == pf.PF_ESTATE
    assert L.pf_energy(ctx.ctx, out) == pf.PF_ESTATE
    assert L.pf_get_state(ctx.ctx, None, None, None, None, None) == pf.PF_ESTATE
    msg = last_error(pf, ctx)
    msg = msg.decode() if isinstance(msg, bytes) else msg
    assert "pf_set_state" in msg
    # the context still works once given a state
    P0 = torch.from_numpy(domain_polarisation(ctx.cfg, 3, block=3)).to("cuda:0")
    ctx.set_state(P0)
    ctx.step(1)
    assert torch.isfinite(ctx.get_state()[0]).all()


def test_invalid_values_are_rejected(pf):
    print("case: invalid values", flush=True)
    c = cfg()
    ctx = pf.Context(c)
    L = pf.lib()
    P0 = torch.from_numpy(domain_polarisation(c, 4, block=3)).to("cuda:0")
    ctx.set_state(P0)
    before = ctx.get_state()[0].clone()
    assert L.pf_step(ctx.ctx, -1, None) == pf.PF_EINVAL
    volts = (ctypes.c_double * 2)(0.5, math.nan)   # the first value must not be taken either
    assert L.pf_set_params(ctx.ctx, volts, c.a1) == pf.PF_EINVAL
    assert L.pf_set_params(ctx.ctx, None, math.inf) == pf.PF_EINVAL
    F = torch.empty_like(P0)
    phi = torch.zeros(c.phi_shape, dtype=torch.float64, device="cuda:0")
    u = torch.zeros((3,) + c.shape, dtype=torch.float64, device="cuda:0")
    assert L.pf_force(ctx.ctx, ptr(P0), None, ptr(u), ptr(F)) == pf.PF_EINVAL      # phi missing
    assert L.pf_force(ctx.ctx, ptr(P0), ptr(phi), None, ptr(F)) == pf.PF_EINVAL    # u missing
    assert L.pf_set_state(ctx.ctx, None, None, None) == pf.PF_EINVAL
    # nothing above changed the state or the parameters: the same two steps
    # as on a fresh context give the same result bit for bit
    assert torch.equal(ctx.get_state()[0], before)
    ctx.step(2)
    ref = pf.Context(c)
    ref.set_state(P0)
    ref.step(2)
    assert torch.equal(ctx.get_state()[0], ref.get_state()[0])


def test_workspace_too_small(pf):
    print("case: workspace too small", flush=True)
    c = cfg()
    cs, keep = pf.make_config(c)
    need = pf.pf_workspace_size(c)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    h = ctypes.c_void_p()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert pf.lib().pf_init(ctypes.byref(cs), ptr(ws), need - 1, stream, ctypes.byref(h)) == pf.PF_ENOMEM
    assert not h.value
    assert ws.data_ptr() % 256 == 0
    misaligned = ctypes.c_void_p(ws.data_ptr() + 8)
    assert pf.lib().pf_init(ctypes.byref(cs), misaligned, need - 8, stream, ctypes.byref(h)) == pf.PF_EINVAL
    assert not h.value
    assert pf.lib().pf_init(ctypes.byref(cs), ptr(ws), need, stream, ctypes.byref(h)) == pf.PF_OK
    pf.lib().pf_destroy(h)


def test_adjoint_needs_fields_refreshed_every_step(pf):
    print("case: adjoint with nonlocal_every 2", flush=True)
    c = cfg(nonlocal_every=2)
    ctx = pf.Context(c)
    P0 = torch.from_numpy(domain_polarisation(c, 5, block=3)).to("cuda:0")
    ctx.set_state(P0)
    lamP, lamV = torch.zeros_like(P0), torch.zeros_like(P0)
    dth = (ctypes.c_double * 3)()
    st = pf.lib().pf_adjoint_step(ctx.ctx, ptr(P0), ptr(P0), ptr(lamP), ptr(lamV), dth)
    assert st == pf.PF_EINVAL
    msg = last_error(pf, ctx)
    msg = msg.decode() if isinstance(msg, bytes) else msg
    assert "every step" in msg
