"""Differentiable TDGL trajectories: P_N = PFSteps.apply(P0, volts, a1, ctx, n, k).

Forward: n library steps from P0 with the electrode voltages and Landau a1
given as tensors, keeping the full state (P, V, phi, u) every k steps.
Backward: for each checkpoint segment, newest first, the segment is
recomputed from its checkpoint (bitwise identical: the library's reductions
are deterministic and the checkpoint carries the solver warm starts; the
newest segment's states are kept from the forward instead), and the
discrete adjoint of every step is applied in reverse with
pf_adjoint_step_u, given the displacement that the step solved for;
finally pf_adjoint_initial_rate folds in the initial rate
V0 = F(P0) of the predictor-corrector.  Gradients are returned for P0, the
voltages and a1.
"""
from __future__ import annotations

import torch

from .pf import Context


class PFSteps(torch.autograd.Function):

    @staticmethod
    def forward(fctx, P0: torch.Tensor, volts: torch.Tensor, a1: torch.Tensor, pf: Context, nsteps: int,
                checkpoint_every: int):
        k = max(1, int(checkpoint_every))
        pf.set_params([float(v) for v in volts.detach().cpu().tolist()], float(a1.detach().cpu()))
        P0c = P0.detach().contiguous()
        pf.set_state(P0c)
        checkpoints = []
        # the states of the last segment are kept as the forward makes them
        # (the backward starts there, so that segment needs no recomputation)
        last_start = ((nsteps - 1) // k) * k if nsteps > 0 else 0
        last = []
        for s in range(nsteps):
            if s % k == 0:
                cp = pf.get_state()
                checkpoints.append(cp)
                # restarting from the checkpoint here too keeps the forward
                # identical to its recomputation (solver warm-start history
                # starts afresh at every checkpoint)
                pf.restore_state(*cp)
            if s >= last_start:
                Pn, Vn = pf.get_fields("P", "V")
                pf.step(1)
                last.append((Pn, Vn, pf.get_fields("u")[0]))
            else:
                pf.step(1)
        PN = pf.get_state()[0]
        fctx.last = last
        fctx.pf = pf
        fctx.nsteps = nsteps
        fctx.k = k
        fctx.checkpoints = checkpoints
        fctx.n_volts = volts.numel()
        fctx.theta_dev = (volts.device, volts.dtype, a1.device, a1.dtype)
        fctx.save_for_backward(P0c)
        return PN

    @staticmethod
    def backward(fctx, grad_PN: torch.Tensor):
        pf: Context = fctx.pf
        (P0,) = fctx.saved_tensors
        lamP = grad_PN.detach().to(pf.state_dtype).contiguous().clone()
        lamV = torch.zeros_like(lamP)
        dtheta = [0.0] * (fctx.n_volts + 1)
        nsteps, k = fctx.nsteps, fctx.k
        if fctx.checkpoints is None:
            raise RuntimeError("PFSteps: the backward frees its checkpoints and runs once per forward")
        nseg = len(fctx.checkpoints)
        # At most one segment's states are held at a time: the newest
        # segment's (kept from the forward) are dropped before the next
        # segment is recomputed, and each checkpoint once its segment is.
        for seg in reversed(range(nseg)):
            if seg == nseg - 1:
                states, fctx.last = fctx.last, None
            else:
                P, V, phi, u, step = fctx.checkpoints[seg]
                start = seg * k
                stop = min(nsteps, start + k)
                pf.restore_state(P, V, phi, u, step)
                del P, V, phi, u
                states = []
                for _ in range(start, stop):
                    st = pf.get_fields("P", "V")
                    pf.step(1)
                    # the displacement step n solved for: the adjoint step's
                    # linearisation point needs no second solve
                    states.append(st + pf.get_fields("u"))
                    del st
            fctx.checkpoints[seg] = None
            while states:
                Pn, Vn, un = states.pop()
                pf.adjoint_step(Pn, Vn, lamP, lamV, dtheta, un)
                del Pn, Vn, un
            del states
        fctx.checkpoints = None
        pf.adjoint_initial_rate(P0, lamP, lamV, dtheta)
        vdev, vdt, adev, adt = fctx.theta_dev
        g_volts = torch.tensor(dtheta[:fctx.n_volts], dtype=vdt, device=vdev)
        g_a1 = torch.tensor(dtheta[fctx.n_volts], dtype=adt, device=adev)
        return lamP.to(grad_PN.dtype), g_volts, g_a1, None, None, None


def tdgl_steps(P0, volts, a1, pf: Context, nsteps: int, checkpoint_every: int = 10):
    return PFSteps.apply(P0, volts, a1, pf, nsteps, checkpoint_every)
