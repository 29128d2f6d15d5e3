"""torch.autograd binding of the library's checkpointed forward run and its hand-written
adjoint (argument marshalling only: the forward steps and the reverse sweep run in the
HIP kernels)."""
from __future__ import annotations

import torch

from .solver import Solver


class PCPFRun(torch.autograd.Function):
    """phi(T), psi(T) after nsteps RK4 steps (with the scheduled resets and
    preconditioning) from phi(0), psi(0) (None: reset at the first step) under the
    velocity amplitude amp. Differentiable in phi0, psi0 and amp."""

    @staticmethod
    def forward(ctx, phi0, psi0, amp, solver: Solver, dt: float, nsteps: int, t0: float = 0.0,
                step0: int = 0, every: int | None = None):
        a = float(amp)
        solver.set_velocity_amplitude(a)
        ctx.inputs = (phi0.detach().clone(), None if psi0 is None else psi0.detach().clone(), a,
                      float(dt), int(nsteps), float(t0), int(step0), every)
        solver.set_state(phi0.detach(), None if psi0 is None else psi0.detach(), t0, step0)
        solver.forward_ckpt(dt, nsteps, every)
        ctx.run_id = solver.run_id
        phi, psi, _, _ = solver.get_state(want_psi=True)
        ctx.solver = solver
        ctx.has_psi0 = psi0 is not None
        ctx.amp_shape = amp.shape if torch.is_tensor(amp) else None
        ctx.amp_dtype = amp.dtype if torch.is_tensor(amp) else torch.float64
        ctx.amp_device = amp.device if torch.is_tensor(amp) else torch.device("cpu")
        return phi, psi

    @staticmethod
    def backward(ctx, gphi, gpsi):
        s: Solver = ctx.solver
        if s.run_id != ctx.run_id:
            # the solver recorded another run (or ran an adjoint) since this forward: record
            # this graph's run again from its saved inputs. The forward run is
            # deterministic, so the checkpoints are bitwise those of the first recording.
            phi0, psi0, a, dt, nsteps, t0, step0, every = ctx.inputs
            s.set_velocity_amplitude(a)
            s.set_state(phi0, psi0, t0, step0)
            s.forward_ckpt(dt, nsteps, every)
        if gphi is None:
            gphi = torch.zeros((s.nelem, s.nupts), dtype=s.dtype, device=s.device)
        gphi0, gpsi0, ga = s.adjoint(gphi.contiguous(),
                                     None if gpsi is None else gpsi.contiguous())
        gamp = None
        if ctx.amp_shape is not None:
            gamp = torch.full(ctx.amp_shape, ga, dtype=ctx.amp_dtype, device=ctx.amp_device)
        return (gphi0, gpsi0 if ctx.has_psi0 else None, gamp, None, None, None, None, None,
                None)


def run(solver: Solver, phi0, amp, dt, nsteps, psi0=None, t0=0.0, step0=0, every=None):
    """Differentiable run; returns (phi(T), psi(T))."""
    if not torch.is_tensor(amp):
        amp = torch.tensor(float(amp), dtype=torch.float64)
    return PCPFRun.apply(phi0, psi0, amp, solver, dt, nsteps, t0, step0, every)
