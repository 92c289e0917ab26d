"""The hand-written adjoint as a torch.autograd.Function.

``simulate(sim, log_E, nu, x0, v0, C0, F0)`` advances the particles by
``sim.n_steps`` substeps through mpm_step_n (writing a checkpoint tape every
``sim.checkpoint_every`` substeps) and returns the final (x, v, C, F).  Its
backward is mpm_backward: the reverse of G2P, the grid update, P2G and the
constitutive stress, recomputed segment by segment from the checkpoints.  It
returns the gradients with respect to the per-particle log E and nu and to
the initial state; gradients with respect to E itself follow from autograd's
chain rule when log_E = log(E) is computed by the caller.

All tensors are device float32 in the library's layout: x0, v0 [3, N]; C0,
F0 [9, N] (row-major 3x3 component planes); log_E, nu [N].  The material
table, masses, rest volumes and material ids are fixed in ``Simulation``.
The adjoint covers the elastic models without plasticity and det F > 0.

One context holds one tape: a backward must run before the next forward of
the same Simulation.  The backward of an earlier forward raises MPMError with
status MPM_ESTATE (a Simulation counts its forwards; mpm_backward itself
rejects a tape that is not the last one its context wrote).
"""
from __future__ import annotations

from typing import Optional

import torch

from . import binding as B


class Simulation:
    """A context plus the fixed per-particle data of one differentiable run."""

    def __init__(self, ctx: B.Context, mass, vol0, mat_id, n_steps: int, checkpoint_every: int = 20,
                 stream=None):
        if n_steps < 0 or checkpoint_every < 1:
            raise ValueError("n_steps >= 0 and checkpoint_every >= 1 are required")
        self.ctx = ctx
        self.mass = mass
        self.vol0 = vol0
        self.mat_id = mat_id
        self.n_steps = int(n_steps)
        self.checkpoint_every = int(checkpoint_every)
        self.stream = stream
        self._tape: Optional[torch.Tensor] = None
        self._generation = 0  # forwards run so far: only the latest one's tape is valid

    def tape(self) -> torch.Tensor:
        nbytes = B.mpm_tape_size(self.ctx, self.n_steps, self.checkpoint_every)
        if self._tape is None or self._tape.numel() * 4 < nbytes:
            self._tape = torch.empty(nbytes // 4 + 64, dtype=torch.float32, device=self.mass.device)
        return self._tape

    def particles(self, x, v, C, F, log_E, nu) -> B.Particles:
        return B.Particles(x=x, v=v, C=C, F=F, mass=self.mass, vol0=self.vol0, log_E=log_E, nu=nu,
                           mat_id=self.mat_id)


class _Simulate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, log_E, nu, x0, v0, C0, F0, sim: Simulation):
        p = sim.particles(x0.detach().clone().contiguous(), v0.detach().clone().contiguous(),
                          C0.detach().clone().contiguous(), F0.detach().clone().contiguous(),
                          log_E.detach().contiguous(), nu.detach().contiguous())
        tape = sim.tape()
        B.mpm_step_n(sim.ctx, p, sim.n_steps, tape=tape, checkpoint_every=sim.checkpoint_every, stream=sim.stream)
        sim._generation += 1
        ctx.generation = sim._generation
        ctx.sim = sim
        ctx.p = p
        ctx.tape = tape
        return p.x, p.v, p.C, p.F

    @staticmethod
    def backward(ctx, gx, gv, gC, gF):
        sim, p = ctx.sim, ctx.p
        if ctx.generation != sim._generation:  # the shared tape now holds a later run
            raise B.MPMError(B.MPM_ESTATE, "backward of a forward whose tape a later forward of the same "
                                           "Simulation has overwritten")
        N = p.n
        dev = p.mass.device
        g = [None if t is None else t.contiguous() for t in (gx, gv, gC, gF)]
        g_log_E = torch.empty(N, dtype=torch.float32, device=dev)
        g_nu = torch.empty(N, dtype=torch.float32, device=dev)
        want = ctx.needs_input_grad
        g0 = [torch.empty(c, N, dtype=torch.float32, device=dev) if want[2 + k] else None
              for k, c in enumerate((3, 3, 9, 9))]
        B.mpm_backward(sim.ctx, p, ctx.tape, sim.n_steps, *g, g_log_E, g_nu, *g0, stream=sim.stream)
        return g_log_E, g_nu, g0[0], g0[1], g0[2], g0[3], None


def simulate(sim: Simulation, log_E, nu, x0, v0, C0, F0):
    """Differentiable n-substep run; returns (x, v, C, F) after sim.n_steps."""
    return _Simulate.apply(log_E, nu, x0, v0, C0, F0, sim)
