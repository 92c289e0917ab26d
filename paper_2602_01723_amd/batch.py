"""Batched forward + adjoint evaluation of many parameter candidates.

Each candidate is its own scene (own grid, own particle count).  The batched
form keeps all candidates in one context and records a whole evaluation
(mpm_step_n with a tape, the position-loss cotangent, mpm_backward) into one
hipGraph; the plain form advances each candidate in its own context with
eager calls, one after the other.  Both return per-particle gradients of
the position loss L_b = mean over scene b's N_b x 3 coordinates of
(x - x*)^2 with respect to log E and nu.
"""
from __future__ import annotations

from typing import List

import numpy as np

from . import binding as B


def loss_weights(offsets) -> np.ndarray:
    """1 / (3 N_b) for every particle of scene b."""
    w = np.zeros(int(offsets[-1]), np.float32)
    for b in range(len(offsets) - 1):
        lo, hi = int(offsets[b]), int(offsets[b + 1])
        if hi > lo:
            w[lo:hi] = 1.0 / (3.0 * (hi - lo))
    return w


class Evaluation:
    """Forward + loss + adjoint of one context (all scenes of `sc`)."""

    def __init__(self, sc, steps: int, K: int, x_target, log_E=None, nu=None, tuning=None, stream=None,
                 deterministic=False):
        import torch
        self.sc = sc
        self.steps = int(steps)
        self.K = int(K)
        offs = None if sc.n_batch == 1 else sc.batch_offsets
        self.ctx = B.mpm_init(sc.grid_res, sc.dt, sc.materials, sc.n, offs, sc.gravity, sc.bound,
                              deterministic=deterministic)
        if tuning:
            B.mpm_set_tuning(self.ctx, **tuning)
        self.p = B.Particles.from_arrays(sc.x, sc.v, sc.C, sc.F, sc.mass, sc.vol0,
                                         sc.log_E if log_E is None else log_E,
                                         sc.nu if nu is None else nu, sc.mat_id)
        self.init = self.p.clone()
        N = sc.n
        self.x_target = torch.as_tensor(np.ascontiguousarray(np.asarray(x_target, np.float32).reshape(N, 3).T)).cuda()
        self.weight = torch.as_tensor(loss_weights(sc.batch_offsets)).cuda()
        self.tape = torch.empty(B.mpm_tape_size(self.ctx, self.steps, self.K) // 4 + 64, device="cuda")
        self.g_x = torch.empty(3, N, device="cuda")
        self.g_log_E = torch.empty(N, device="cuda")
        self.g_nu = torch.empty(N, device="cuda")
        self.graph = None
        self.stream = torch.cuda.Stream() if stream is None else stream

    def reset(self):
        """Restore the initial particle state (eager copies)."""
        for k in ("x", "v", "C", "F"):
            getattr(self.p, k).copy_(getattr(self.init, k))

    def _record(self, stream):
        B.mpm_step_n(self.ctx, self.p, self.steps, tape=self.tape, checkpoint_every=self.K, stream=stream)
        B.mpm_position_loss_grad(self.ctx, self.p.x, self.x_target, self.weight, self.g_x, stream=stream)
        B.mpm_backward(self.ctx, self.p, self.tape, self.steps, g_x=self.g_x, g_log_E=self.g_log_E,
                       g_nu=self.g_nu, stream=stream)

    def run_eager(self):
        import torch
        self.reset()
        with torch.cuda.stream(self.stream):
            self.stream.wait_stream(torch.cuda.default_stream())
            self._record(self.stream)
        torch.cuda.default_stream().wait_stream(self.stream)

    def capture(self):
        import torch
        self.reset()
        torch.cuda.synchronize()
        B.mpm_graph_begin(self.ctx, self.stream)
        try:
            self._record(self.stream)
        finally:
            self.graph = B.mpm_graph_end(self.ctx, self.stream,
                                         keep=(self.p, self.tape, self.g_x, self.g_log_E, self.g_nu,
                                               self.x_target, self.weight))
        return self.graph

    def run_graph(self):
        import torch
        self.reset()
        self.stream.wait_stream(torch.cuda.default_stream())
        self.graph.launch(self.stream)
        torch.cuda.default_stream().wait_stream(self.stream)

    def losses(self) -> np.ndarray:
        x = self.p.x.T.cpu().numpy()
        xt = self.x_target.T.cpu().numpy()
        offs = self.sc.batch_offsets
        return np.array([((x[offs[b]:offs[b + 1]] - xt[offs[b]:offs[b + 1]]) ** 2).mean()
                         if offs[b + 1] > offs[b] else 0.0 for b in range(len(offs) - 1)])

    def gradients(self):
        return self.g_log_E.cpu().numpy(), self.g_nu.cpu().numpy()


def target_positions(sc, steps, log_E, nu, deterministic=False) -> np.ndarray:
    """Final positions of the scene advanced with other (hidden) parameters."""
    import torch
    offs = None if sc.n_batch == 1 else sc.batch_offsets
    ctx = B.mpm_init(sc.grid_res, sc.dt, sc.materials, sc.n, offs, sc.gravity, sc.bound, deterministic=deterministic)
    p = B.Particles.from_arrays(sc.x, sc.v, sc.C, sc.F, sc.mass, sc.vol0, log_E, nu, sc.mat_id)
    B.mpm_step_n(ctx, p, steps)
    torch.cuda.synchronize()
    return p.state_numpy()[0]


def per_particle(values_per_scene, offsets) -> np.ndarray:
    out = np.zeros(int(offsets[-1]), np.float32)
    for b in range(len(offsets) - 1):
        out[offsets[b]:offsets[b + 1]] = values_per_scene[b]
    return out


def plain_evaluations(sc, steps, K, x_target, tuning=None, deterministic=False) -> List[Evaluation]:
    """One single-scene Evaluation per candidate of the batched scene `sc`,
    all on one shared stream (they run one after the other)."""
    import torch
    stream = torch.cuda.Stream()
    evs = []
    for b in range(sc.n_batch):
        sub = sc.subset(b)
        lo, hi = int(sc.batch_offsets[b]), int(sc.batch_offsets[b + 1])
        evs.append(Evaluation(sub, steps, K, np.asarray(x_target)[lo:hi], tuning=tuning, stream=stream,
                              deterministic=deterministic))
    return evs
