"""BGDO, bidirectional graph decoupling optimisation (Alg. 1; Sec. 4.2;
App. B.3-B.4), driven through the C ABI.

Stage 1 advances the particles without gradients for `frames` frames of
`substeps_per_frame` substeps (the scene held in the context: mpm_load once,
mpm_advance per frame) and keeps a device copy of the state at the start of
every key frame (mpm_store).  Stage 2 takes, for each stored key
frame, one substep from it (mpm_substep on a copy) and lets
mpm_bgdo_accumulate add the per-particle term
    eta log(1 + |d|tau|/d log E|) - (1 - eta) (|F' - I|_F - delta_target),
eta = min(1, 0.1 log(1 + E)); mpm_bgdo_apply then sets
log E <- log E - g_total / |K|.  All arithmetic runs in the library's kernels;
this module only sequences the calls and holds the copies.
"""
from __future__ import annotations

from typing import Optional, Sequence

from . import binding as B

DELTA_TARGET = 0.1


def default_key_frames(frames: int):
    """{0, t, n}: first, middle and last frame."""
    return sorted({0, frames // 2, frames - 1})


def bgdo(ctx: B.Context, particles: B.Particles, frames: int, substeps_per_frame: int,
         key_frames: Optional[Sequence[int]] = None, delta_target: float = DELTA_TARGET, iterations: int = 1,
         stream=None):
    """Run Alg. 1 `iterations` times from the state in `particles` (left
    unchanged) and update particles.log_E in place; returns it."""
    import torch
    if frames < 1 or substeps_per_frame < 1 or iterations < 1:
        raise ValueError("frames, substeps_per_frame and iterations must be >= 1")
    keys = sorted(set(int(k) for k in (default_key_frames(frames) if key_frames is None else key_frames)))
    if not keys or keys[0] < 0 or keys[-1] >= frames:
        raise ValueError("key frames must lie in [0, frames)")
    init = particles.clone()
    for _ in range(iterations):
        p = init.clone()
        p.log_E = particles.log_E
        stored = []
        B.mpm_load(ctx, p, stream=stream)
        for frame in range(frames):  # stage 1: gradient-free forward run
            if frame in keys:
                B.mpm_store(ctx, p, stream=stream)
                stored.append(p.clone())
            B.mpm_advance(ctx, substeps_per_frame, stream=stream)
        g_total = torch.zeros(particles.n, dtype=torch.float32, device=particles.log_E.device)
        for snap in stored:  # stage 2: one substep from each key frame
            nxt = snap.clone()
            B.mpm_substep(ctx, nxt, stream=stream)
            B.mpm_bgdo_accumulate(ctx, snap, nxt.F, delta_target, g_total, stream=stream)
        B.mpm_bgdo_apply(ctx, particles.log_E, g_total, len(stored), stream=stream)
    return particles.log_E
