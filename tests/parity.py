"""Shared helpers of the parity tests: the comparison metric and runners.

Metric (per field X): err = |X_gpu - X_ref|_2 / max(|X_ref|_2, s_X sqrt(count))
with natural-scale floors s_x = dx, s_v = max(|v|_inf, |g| dt),
s_C = s_v / dx, s_F = 1, s_m = mean particle mass, s_mv = s_m s_v.
Grid velocity is compared on nodes with m > 1e-6 max m.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from oracle import mpm_oracle as O

TOL_SUBSTEP = 1e-5       # relative, per substep, grid and particle state
TOL_LONG_X = 1e-3        # relative, positions after 100 substeps


def rel_err(gpu, ref, scale):
    g = np.asarray(gpu, np.float64).ravel()
    r = np.asarray(ref, np.float64).ravel()
    if r.size == 0:
        return 0.0
    den = max(np.linalg.norm(r), scale * math.sqrt(r.size))
    return float(np.linalg.norm(g - r) / den) if den > 0 else float(np.linalg.norm(g - r))


def scales(scene_like, v_ref, dt, grid_res, gravity=(0, -9.8, 0), mass=None):
    s_v = max(float(np.abs(v_ref).max()) if v_ref.size else 0.0, float(np.linalg.norm(gravity)) * dt)
    s_m = float(np.mean(mass)) if mass is not None and len(mass) else 1.0
    return dict(x=1.0 / grid_res, v=s_v, C=s_v * grid_res, F=1.0, m=s_m, mv=s_m * s_v)


def compare_substep(state0, gpu_state, gpu_grid, params: O.Params, mass):
    """One oracle substep from the float32 state0; returns dict of errors."""
    s0 = tuple(torch.as_tensor(np.asarray(a, np.float64)) for a in state0)
    (x1, v1, C1, F1), grids = O.substep(s0, params, return_grid=True)
    ref = dict(x=x1.numpy(), v=v1.numpy(), C=C1.numpy(), F=F1.numpy())
    gx, gv, gC, gF = gpu_state
    sc = scales(None, ref["v"], params.dt, params.n, params.gravity, mass)
    errs = {}
    for k, gval in (("x", gx), ("v", gv), ("C", gC), ("F", gF)):
        errs[k] = rel_err(gval, ref[k], sc[k])
    # displacement, a stricter view of x
    errs["dx"] = rel_err(np.asarray(gx, np.float64) - state0[0], ref["x"] - np.asarray(state0[0], np.float64),
                         params.dt * sc["v"])
    if gpu_grid is not None:
        m_g, mv_g, v_g = gpu_grid
        n3 = params.n ** 3
        m_r = torch.cat([g[0] for g in grids]).numpy()
        mv_r = torch.cat([g[1] for g in grids]).numpy()
        v_r = torch.cat([g[2] for g in grids]).numpy()
        errs["m"] = rel_err(m_g, m_r, sc["m"])
        errs["mv"] = rel_err(mv_g, mv_r, sc["mv"])
        sel = m_r > 1e-6 * max(m_r.max(), 1e-300)
        errs["grid_v"] = rel_err(v_g[sel], v_r[sel], sc["v"])
    return errs, ref
