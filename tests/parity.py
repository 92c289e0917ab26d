"""Shared helpers of the parity tests: the comparison metrics and runners.

Two metrics per field X, both with natural-scale floors s_x = max(dx, dt s_v),
s_v = max(|v|_inf, |g| dt), s_C = s_v / dx, s_F = max(1, dt s_C), s_m = mean
particle mass, s_mv = s_m s_v:

  norm     err   = |X_gpu - X_ref|_2 / max(|X_ref|_2, s_X sqrt(count))
  element  err_e = max_i |X_gpu,i - X_ref,i| / max(|X_ref,i|, s_X,i)

The element-wise floor of a node's momentum is that node's mass at the
scene's speed, s_mv,i = max(m_i, s_m) s_v: mv_i = m_i v_i, so an error that
the grid-velocity gate allows at node i (1e-5 of s_v) is 1e-5 m_i s_v in mv_i.
With one particle's momentum as the floor, a node holding thousands of
particles whose momenta nearly cancel would be judged against its small net
value, where the float32 rounding of the summed contributions (a bound
relative to their magnitudes, not to their sum) dominates.

The element-wise form is the gate that a single bad particle or node cannot
hide in; the norm is reported beside it.  Grid velocity is compared on nodes
with m > 1e-6 max m.  The displacement of one substep, dx = x' - x, is
compared as well: its bound adds to the 1e-5 the half-ulp rounding of the
stored float32 position, relative to the displacement scale dt s_v.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from oracle import mpm_oracle as O

TOL_SUBSTEP = 1e-5       # relative, per substep, grid and particle state (norm and element-wise)
TOL_LONG_X = 1e-3        # relative, positions after 100 substeps
FIELDS = ("x", "v", "C", "F", "m", "mv", "grid_v")


def rel_err(gpu, ref, scale):
    g = np.asarray(gpu, np.float64).ravel()
    r = np.asarray(ref, np.float64).ravel()
    if r.size == 0:
        return 0.0
    den = max(np.linalg.norm(r), scale * math.sqrt(r.size))
    return float(np.linalg.norm(g - r) / den) if den > 0 else float(np.linalg.norm(g - r))


def elem_err(gpu, ref, scale):
    """max_i |g_i - r_i| / max(|r_i|, scale_i); scale is one floor or one
    per element (in the raveled order of ref)."""
    g = np.asarray(gpu, np.float64).ravel()
    r = np.asarray(ref, np.float64).ravel()
    if r.size == 0:
        return 0.0
    sc = np.asarray(scale, np.float64)
    den = np.maximum(np.abs(r), sc.ravel() if sc.ndim else sc)
    den = np.where(den > 0, den, 1.0)  # a zero reference with a zero floor: absolute error
    return float(np.max(np.abs(g - r) / den))


def grad_elem_err(gpu, ref):
    """Element-wise error of a gradient field, each entry against
    max(|r_i|, rms(r)) (a gradient has no natural scale of its own)."""
    r = np.asarray(ref, np.float64).ravel()
    rms = float(np.sqrt(np.mean(r * r))) if r.size else 0.0
    return elem_err(gpu, ref, rms if rms > 0 else 1e-300)


def dx_tolerance(x_ref, dt, s_v, tol=TOL_SUBSTEP):
    """Bound of the displacement error: tol, plus the half-ulp rounding of a
    float32 position (2^-24 |x|) relative to the displacement scale dt s_v."""
    xmax = float(np.abs(x_ref).max()) if np.size(x_ref) else 0.0
    return tol + 2.0 ** -24 * xmax / max(dt * s_v, 1e-300)


def scales(scene_like, v_ref, dt, grid_res, gravity=(0, -9.8, 0), mass=None):
    """Floors of the metrics.  x' = x + dt v' and F' = (I + dt C') F carry
    the errors of v' and C' multiplied by dt, so their floors also take the
    substep's own scales dt s_v and dt s_C when those are larger (only in
    runs far beyond the CFL limit, where particles cross cells in a step)."""
    s_v = max(float(np.abs(v_ref).max()) if v_ref.size else 0.0, float(np.linalg.norm(gravity)) * dt)
    s_m = float(np.mean(mass)) if mass is not None and len(mass) else 1.0
    return dict(x=max(1.0 / grid_res, dt * s_v), v=s_v, C=s_v * grid_res, F=max(1.0, dt * s_v * grid_res), m=s_m,
                mv=s_m * s_v)


def compare_fields(gpu, ref, sc, errs):
    """Norm and element-wise errors of matching dicts of fields."""
    for k, gval in gpu.items():
        errs[k] = rel_err(gval, ref[k], sc[k])
        errs[k + "_e"] = elem_err(gval, ref[k], sc[k])
    return errs


def compare_substep(state0, gpu_state, gpu_grid, params: O.Params, mass):
    """One oracle substep from the float32 state0; returns dict of errors:
    the norm error of each field under its name, the element-wise error
    under name + "_e", and the displacement errors dx / dx_e with their
    bound dx_tol."""
    s0 = tuple(torch.as_tensor(np.asarray(a, np.float64)) for a in state0)
    (x1, v1, C1, F1), grids = O.substep(s0, params, return_grid=True)
    ref = dict(x=x1.numpy(), v=v1.numpy(), C=C1.numpy(), F=F1.numpy())
    gx, gv, gC, gF = gpu_state
    sc = scales(None, ref["v"], params.dt, params.n, params.gravity, mass)
    errs = compare_fields(dict(x=gx, v=gv, C=gC, F=gF), ref, sc, {})
    # displacement, a stricter view of x
    x0 = np.asarray(state0[0], np.float64)
    d_g, d_r = np.asarray(gx, np.float64) - x0, ref["x"] - x0
    errs["dx"] = rel_err(d_g, d_r, params.dt * sc["v"])
    errs["dx_e"] = elem_err(d_g, d_r, params.dt * sc["v"])
    errs["dx_tol"] = dx_tolerance(ref["x"], params.dt, sc["v"])
    if gpu_grid is not None:
        m_g, mv_g, v_g = gpu_grid
        m_r = torch.cat([g[0] for g in grids]).numpy()
        mv_r = torch.cat([g[1] for g in grids]).numpy()
        v_r = torch.cat([g[2] for g in grids]).numpy()
        sel = m_r > 1e-6 * max(m_r.max(), 1e-300)
        compare_fields(dict(m=m_g, grid_v=np.asarray(v_g)[sel]), dict(m=m_r, grid_v=v_r[sel]),
                       dict(m=sc["m"], grid_v=sc["v"]), errs)
        # momentum: element-wise against each node's mass at the scene's speed
        errs["mv"] = rel_err(mv_g, mv_r, sc["mv"])
        node_floor = np.maximum(np.asarray(m_r, np.float64).reshape(-1), sc["m"]) * sc["v"]
        errs["mv_e"] = elem_err(mv_g, mv_r, np.repeat(node_floor, 3))
    return errs, ref


def parity_failures(errs, tol=TOL_SUBSTEP, keys=FIELDS, displacement=True):
    """Fields whose norm or element-wise error exceeds tol (and the
    displacement beyond its bound)."""
    bad = {}
    for k in keys:
        for kk in (k, k + "_e"):
            if kk in errs and not errs[kk] <= tol:
                bad[kk] = errs[kk]
    if displacement and "dx" in errs:
        for kk in ("dx", "dx_e"):
            if not errs[kk] <= errs["dx_tol"]:
                bad[kk] = errs[kk]
    return bad
