"""Parity at the full benchmark size (2,000,000 particles, 128^3 grid, the
default launch configuration that bench.py times), on outputs the FP64
oracle can compute one by one:

* P2G at sampled grid nodes, from only the particles whose stencil covers them;
* the grid update of the GPU's own (m, mv) on the whole grid;
* G2P + F update + return map of sampled particles, from the GPU's grid
  velocities.

Plus properties that hold at any size: mass conservation over the grid.
"""
import numpy as np
import pytest
import torch

from oracle import mpm_oracle as O
from paper_2602_01723_amd import binding as B
from paper_2602_01723_amd import scenes
from tests.parity import TOL_SUBSTEP, dx_tolerance, elem_err, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["step_n", "resident"])
def fullsize_step(request):
    """The substep after 40 others, through mpm_step_n (as configured by
    default), or through the resident frame loop that bench.py times
    (re-sort every 32 substeps; the last substep's G2P reads the grid that
    the previous mpm_advance call left behind)."""
    sc = scenes.make_scene("large_scene")
    p = B.Particles.from_scene(sc)
    if request.param == "step_n":
        ctx = B.init_from_scene(sc)
        B.mpm_step_n(ctx, p, 40)  # deform the bodies first (re-sorts, work-item tables rebuilt)
        torch.cuda.synchronize()
        state0 = p.state_numpy()
        B.mpm_substep(ctx, p)
    else:
        ctx = B.init_from_scene(sc, sort_every=32)
        B.mpm_load(ctx, p)
        B.mpm_advance(ctx, 40)
        B.mpm_store(ctx, p)
        torch.cuda.synchronize()
        state0 = p.state_numpy()
        B.mpm_advance(ctx, 1)
        B.mpm_store(ctx, p)
    torch.cuda.synchronize()
    m, mv, v = (t.cpu().numpy().astype(np.float64) for t in B.grid_state(ctx))
    diag = B.mpm_get_diagnostics(ctx)
    return sc, state0, p.state_numpy(), (m, mv, v), diag


def test_fullsize_diagnostics_and_mass(fullsize_step):
    sc, state0, state1, (m, mv, v), diag = fullsize_step
    assert diag["nonfinite"] == 0 and diag["out_of_grid"] == 0
    total = sc.mass.astype(np.float64).sum()
    assert abs(m.sum() - total) <= 1e-5 * total


def test_fullsize_p2g_sampled_nodes(fullsize_step):
    sc, state0, _, (m, mv, _), _ = fullsize_step
    n = sc.grid_res
    rng = np.random.default_rng(0)
    active = np.nonzero(m > 0)[0]
    nodes = rng.choice(active, 200, replace=False)
    idx = np.stack([nodes // (n * n), (nodes // n) % n, nodes % n], -1)
    x0 = state0[0].astype(np.float64)
    base = np.floor(x0 * n - 0.5).astype(np.int64)
    # particles whose 3-node stencil covers any sampled node
    sel = np.zeros(len(x0), bool)
    for node in idx:
        sel |= np.all((base <= node) & (base >= node - 2), axis=1)
    sub = np.nonzero(sel)[0]
    params = O.Params(sc.mass[sub], sc.vol0[sub], sc.log_E[sub], sc.nu[sub], sc.mat_id[sub], sc.materials, n, sc.dt)
    F0 = torch.tensor(state0[3][sub], dtype=torch.float64)
    mu, lam = O.lame(params.log_E, params.nu)
    tau = O.kirchhoff_stress(F0, mu, lam, params.mat_id, params.materials)
    mr, mvr = O.p2g(torch.tensor(x0[sub]), torch.tensor(state0[1][sub], dtype=torch.float64),
                    torch.tensor(state0[2][sub], dtype=torch.float64), tau, params.mass, params.vol0, n, sc.dt)
    mr, mvr = mr.numpy()[nodes], mvr.numpy()[nodes]
    s_m = float(sc.mass.mean())
    s_v = max(float(np.abs(state0[1]).max()), 9.8 * sc.dt)
    errs = dict(m=rel_err(m[nodes], mr, s_m), mv=rel_err(mv[nodes], mvr, s_m * s_v),
                m_e=elem_err(m[nodes], mr, s_m),
                mv_e=elem_err(mv[nodes], mvr, np.repeat(np.maximum(mr, s_m) * s_v, 3)))  # per-node floor m_i s_v
    print("sampled nodes", len(nodes), "particles", len(sub), errs, flush=True)
    assert max(errs.values()) <= TOL_SUBSTEP, errs


def test_fullsize_grid_update_and_g2p_sampled_particles(fullsize_step):
    sc, state0, state1, (m, mv, v), _ = fullsize_step
    n = sc.grid_res
    vr = O.grid_update(torch.tensor(m), torch.tensor(mv), n, sc.dt, sc.gravity, sc.bound).numpy()
    sel = m > 1e-6 * m.max()
    s_v = max(float(np.abs(vr).max()), 9.8 * sc.dt)
    e_v = (rel_err(v[sel], vr[sel], s_v), elem_err(v[sel], vr[sel], s_v))
    print("grid update", e_v, flush=True)
    assert max(e_v) <= TOL_SUBSTEP
    rng = np.random.default_rng(1)
    pick = rng.choice(sc.n, 20000, replace=False)
    params = O.Params(sc.mass[pick], sc.vol0[pick], sc.log_E[pick], sc.nu[pick], sc.mat_id[pick], sc.materials, n,
                      sc.dt)
    x0 = torch.tensor(state0[0][pick], dtype=torch.float64)
    F0 = torch.tensor(state0[3][pick], dtype=torch.float64)
    x1, v1, C1, Ftr = O.g2p(x0, F0, torch.tensor(v), n, sc.dt)
    mu, lam = O.lame(params.log_E, params.nu)
    F1 = O.plasticity(Ftr, mu, lam, params.mat_id, params.materials)
    sv = max(float(v1.abs().max()), 9.8 * sc.dt)
    errs = {}
    for k, g, r, s in (("x", state1[0][pick], x1.numpy(), 1.0 / n), ("v", state1[1][pick], v1.numpy(), sv),
                       ("C", state1[2][pick], C1.numpy(), sv * n), ("F", state1[3][pick], F1.numpy(), 1.0)):
        errs[k] = rel_err(g, r, s)
        errs[k + "_e"] = elem_err(g, r, s)
    d_g = state1[0][pick].astype(np.float64) - x0.numpy()
    d_r = x1.numpy() - x0.numpy()
    e_dx = elem_err(d_g, d_r, sc.dt * sv)
    dx_tol = dx_tolerance(x1.numpy(), sc.dt, sv)
    print("sampled particles", len(pick), errs, "dx_e", e_dx, "bound", dx_tol, flush=True)
    assert max(errs.values()) <= TOL_SUBSTEP, errs
    assert e_dx <= dx_tol
