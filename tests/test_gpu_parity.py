"""HIP path vs the FP64 oracle, element by element, through the C ABI."""
import math

import numpy as np
import pytest
import torch

from oracle import mpm_oracle as O
from paper_2602_01723_amd import binding as B
from paper_2602_01723_amd import scenes
from tests.parity import TOL_LONG_X, TOL_SUBSTEP, compare_substep, elem_err, parity_failures, rel_err

pytestmark = pytest.mark.gpu

MATS_MIXED = [dict(elastic=0, plastic=0, yield_stress=0.0, friction_deg=0.0),
              dict(elastic=1, plastic=0, yield_stress=0.0, friction_deg=0.0),
              dict(elastic=1, plastic=1, yield_stress=1e3, friction_deg=0.0),
              dict(elastic=1, plastic=2, yield_stress=0.0, friction_deg=30.0),
              dict(elastic=0, plastic=1, yield_stress=2e3, friction_deg=0.0)]


# every elastic model alone, and each plastic model under a different elastic one
MATS_ALL = [dict(elastic=e, plastic=0, yield_stress=0.0, friction_deg=0.0) for e in range(6)] + [
    dict(elastic=2, plastic=1, yield_stress=2e3, friction_deg=0.0),
    dict(elastic=3, plastic=2, yield_stress=0.0, friction_deg=30.0),
    dict(elastic=0, plastic=3, yield_stress=0.0, friction_deg=0.0),
    dict(elastic=1, plastic=4, yield_stress=0.0, friction_deg=0.0),
    dict(elastic=5, plastic=3, yield_stress=0.0, friction_deg=0.0),
    dict(elastic=2, plastic=4, yield_stress=0.0, friction_deg=0.0),
    dict(elastic=4, plastic=4, yield_stress=0.0, friction_deg=0.0)]


def _grid_np(ctx):
    m, mv, v = B.grid_state(ctx)
    torch.cuda.synchronize()
    return m.cpu().numpy(), mv.cpu().numpy(), v.cpu().numpy()


def random_scene(seed, N, n=32, dt=1e-4, mats=MATS_MIXED, spread=0.35, fdev=0.08, cgrad=20.0, vel=0.5,
                 centre=0.5, E=(1e4, 1e6)):
    rng = np.random.default_rng(seed)
    x, v, C, F = scenes.random_state(rng, N, n, spread=spread, vel=vel, cgrad=cgrad, fdev=fdev, centre=centre)
    mass = rng.uniform(0.5, 2.0, N).astype(np.float32) * 1e-5
    vol0 = (mass / 1000.0).astype(np.float32)
    log_E = np.log(rng.uniform(E[0], E[1], N)).astype(np.float32)
    nu = rng.uniform(0.2, 0.4, N).astype(np.float32)
    mat = rng.integers(0, len(mats), N).astype(np.int32)
    return dict(x=x, v=v, C=C, F=F, mass=mass, vol0=vol0, log_E=log_E, nu=nu, mat_id=mat, mats=mats, n=n, dt=dt)


def run_case(d, warm=0, sort_every=0, tile_cap=0, offsets=None, grid="auto", deterministic=False):
    N = len(d["mass"])
    ctx = B.mpm_init(d["n"], d["dt"], d["mats"], N, offsets, sort_every=sort_every, grid=grid,
                     deterministic=deterministic)
    if tile_cap:
        B.mpm_set_tuning(ctx, tile_cap=tile_cap)
    p = B.Particles.from_arrays(d["x"], d["v"], d["C"], d["F"], d["mass"], d["vol0"], d["log_E"], d["nu"],
                                d["mat_id"])
    if warm:
        B.mpm_step_n(ctx, p, warm)
    state0 = p.state_numpy()
    B.mpm_substep(ctx, p)
    torch.cuda.synchronize()
    gpu = p.state_numpy()
    grid = _grid_np(ctx)
    params = O.Params(d["mass"], d["vol0"], d["log_E"], d["nu"], d["mat_id"], d["mats"], d["n"], d["dt"],
                      batch_offsets=offsets)
    errs, ref = compare_substep(state0, gpu, grid, params, d["mass"])
    diag = B.mpm_get_diagnostics(ctx)
    return errs, diag, ctx, p


def assert_parity(errs, tol=TOL_SUBSTEP):
    """Norm and element-wise errors of every field within tol, and the
    displacement within its bound."""
    bad = parity_failures(errs, tol)
    assert not bad, f"parity failed: {bad} (all: {errs})"


@pytest.mark.parametrize("N", [1, 2, 63, 257, 5000])
def test_substep_random_mixed_materials(N):
    d = random_scene(100 + N, N)
    errs, diag, _, _ = run_case(d)
    print(N, errs, diag, flush=True)
    assert diag["nonfinite"] == 0 and diag["out_of_grid"] == 0
    assert_parity(errs)


@pytest.mark.parametrize("N", [257, 5000])
def test_substep_all_constitutive_models(N):
    d = random_scene(300 + N, N, mats=MATS_ALL)
    errs, diag, _, _ = run_case(d)
    print(N, errs, diag, flush=True)
    assert diag["nonfinite"] == 0 and diag["out_of_grid"] == 0
    assert_parity(errs)


def test_substep_large_volume_change_models():
    """F = s (I + 0.05 N) with s^3 in [0.01, 2]: the sigma clamp of J acts
    on both sides, the J floors of the Neo-Hookean and volume models do not."""
    N = 3000
    d = random_scene(77, N, mats=MATS_ALL, cgrad=5.0)
    rng = np.random.default_rng(78)
    s = np.cbrt(rng.uniform(0.01, 2.0, N))
    d["F"] = (s[:, None, None] * (np.eye(3) + rng.normal(0, 0.05, (N, 3, 3)))).astype(np.float32)
    J = np.linalg.det(d["F"].astype(np.float64))
    assert (J < 0.05).any() and (J > 1.2).any() and (J > 0).all()
    errs, diag, _, _ = run_case(d)
    print(errs, diag, flush=True)
    assert diag["nonfinite"] == 0 and diag["out_of_grid"] == 0
    assert_parity(errs)


def test_substep_inverted_deformation_gradients():
    """Inverted particles (det F < 0) of every elastic model: the polar
    iteration declines them and the SVD (sign on the last singular value)
    takes over; the J floors of the Neo-Hookean and volume models apply.
    Singular values are kept apart so that U and V are unique."""
    N = 2000
    mats = [dict(elastic=e, plastic=0, yield_stress=0.0, friction_deg=0.0) for e in range(6)]
    d = random_scene(91, N, mats=mats, cgrad=5.0)
    rng = np.random.default_rng(92)
    F = np.empty((N, 3, 3))
    for p in range(N):
        Q1, Q2 = scenes.haar_rotation(rng), scenes.haar_rotation(rng)
        sig = np.array([rng.uniform(1.1, 1.3), rng.uniform(0.85, 1.0), rng.uniform(0.5, 0.7)])
        if p % 2 == 0:
            sig[2] = -sig[2]  # inverted
        F[p] = Q1 @ np.diag(sig) @ Q2.T
    d["F"] = F.astype(np.float32)
    assert (np.linalg.det(F) < 0).sum() == N // 2
    errs, diag, _, _ = run_case(d)
    print(errs, diag, flush=True)
    assert diag["out_of_grid"] == 0
    assert_parity(errs)


def test_substep_after_warmup_cube_lattice():
    sc = scenes.make_scene("cube_lattice")
    d = dict(x=sc.x, v=sc.v, C=sc.C, F=sc.F, mass=sc.mass, vol0=sc.vol0, log_E=sc.log_E, nu=sc.nu,
             mat_id=sc.mat_id, mats=sc.materials, n=sc.grid_res, dt=sc.dt)
    for warm in (0, 50):
        errs, diag, _, _ = run_case(d, warm=warm)
        print(warm, errs, flush=True)
        assert_parity(errs)


def test_substep_global_fallback_matches():
    """tile_cap = 27 forces every chunk onto the global-memory P2G / G2P path."""
    d = random_scene(7, 3000)
    errs, diag, _, _ = run_case(d, tile_cap=27)
    assert diag["tile_overflow"] > 0
    assert_parity(errs)


def test_substep_max_contention_one_cell():
    """All particles inside one cell: every stencil hits the same 27 nodes."""
    rng = np.random.default_rng(3)
    d = random_scene(3, 4096)
    n = d["n"]
    d["x"] = ((16.6 + rng.uniform(0, 0.8, (4096, 3))) / n).astype(np.float32)
    errs, diag, _, _ = run_case(d)
    print(errs, flush=True)
    assert_parity(errs)


def test_substep_non_power_of_two_grid_and_half_cell():
    """n = 48 (x n inexact in float32) and coordinates with x/dx - 0.5 integral."""
    d = random_scene(11, 2000, n=48)
    d["x"][:50] = ((np.floor(d["x"][:50] * 48) + 0.5) / 48).astype(np.float32)
    errs, diag, _, _ = run_case(d)
    assert_parity(errs)


@pytest.mark.parametrize("mode", [dict(grid="dense"), dict(grid="sparse"), dict(deterministic=True)],
                         ids=["dense", "sparse", "deterministic"])
def test_batched_scenes_with_empty_scene(mode):
    """Three scenes, the middle one empty, after 5 warm-up substeps, in
    each grid mode."""
    d1 = random_scene(21, 700, n=24)
    d2 = random_scene(22, 1300, n=24)
    d = {k: (np.concatenate([d1[k], d2[k]]) if isinstance(d1[k], np.ndarray) else d1[k]) for k in d1}
    offsets = [0, 700, 700, 2000]
    errs, diag, _, _ = run_case(d, warm=5, offsets=offsets, **mode)
    assert_parity(errs)


@pytest.mark.parametrize("mode", [dict(grid="dense"), dict(grid="sparse"), dict(deterministic=True)],
                         ids=["dense", "sparse", "deterministic"])
@pytest.mark.parametrize("tile_cap", [0, 64])
def test_substep_modes_after_warmup(mode, tile_cap):
    """A random cloud after 8 warm-up substeps with re-sorts every 3, in each
    grid mode, with the LDS tiles and with nearly every item in global
    memory (tile_cap 64)."""
    d = random_scene(31, 6000, vel=3.0)
    errs, diag, ctx, _ = run_case(d, warm=8, sort_every=3, tile_cap=tile_cap, **mode)
    print(mode, tile_cap, diag, flush=True)
    assert_parity(errs)


def test_sorted_resort_path_matches():
    """Several substeps with a re-sort after every one, then a parity step."""
    d = random_scene(5, 8000, fdev=0.02, cgrad=2.0)
    errs, diag, _, _ = run_case(d, warm=6, sort_every=1)
    assert_parity(errs)


def test_gaussian_cloud_reduced_mixed():
    sc = scenes.make_scene("gaussian_cloud", n_total=40_000)
    d = dict(x=sc.x, v=sc.v, C=sc.C, F=sc.F, mass=sc.mass, vol0=sc.vol0, log_E=sc.log_E, nu=sc.nu,
             mat_id=sc.mat_id, mats=sc.materials, n=sc.grid_res, dt=sc.dt)
    errs, diag, _, _ = run_case(d, warm=200)
    print(errs, diag, flush=True)
    assert_parity(errs)


def test_cube_lattice_100_substeps_positions():
    sc = scenes.make_scene("cube_lattice")
    ctx = B.init_from_scene(sc)
    p = B.Particles.from_scene(sc)
    B.mpm_step_n(ctx, p, 100)
    torch.cuda.synchronize()
    xg = p.state_numpy()[0]
    params = O.Params.from_scene(sc)
    xr = O.step_n(O.state_from_scene(sc), params, 100)[0].numpy()
    err = np.abs(xg - xr).max() / np.abs(xr).max()
    disp = np.linalg.norm((xg - sc.x) - (xr - sc.x)) / np.linalg.norm(xr - sc.x)
    print("x rel", err, "displacement rel", disp, flush=True)
    assert err <= TOL_LONG_X
    assert disp <= 1e-3


def test_item_boxes_handed_between_substeps():
    """Each substep kernel hands the next one a box of its particles' new
    cells: the current box widened by the particles that changed cell.  A
    rigidly translating and spinning cloud moving about 0.3 cells per
    substep changes cells often.  The run without re-sorts, where boxes are
    handed over for all 16 substeps, must match the run that re-sorts every
    substep, where every kernel reads x for its boxes (same physics, other
    item composition: rounding only), and the oracle."""
    N, n, dt = 4000, 32, 1e-4
    d = random_scene(91, N, n=n, dt=dt, cgrad=0.0, fdev=0.02, spread=0.3)
    c = np.array([0.5, 0.5, 0.5], np.float32)
    speed = 0.3 / n / dt  # 0.3 cells per substep
    omega = np.array([0.0, 0.0, 1.0], np.float32) * (speed / 0.15) * 0.3
    d["v"] = (np.array([0.6, 0.3, -0.5], np.float32) * speed + np.cross(omega, d["x"] - c)).astype(np.float32)
    outs = []
    for se in (1, 64):
        ctx = B.mpm_init(n, dt, d["mats"], N, None, sort_every=se)
        p = B.Particles.from_arrays(d["x"], d["v"], d["C"], d["F"], d["mass"], d["vol0"], d["log_E"], d["nu"],
                                    d["mat_id"])
        B.mpm_step_n(ctx, p, 16)
        torch.cuda.synchronize()
        diag = B.mpm_get_diagnostics(ctx)
        assert diag["nonfinite"] == 0 and diag["out_of_grid"] == 0, diag
        outs.append(p.state_numpy())
    moved = np.abs(outs[1][0] - d["x"]).max() * n
    assert moved > 3.0, moved  # particles crossed several cells
    s_v = float(np.abs(outs[0][1]).max())
    floors = (1.0 / n, s_v, s_v * n, 1.0)
    for k in range(4):
        e = (rel_err(outs[1][k], outs[0][k], floors[k]), elem_err(outs[1][k], outs[0][k], floors[k]))
        print("handed-over vs box pass", k, e, flush=True)
        assert max(e) <= 1e-5, (k, e)
    params = O.Params(d["mass"], d["vol0"], d["log_E"], d["nu"], d["mat_id"], d["mats"], n, dt)
    s0 = tuple(torch.as_tensor(np.asarray(a, np.float64)) for a in (d["x"], d["v"], d["C"], d["F"]))
    xr = O.step_n(s0, params, 16)[0].numpy()
    e = (rel_err(outs[1][0], xr, 1.0 / n), np.abs(outs[1][0] - xr).max() / np.abs(xr).max())
    print("vs oracle x", e, flush=True)
    assert max(e) <= TOL_LONG_X


def test_zero_particles_and_zero_steps():
    ctx = B.mpm_init(16, 1e-4, MATS_MIXED[:1], 0)
    p = B.Particles.from_arrays(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3, 3)), np.zeros((0, 3, 3)),
                                np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0, np.int32))
    B.mpm_step_n(ctx, p, 5)
    d = random_scene(1, 10, n=16)
    ctx = B.mpm_init(16, 1e-4, MATS_MIXED, 10)
    p = B.Particles.from_arrays(d["x"], d["v"], d["C"], d["F"], d["mass"], d["vol0"], d["log_E"], d["nu"],
                                d["mat_id"])
    before = p.state_numpy()
    B.mpm_step_n(ctx, p, 0)
    after = p.state_numpy()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)


def test_covariance_export():
    rng = np.random.default_rng(0)
    N = 1000
    F = (np.eye(3) + rng.normal(0, 0.1, (N, 3, 3))).astype(np.float32)
    q = rng.normal(0, 1, (N, 3, 3))
    S = (q @ q.transpose(0, 2, 1) * 1e-4).astype(np.float32)
    cov0 = np.stack([S[:, 0, 0], S[:, 0, 1], S[:, 0, 2], S[:, 1, 1], S[:, 1, 2], S[:, 2, 2]], 0)
    ctx = B.mpm_init(16, 1e-4, MATS_MIXED[:1], 0)
    Ft = torch.tensor(F.reshape(N, 9).T.copy()).cuda()
    c0 = torch.tensor(cov0.copy()).cuda()
    out = torch.empty(6, N, device="cuda")
    B.mpm_export_covariance(ctx, Ft, c0, out)
    ref = O.covariance(torch.tensor(F, dtype=torch.float64), cov0.T).numpy()
    assert rel_err(out.cpu().numpy().T, ref, 1e-6) < 1e-6
