"""Failure detection and state handling through the C ABI.  Every failing
condition is forced from host-side inputs; the kernels bounds-check every
access, so a bad particle is counted and skipped, never dereferenced."""
import math

import numpy as np
import pytest
import torch

from paper_2602_01723_amd import binding as B
from paper_2602_01723_amd import scenes

pytestmark = pytest.mark.gpu


def _cube(**kw):
    sc = scenes.make_scene("cube_lattice", per_axis=12, **kw)
    return sc


def test_nan_in_F_is_counted_and_isolated():
    sc = _cube()
    F = sc.F.copy()
    F[7, 1, 1] = np.nan
    ctx = B.init_from_scene(sc)
    p = B.Particles.from_arrays(sc.x, sc.v, sc.C, F, sc.mass, sc.vol0, sc.log_E, sc.nu, sc.mat_id)
    B.mpm_step_n(ctx, p, 3)
    d = B.mpm_get_diagnostics(ctx)
    assert d["nonfinite"] >= 1 and d["status"] == B.MPM_EUNSTABLE
    x, v, C, Fo = p.state_numpy()
    others = np.ones(sc.n, bool)
    others[7] = False
    assert np.isfinite(x[others]).all() and np.isfinite(Fo[others]).all()  # the grid stayed clean


def test_particle_outside_stencil_box_is_counted_and_skipped():
    sc = _cube()
    x = sc.x.copy()
    x[3] = (0.01, 0.5, 0.5)  # base cell -1: its stencil would leave the grid
    ctx = B.init_from_scene(sc)
    p = B.Particles.from_arrays(x, sc.v, sc.C, sc.F, sc.mass, sc.vol0, sc.log_E, sc.nu, sc.mat_id)
    B.mpm_step_n(ctx, p, 2)
    d = B.mpm_get_diagnostics(ctx)
    assert d["out_of_grid"] >= 1 and d["status"] == B.MPM_EUNSTABLE
    xo = p.state_numpy()[0]
    assert np.array_equal(xo[3], x[3])  # left where it was
    assert np.isfinite(xo).all()


def test_overstiff_material_trips_the_cfl_watch_before_it_blows_up():
    """E0 = 3e10 (the paper's failing initial guess) with dt = 1e-4 violates
    the elastic CFL bound by orders of magnitude.  The wave-speed figure says
    so from the start; the velocity watch (|v'| dt / dx > 1/2) trips in a
    substep at which every particle is still finite and on the grid, and the
    run blows up later."""
    sc = _cube(E=3e10)
    v = sc.v.copy()
    v[:, 1] = -2.0
    ctx = B.init_from_scene(sc)
    p = B.Particles.from_arrays(sc.x, v, sc.C, sc.F, sc.mass, sc.vol0, sc.log_E, sc.nu, sc.mat_id)
    tripped_at, blown_at = None, None
    for k in range(1, 201):
        B.mpm_step_n(ctx, p, 1)
        d = B.mpm_get_diagnostics(ctx)
        if k == 1:
            assert d["max_wave_cfl"] > 10.0, d  # c dt / dx of E = 3e10
        if tripped_at is None and d["cfl_violations"] > 0:
            tripped_at = k
            print("CFL watch tripped at substep", k, d, flush=True)
            assert d["nonfinite"] == 0 and d["out_of_grid"] == 0 and d["status"] == B.MPM_EUNSTABLE, d
            assert np.isfinite(p.state_numpy()[0]).all()
        if d["nonfinite"] + d["out_of_grid"] > 0:
            blown_at = k
            break
    print("blown up at substep", blown_at, d, flush=True)
    assert tripped_at is not None and (blown_at is None or tripped_at < blown_at)


def test_cfl_figures_of_a_free_fall():
    """A lattice cube at rest with F = I falls freely (no stress): after k
    substeps every particle has |v| = k dt g, so the largest |v| dt / dx is
    k dt^2 g n; the P-wave figure is sqrt((lam + 2 mu) V0 / m) dt n."""
    sc = _cube()
    ctx = B.init_from_scene(sc)
    p = B.Particles.from_scene(sc)
    k = 12
    B.mpm_step_n(ctx, p, k)
    d = B.mpm_get_diagnostics(ctx)
    n, dt = sc.grid_res, sc.dt
    want = k * dt * dt * 9.8 * n
    E, nu = math.exp(float(sc.log_E[0])), float(sc.nu[0])
    c = math.sqrt(E * (1 - nu) / ((1 + nu) * (1 - 2 * nu)) * float(sc.vol0[0]) / float(sc.mass[0]))
    print(d, want, c * dt * n, flush=True)
    assert d["status"] == B.MPM_OK and d["cfl_violations"] == 0
    assert abs(d["max_cfl"] - want) <= 1e-5 * want
    assert abs(d["max_wave_cfl"] - c * dt * n) <= 1e-6 * c * dt * n


def test_resume_matches_one_long_call():
    sc = scenes.make_scene("gaussian_cloud", n_total=20_000)
    ctx = B.init_from_scene(sc)
    a = B.Particles.from_scene(sc)
    b = B.Particles.from_scene(sc)
    B.mpm_step_n(ctx, a, 30)
    B.mpm_step_n(ctx, b, 15)
    B.mpm_step_n(ctx, b, 15)
    xa, xb = a.state_numpy()[0], b.state_numpy()[0]
    disp = np.linalg.norm(xa - sc.x)
    assert np.linalg.norm(xa - xb) <= 1e-4 * disp


def test_tuning_validation():
    sc = _cube()
    ctx = B.init_from_scene(sc)
    for bad in (dict(chunk=100), dict(chunk=32), dict(tile_cap=5000), dict(sort_every=-1), dict(workgroups=-2)):
        with pytest.raises(B.MPMError) as e:
            B.mpm_set_tuning(ctx, **bad)
        assert e.value.status == B.MPM_EINVAL
    B.mpm_set_tuning(ctx, chunk=512, sort_every=4, tile_cap=729, workgroups=1024)
    t = B.mpm_get_tuning(ctx)
    assert (t["chunk"], t["sort_every"], t["tile_cap"], t["workgroups"]) == (512, 4, 729, 1024)
    p = B.Particles.from_scene(sc)
    B.mpm_step_n(ctx, p, 5)  # runs with the new settings
    assert B.mpm_get_diagnostics(ctx)["status"] == B.MPM_OK


def test_profile_counts_launches_by_class():
    sc = _cube()
    ctx = B.init_from_scene(sc)
    p = B.Particles.from_scene(sc)
    B.mpm_step_n(ctx, p, 2)
    torch.cuda.synchronize()
    B.mpm_profile(ctx, True)
    B.mpm_profile_read(ctx)  # reset
    B.mpm_step_n(ctx, p, 10)
    torch.cuda.synchronize()
    prof = B.mpm_profile_read(ctx)
    B.mpm_profile(ctx, False)
    # one P2G-only launch, fused launches for the rest, one G2P-only launch
    assert prof["p2g_only"][1] == 1 and prof["g2p_only"][1] == 1
    assert prof["fused_substep"][1] == 9
    assert all(ms > 0.0 for ms, n in prof.values() if n)
    assert prof["caller_io"][1] >= 2  # gather from and scatter back to the caller's order
    B.mpm_step_n(ctx, p, 3)
    torch.cuda.synchronize()
    assert all(n == 0 for _, n in B.mpm_profile_read(ctx).values())  # disabled: nothing recorded


def test_position_loss_cotangent_closed_form():
    rng = np.random.default_rng(31)
    N = 5000
    sc = _cube()
    x = torch.tensor(rng.uniform(0, 1, (3, N)).astype(np.float32)).cuda()
    xt = torch.tensor(rng.uniform(0, 1, (3, N)).astype(np.float32)).cuda()
    w = torch.tensor(rng.uniform(0.5, 2.0, N).astype(np.float32)).cuda()
    g = torch.empty(3, N, device="cuda")
    ctx = B.mpm_init(16, 1e-4, sc.materials, N)
    B.mpm_position_loss_grad(ctx, x, xt, w, g)
    torch.cuda.synchronize()
    assert torch.allclose(g, 2.0 * w * (x - xt), rtol=1e-6, atol=1e-7)
