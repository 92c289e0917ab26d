"""Caller-order I/O through the C ABI.  The library keeps particles sorted by
cell and moves every per-particle array between the caller's order and its
own with a bucketed two-pass permutation (positions by destination bucket,
then each bucket placed in LDS).  The caller's order must not change the
result, and the state a substep carries over unchanged must come back bit
for bit.  Sizes span one bucket and tile (N < 4096), several of each, and a
ragged last bucket and tile."""
import numpy as np
import pytest

from paper_2602_01723_amd import binding as B
from paper_2602_01723_amd import scenes

pytestmark = pytest.mark.gpu


def _run(sc, order, n_steps):
    ctx = B.init_from_scene(sc)
    p = B.Particles.from_arrays(sc.x[order], sc.v[order], sc.C[order], sc.F[order], sc.mass[order],
                                sc.vol0[order], sc.log_E[order], sc.nu[order], sc.mat_id[order])
    B.mpm_step_n(ctx, p, n_steps)
    inv = np.argsort(order)
    return [a[inv] for a in p.state_numpy()], B.mpm_get_diagnostics(ctx)


@pytest.mark.parametrize("n_total", [3000, 41000, 120000])
def test_result_does_not_depend_on_caller_order(n_total):
    sc = scenes.make_scene("gaussian_cloud", n_total=n_total)
    rng = np.random.default_rng(n_total)
    ident = np.arange(sc.n)
    shuffled = rng.permutation(sc.n)
    reversed_ = ident[::-1].copy()
    ref, d0 = _run(sc, ident, 4)
    assert d0["nonfinite"] == 0 and d0["out_of_grid"] == 0
    # natural scales (as in the parity metric): dx, a velocity, velocity / dx, 1
    s_v = max(float(np.abs(ref[1]).max()), 9.8 * sc.dt)
    floors = (1.0 / sc.grid_res, s_v, s_v * sc.grid_res, 1.0)
    for order in (shuffled, reversed_):
        out, _ = _run(sc, order, 4)
        for k, (a, b) in enumerate(zip(out, ref)):
            # only the order of floating-point sums differs (grid atomics)
            scale = max(float(np.abs(b).max()), floors[k])
            assert np.abs(a - b).max() <= 2e-5 * scale, (k, np.abs(a - b).max(), scale)


def test_skipped_particles_come_back_bit_for_bit():
    """Particles whose stencil leaves the grid are carried over unchanged:
    their x, v, C and F after a call equal the input exactly, whatever
    slots the sort gave them."""
    sc = scenes.make_scene("gaussian_cloud", n_total=20000)
    rng = np.random.default_rng(5)
    order = rng.permutation(sc.n)
    x = sc.x.copy()
    out_idx = rng.choice(sc.n, 37, replace=False)
    x[out_idx, 0] = 0.002 + 0.001 * rng.random(37)  # below the first base cell
    ctx = B.init_from_scene(sc)
    p = B.Particles.from_arrays(x[order], sc.v[order], sc.C[order], sc.F[order], sc.mass[order], sc.vol0[order],
                                sc.log_E[order], sc.nu[order], sc.mat_id[order])
    B.mpm_step_n(ctx, p, 3)
    d = B.mpm_get_diagnostics(ctx)
    assert d["out_of_grid"] >= 37
    inv = np.argsort(order)
    xo, vo, Co, Fo = [a[inv] for a in p.state_numpy()]
    assert np.array_equal(xo[out_idx], x[out_idx])
    assert np.array_equal(vo[out_idx], sc.v[out_idx])
    assert np.array_equal(Co[out_idx], sc.C[out_idx])
    assert np.array_equal(Fo[out_idx], sc.F[out_idx])


def test_large_n_unstaged_first_pass():
    """Above 2048 destination buckets (N > 2^23) the first pass of the
    permutation writes scattered instead of staging tiles in LDS.  9 M random
    particles, one substep, identity vs shuffled caller order."""
    N, n, dt = 9_000_000, 128, 5e-5
    rng = np.random.default_rng(2024)
    x, v, C, F = scenes.random_state(rng, N, n, spread=0.3, vel=0.2, cgrad=1.0, fdev=0.02)
    mass = np.full(N, 1e-6, np.float32)
    vol0 = np.full(N, 1e-9, np.float32)
    log_E = np.full(N, np.log(1e5), np.float32)
    nu = np.full(N, 0.3, np.float32)
    mat = np.zeros(N, np.int32)
    mats = [dict(elastic=0, plastic=0, yield_stress=0.0, friction_deg=0.0)]
    outs = []
    for order in (np.arange(N), rng.permutation(N)):
        ctx = B.mpm_init(n, dt, mats, N, None)
        p = B.Particles.from_arrays(x[order], v[order], C[order], F[order], mass[order], vol0[order], log_E[order],
                                    nu[order], mat[order])
        B.mpm_step_n(ctx, p, 2)
        d = B.mpm_get_diagnostics(ctx)
        assert d["nonfinite"] == 0 and d["out_of_grid"] == 0, d
        inv = np.argsort(order)
        outs.append([a[inv] for a in p.state_numpy()])
        del ctx, p
    s_v = max(float(np.abs(outs[0][1]).max()), 9.8 * dt)
    floors = (1.0 / n, s_v, s_v * n, 1.0)
    for k in range(4):
        scale = max(float(np.abs(outs[0][k]).max()), floors[k])
        assert np.abs(outs[1][k] - outs[0][k]).max() <= 2e-5 * scale, k
