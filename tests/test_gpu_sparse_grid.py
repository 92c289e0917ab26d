"""Block-sparse grid activity (MPM_FLAG_GRID_SPARSE) through the C ABI.

The substeps flag the 4^3-node blocks they add mass to and clear only the
flagged blocks of a buffer before it is written again.  A block holding mass
that escaped the flags would leave stale mass in a buffer three substeps
later, which moves particles: so the sparse runs are checked against the
dense runs (to the rounding of the grid atomics) and against the oracle,
with particles crossing the domain, calls split, re-sorts, the resident
path and batched scenes, and on a large, mostly empty domain."""
import numpy as np
import pytest
import torch

from oracle import mpm_oracle as O
from paper_2602_01723_amd import binding as B
from paper_2602_01723_amd import scenes
from tests.parity import TOL_SUBSTEP, compare_substep, parity_failures, rel_err

pytestmark = pytest.mark.gpu


def fast_cloud(n=6000, grid_res=40, seed=3):
    """A cloud that crosses blocks: a uniform velocity of about 16 m/s plus
    a spin, so particles move up to about 0.08 cell per substep into fresh
    blocks."""
    rng = np.random.default_rng(seed)
    sc = scenes.make_scene("gaussian_cloud", n_total=n, grid_res=grid_res)
    c = sc.x.mean(0)
    r = sc.x - c
    spin = np.stack([-r[:, 1], r[:, 0], np.zeros(len(r))], 1) * 30.0
    sc.v = (np.array([12.0, 6.0, -9.0]) + spin + rng.normal(0, 0.1, sc.x.shape)).astype(np.float32)
    return sc


def run(sc, steps, grid, calls=None, sort_every=5):
    print(f"sparse grid: N={sc.n} n={sc.grid_res} steps={steps} grid={grid} calls={calls}", flush=True)
    ctx = B.init_from_scene(sc, sort_every=sort_every, grid=grid)
    p = B.Particles.from_scene(sc)
    for k in (calls or [steps]):
        B.mpm_step_n(ctx, p, k)
    torch.cuda.synchronize()
    d = B.mpm_get_diagnostics(ctx)
    assert d["nonfinite"] == 0 and d["out_of_grid"] == 0, d
    return p.state_numpy()


def assert_close(a, b, sc, tol=1e-5):
    s_v = max(float(np.abs(b[1]).max()), 9.8 * sc.dt)
    floors = (1.0 / sc.grid_res, s_v, s_v * sc.grid_res, 1.0)
    for k in range(4):
        e = rel_err(a[k], b[k], floors[k])
        print("sparse vs dense", "xvCF"[k], e, flush=True)
        assert e <= tol, ("xvCF"[k], e)


def test_one_substep_matches_the_oracle():
    sc = fast_cloud(4000)
    got = run(sc, 1, "sparse")
    errs, _ = compare_substep((sc.x, sc.v, sc.C, sc.F), got, None, O.Params.from_scene(sc), sc.mass)
    assert not parity_failures(errs, TOL_SUBSTEP), errs


@pytest.mark.parametrize("calls", [None, [7, 5, 1, 11]])
def test_particles_crossing_blocks_match_the_dense_grid(calls):
    """40 substeps, whole or split into calls (each call starts from a fresh
    P2G into buffers the previous call left)."""
    sc = fast_cloud()
    steps = 40 if calls is None else sum(calls)
    a = run(sc, steps, "sparse", calls)
    b = run(sc, steps, "dense", calls)
    assert np.abs(a[0] - sc.x).max() > 1.5 / sc.grid_res  # particles crossed into other blocks
    assert_close(a, b, sc, 1e-4)


def test_resident_and_batched_match_the_dense_grid():
    sc = scenes.make_scene("candidate_batch", n_batch=3, grid_res=32, n_min=1500, n_max=4000)
    outs = []
    for grid in ("sparse", "dense"):
        ctx = B.init_from_scene(sc, sort_every=4, grid=grid)
        p = B.Particles.from_scene(sc)
        B.mpm_load(ctx, p)
        for k in (9, 13):
            B.mpm_advance(ctx, k)
        B.mpm_store(ctx, p)
        torch.cuda.synchronize()
        outs.append(p.state_numpy())
    assert_close(outs[0], outs[1], sc, 1e-4)


def test_large_mostly_empty_domain():
    """30,000 particles in a 256^3 grid (16.8 M nodes, default: sparse),
    against the dense grid after 30 substeps, and the sparse run faster."""
    sc = scenes.make_scene("gaussian_cloud", n_total=30_000, grid_res=256, dt=2e-5)
    ms = {}
    outs = {}
    for grid in ("auto", "dense"):
        ctx = B.init_from_scene(sc, sort_every=8, grid=grid)
        p = B.Particles.from_scene(sc)
        B.mpm_load(ctx, p)
        B.mpm_advance(ctx, 2)
        torch.cuda.synchronize()
        B.mpm_profile(ctx, True)
        B.mpm_profile_read(ctx)
        B.mpm_advance(ctx, 28)
        torch.cuda.synchronize()
        t, n = B.mpm_profile_read(ctx)["fused_substep"]
        ms[grid] = t / n
        B.mpm_store(ctx, p)
        torch.cuda.synchronize()
        outs[grid] = p.state_numpy()
    print("fused substep ms: sparse", ms["auto"], "dense", ms["dense"], flush=True)
    assert_close(outs["auto"], outs["dense"], sc, 1e-4)
    assert ms["auto"] < ms["dense"]


def corner_cloud(n=6000, grid_res=38):
    """A cloud pressed into the upper corner of a 38^3 grid, whose last 4^3
    block on each axis is partial (nodes 36-37): moving at +6 m/s per axis,
    particles reach the sticky wall band there."""
    sc = scenes.make_scene("gaussian_cloud", n_total=n, grid_res=grid_res)
    sc.x = (sc.x + (0.9 - sc.x.max(0))).astype(np.float32)
    rng = np.random.default_rng(5)
    sc.v = (np.array([6.0, 6.0, 6.0]) + rng.normal(0, 0.1, sc.x.shape)).astype(np.float32)
    return sc


def test_partial_edge_blocks_match_the_dense_grid_and_the_oracle():
    sc = corner_cloud()
    errs, _ = compare_substep((sc.x, sc.v, sc.C, sc.F), run(sc, 1, "sparse"), None, O.Params.from_scene(sc), sc.mass)
    assert not parity_failures(errs, TOL_SUBSTEP), errs
    a = run(sc, 40, "sparse", [13, 27])
    b = run(sc, 40, "dense", [13, 27])
    assert a[0].max() > 34.5 / sc.grid_res  # base cell 34: stencils reach node 36 of the partial blocks
    assert_close(a, b, sc, 1e-4)
