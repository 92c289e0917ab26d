"""Deterministic mode (MPM_FLAG_DETERMINISTIC) through the C ABI.

With the flag the forward state is a function of the inputs alone: the P2G
sums are 64-bit integers at one fixed-point scale per scene (exact in any
order of the atomics), each cell's particles are ordered by index at
every sort, and the stress is taken from the stored float32 F.  Checked bit
for bit: repeated runs, the caller's particle order permuted, resident and
mpm_step_n runs split into calls against one call, a stored state loaded
into a new context, a batched context against each scene alone, and
fixed-point scales predicted from a different state.  The mode keeps the substep's parity with the
oracle, and its state stays within rounding of the default mode."""
import numpy as np
import pytest
import torch

from oracle import mpm_oracle as O
from paper_2602_01723_amd import batch as BT
from paper_2602_01723_amd import binding as B
from paper_2602_01723_amd import scenes
from tests.parity import TOL_SUBSTEP, compare_substep, parity_failures, rel_err

pytestmark = pytest.mark.gpu


def state_bits(p):
    return [a.view(np.uint32) for a in p.state_numpy()]


def assert_same_bits(a, b, what):
    for k, (x, y) in enumerate(zip(a, b)):
        diff = int(np.count_nonzero(x != y))
        assert diff == 0, f"{what}: field {'xvCF'[k]} differs in {diff} entries"


def pair_scene(n=40_000):
    """Two ellipsoids colliding at +-1 m/s (contact, particles crossing
    item boxes), 48^3 grid, with a von Mises half so a return map runs."""
    sc = scenes.make_scene("colliding_pair", n_total=n, grid_res=48)
    sc.materials = [dict(sc.materials[0]), scenes._material(scenes.ELASTIC_HENCKY, scenes.PLASTIC_VON_MISES, 2e3)]
    sc.mat_id = np.where(np.arange(sc.n) < sc.n // 2, 0, 1).astype(np.int32)
    return sc


def run_step_n(sc, n_steps, det=True, order=None, sort_every=6, tile_cap=0):
    order = np.arange(sc.n) if order is None else order
    print(f"determinism: step_n N={sc.n} steps={n_steps} det={det} tile_cap={tile_cap}", flush=True)
    ctx = B.init_from_scene(sc, sort_every=sort_every, deterministic=det)
    if tile_cap:
        B.mpm_set_tuning(ctx, tile_cap=tile_cap)
    p = B.Particles.from_arrays(sc.x[order], sc.v[order], sc.C[order], sc.F[order], sc.mass[order],
                                sc.vol0[order], sc.log_E[order], sc.nu[order], sc.mat_id[order])
    B.mpm_step_n(ctx, p, n_steps)
    torch.cuda.synchronize()
    d = B.mpm_get_diagnostics(ctx)
    assert d["nonfinite"] == 0 and d["out_of_grid"] == 0 and d["order_fallbacks"] == 0, d
    return p, d


@pytest.mark.parametrize("tile_cap", [0, 64])
def test_repeated_runs_are_bitwise_equal(tile_cap):
    """Two runs from the same input; with tile_cap = 64 nearly every item
    exceeds its LDS tiles, so G2P reads and P2G adds node by node in global
    memory (the 64-bit fixed-point grid directly)."""
    sc = pair_scene()
    a, da = run_step_n(sc, 40, tile_cap=tile_cap)
    b, _ = run_step_n(sc, 40, tile_cap=tile_cap)
    if tile_cap:
        assert da["tile_overflow"] > 0
    assert_same_bits(state_bits(a), state_bits(b), "two runs")


def test_caller_order_does_not_change_the_bits():
    """The caller's particle order changes the atomics' order and the
    counting sort's slots; the deterministic sort orders each cell by index,
    and the state in caller order must come out the same."""
    sc = pair_scene(30_000)
    order = np.random.default_rng(5).permutation(sc.n)
    a, _ = run_step_n(sc, 30)
    b, _ = run_step_n(sc, 30, order=order)
    inv = np.argsort(order)
    bs = [x[inv] for x in state_bits(b)]
    # the within-cell order follows the caller index, which the permutation
    # changes, so the grouping of particles into items differs: the P2G sums
    # are exact either way, and every per-particle path must agree bitwise
    assert_same_bits(state_bits(a), bs, "caller order")


def test_resident_calls_split_equal_one_call():
    """mpm_advance(12) + mpm_advance(8) against mpm_advance(20), re-sorting
    every 6 substeps across the call boundary."""
    sc = pair_scene(30_000)
    outs = []
    for splits in ((12, 8), (20,)):
        ctx = B.init_from_scene(sc, sort_every=6, deterministic=True)
        p = B.Particles.from_scene(sc)
        B.mpm_load(ctx, p)
        for n in splits:
            B.mpm_advance(ctx, n)
        B.mpm_store(ctx, p)
        torch.cuda.synchronize()
        outs.append(state_bits(p))
    assert_same_bits(outs[0], outs[1], "split resident run")


def test_step_n_calls_split_equal_one_call():
    """mpm_step_n(12) then mpm_step_n(18) on the same arrays against one
    mpm_step_n(30): the second call sorts the stored state afresh and starts
    with a P2G-only launch from the stored float32 state, which in
    deterministic mode is what the fused launch computes as well."""
    sc = pair_scene(30_000)
    a, _ = run_step_n(sc, 30)
    ctx = B.init_from_scene(sc, sort_every=6, deterministic=True)
    p = B.Particles.from_scene(sc)
    B.mpm_step_n(ctx, p, 12)
    B.mpm_step_n(ctx, p, 18)
    torch.cuda.synchronize()
    assert_same_bits(state_bits(a), state_bits(p), "mpm_step_n 12 + 18")


def test_store_and_load_into_a_new_context_resume_bitwise():
    """mpm_advance(10), mpm_store, a new context, mpm_load, mpm_advance(10)
    against mpm_advance(20) in one context."""
    sc = pair_scene(30_000)
    outs = []
    ctx = B.init_from_scene(sc, sort_every=6, deterministic=True)
    p = B.Particles.from_scene(sc)
    B.mpm_load(ctx, p)
    B.mpm_advance(ctx, 20)
    B.mpm_store(ctx, p)
    torch.cuda.synchronize()
    outs.append(state_bits(p))
    q = B.Particles.from_scene(sc)
    c1 = B.init_from_scene(sc, sort_every=6, deterministic=True)
    B.mpm_load(c1, q)
    B.mpm_advance(c1, 10)
    B.mpm_store(c1, q)
    c2 = B.init_from_scene(sc, sort_every=6, deterministic=True)
    B.mpm_load(c2, q)
    B.mpm_advance(c2, 10)
    B.mpm_store(c2, q)
    torch.cuda.synchronize()
    outs.append(state_bits(q))
    assert_same_bits(outs[0], outs[1], "store + load resume")


def test_batched_context_equals_each_scene_alone():
    """Three candidate scenes of different sizes in one context against
    each in a context of its own, through mpm_step_n and through the
    resident path."""
    sc = scenes.make_scene("candidate_batch", n_batch=3, grid_res=32, n_min=3000, n_max=9000)
    off = sc.batch_offsets
    batched, _ = run_step_n(sc, 25)
    got = state_bits(batched)
    for b in range(3):
        alone, _ = run_step_n(sc.subset(b), 25)
        assert_same_bits([g[off[b]:off[b + 1]] for g in got], state_bits(alone), f"scene {b}, step_n")
    ctx = B.init_from_scene(sc, sort_every=6, deterministic=True)
    p = B.Particles.from_scene(sc)
    B.mpm_load(ctx, p)
    B.mpm_advance(ctx, 25)
    B.mpm_store(ctx, p)
    torch.cuda.synchronize()
    res = state_bits(p)
    for b in range(3):
        sub = sc.subset(b)
        c1 = B.init_from_scene(sub, sort_every=6, deterministic=True)
        q = B.Particles.from_scene(sub)
        B.mpm_load(c1, q)
        B.mpm_advance(c1, 25)
        B.mpm_store(c1, q)
        torch.cuda.synchronize()
        assert_same_bits([r[off[b]:off[b + 1]] for r in res], state_bits(q), f"scene {b}, resident")


def test_predicted_scales_that_miss_are_redone():
    """After its first P2G launch a context takes each launch's fixed-point
    scales from the previous launch's bounds while it measures this
    launch's, and scatters a scene again from the stored state when its
    measured scale differs.  A context that first ran a copy of the batch in
    which scene 1 moves 20x faster (bounds about 20x larger) predicts wrong
    scales for scene 1 of the real batch: the state must equal fresh
    contexts' of each scene alone bit for bit, with the miss counted."""
    import copy
    sc = scenes.make_scene("candidate_batch", n_batch=3, grid_res=32, n_min=3000, n_max=9000)
    off = sc.batch_offsets
    fast = copy.deepcopy(sc)
    fast.v[off[1]:off[2]] *= 20.0
    fast.C[off[1]:off[2]] *= 20.0
    print("determinism: primed by a faster scene 1", flush=True)
    ctx = B.init_from_scene(sc, sort_every=6, deterministic=True)
    pf = B.Particles.from_scene(fast)
    B.mpm_step_n(ctx, pf, 2)
    torch.cuda.synchronize()
    r0 = B.mpm_get_diagnostics(ctx)["det_rescales"]
    p = B.Particles.from_scene(sc)
    B.mpm_step_n(ctx, p, 25)
    torch.cuda.synchronize()
    d = B.mpm_get_diagnostics(ctx)
    print("rescales while priming", r0, "in the run", d["det_rescales"] - r0, flush=True)
    assert d["det_rescales"] > r0
    got = state_bits(p)
    for b in range(3):
        alone, da = run_step_n(sc.subset(b), 25)
        print(f"scene {b} alone: rescales {da['det_rescales']} in 26 P2G launches", flush=True)
        assert_same_bits([g[off[b]:off[b + 1]] for g in got], state_bits(alone), f"scene {b} after priming")


def test_grid_not_a_multiple_of_four():
    """A 38^3 grid (partial 4^3 blocks at the upper faces, where the cloud
    is pressed against the sticky walls): two runs bitwise equal, and one
    substep against the oracle."""
    sc = scenes.make_scene("gaussian_cloud", n_total=6000, grid_res=38)
    sc.x = (sc.x + (0.9 - sc.x.max(0))).astype(np.float32)
    sc.v = np.tile(np.array([[6.0, 6.0, 6.0]], np.float32), (sc.n, 1))
    a, _ = run_step_n(sc, 30)
    b, _ = run_step_n(sc, 30)
    assert_same_bits(state_bits(a), state_bits(b), "38^3 grid")
    one, _ = run_step_n(sc, 1)
    errs, _ = compare_substep((sc.x, sc.v, sc.C, sc.F), one.state_numpy(), None, O.Params.from_scene(sc), sc.mass)
    assert not parity_failures(errs, TOL_SUBSTEP), errs


def test_deterministic_substep_matches_the_oracle():
    """One substep in deterministic mode against the oracle, to the same
    element-wise bar as the default mode."""
    sc = pair_scene(8_000)
    p, _ = run_step_n(sc, 1)
    errs, _ = compare_substep((sc.x, sc.v, sc.C, sc.F), p.state_numpy(), None, O.Params.from_scene(sc), sc.mass)
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert not parity_failures(errs, TOL_SUBSTEP), errs


def test_deterministic_state_is_close_to_the_default_mode():
    sc = pair_scene(30_000)
    a, _ = run_step_n(sc, 30, det=True)
    b, _ = run_step_n(sc, 30, det=False)
    xa, xb = a.state_numpy()[0], b.state_numpy()[0]
    da, db = xa - sc.x, xb - sc.x
    e = rel_err(da, db, 1e-30)
    print("displacement rel diff det vs default", e, flush=True)
    assert e <= 1e-4


def test_deterministic_backward_runs_and_matches_the_default_mode():
    """The taped forward and mpm_backward in deterministic mode (the
    recompute uses the deterministic launches): the parameter gradients
    agree with the default mode's within the rounding of the forward."""
    sc = pair_scene(8_000)
    grads = []
    for det in (True, False):
        ctx = B.init_from_scene(sc, sort_every=6, deterministic=det)
        p = B.Particles.from_scene(sc)
        tape = torch.empty(B.mpm_tape_size(ctx, 12, 4) // 4 + 64, dtype=torch.float32, device="cuda")
        B.mpm_step_n(ctx, p, 12, tape=tape, checkpoint_every=4)
        gl, gn = torch.empty(sc.n, device="cuda"), torch.empty(sc.n, device="cuda")
        B.mpm_backward(ctx, p, tape, 12, g_x=torch.ones_like(p.x), g_log_E=gl, g_nu=gn)
        torch.cuda.synchronize()
        grads.append((gl.cpu().numpy(), gn.cpu().numpy()))
    for a, b in zip(*grads):
        e = rel_err(a, b, 1e-30)
        print("gradient rel diff", e, flush=True)
        assert e <= 1e-3


def test_batched_graph_gradients_equal_plain_bitwise():
    """The batched forward + loss + adjoint, captured into one hipGraph and
    replayed, against its eager run and against each candidate evaluated
    alone: with the deterministic adjoint scatter (exact fixed-point sums of
    the grid-velocity adjoint per scene) every gradient agrees bit for bit."""
    sc = scenes.make_scene("candidate_batch", n_batch=3, grid_res=32, n_min=3000, n_max=9000)
    steps, K = 30, 10
    tl = BT.per_particle(sc.extras["target_log_E"], sc.batch_offsets)
    tn = BT.per_particle(sc.extras["target_nu"], sc.batch_offsets)
    xt = BT.target_positions(sc, steps, tl, tn, deterministic=True)
    ev = BT.Evaluation(sc, steps, K, xt, deterministic=True)
    ev.run_eager()
    torch.cuda.synchronize()
    gl_e, gn_e = (g.copy() for g in ev.gradients())
    assert np.all(np.isfinite(gl_e)) and np.abs(gl_e).max() > 0
    ev.capture()
    for rep in range(2):
        ev.run_graph()
        torch.cuda.synchronize()
        gl, gn = ev.gradients()
        assert np.array_equal(gl.view(np.uint32), gl_e.view(np.uint32)), f"replay {rep}: log E gradients differ"
        assert np.array_equal(gn.view(np.uint32), gn_e.view(np.uint32)), f"replay {rep}: nu gradients differ"
        _ = torch.ones(1000, device="cuda").sum().item()
    off = sc.batch_offsets
    for b, pe in enumerate(BT.plain_evaluations(sc, steps, K, xt, deterministic=True)):
        pe.run_eager()
        torch.cuda.synchronize()
        g1, n1 = pe.gradients()
        lo, hi = off[b], off[b + 1]
        d1 = int(np.count_nonzero(g1.view(np.uint32) != gl_e[lo:hi].view(np.uint32)))
        d2 = int(np.count_nonzero(n1.view(np.uint32) != gn_e[lo:hi].view(np.uint32)))
        print(f"candidate {b}: {d1} log E and {d2} nu gradients differ", flush=True)
        assert d1 == 0 and d2 == 0


def test_deterministic_gradients_repeat_bitwise():
    """Two taped runs and backwards from the same input, with a return map
    in the scene: the parameter gradients agree bit for bit."""
    sc = pair_scene(8_000)
    outs = []
    for _ in range(2):
        ctx = B.init_from_scene(sc, sort_every=6, deterministic=True)
        p = B.Particles.from_scene(sc)
        tape = torch.empty(B.mpm_tape_size(ctx, 12, 4) // 4 + 64, dtype=torch.float32, device="cuda")
        B.mpm_step_n(ctx, p, 12, tape=tape, checkpoint_every=4)
        gl, gn = torch.empty(sc.n, device="cuda"), torch.empty(sc.n, device="cuda")
        B.mpm_backward(ctx, p, tape, 12, g_x=torch.ones_like(p.x), g_log_E=gl, g_nu=gn)
        torch.cuda.synchronize()
        outs.append([gl.cpu().numpy().view(np.uint32), gn.cpu().numpy().view(np.uint32)])
    for k, (a, b) in enumerate(zip(outs[0], outs[1])):
        assert int(np.count_nonzero(a != b)) == 0, f"gradient {k} differs"
