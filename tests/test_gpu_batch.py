"""Batched candidates: one hipGraph of forward + loss + adjoint for all
candidates vs per-candidate eager solves; graph replays vs eager; autotuner."""
import numpy as np
import pytest
import torch

from oracle import mpm_oracle as O
from paper_2602_01723_amd import batch as BT
from paper_2602_01723_amd import binding as B
from paper_2602_01723_amd import scenes
from tests.parity import compare_substep, rel_err

pytestmark = pytest.mark.gpu


def small_batch():
    # dt 2e-4: the bodies land after about 10 substeps and deform for the rest
    return scenes.make_scene("candidate_batch", n_batch=6, n_min=1500, n_max=6000, grid_res=32, n_substeps=60,
                             dt=2e-4)


def test_batched_graph_matches_eager_and_plain():
    sc = small_batch()
    steps, K = 60, 15
    tl = BT.per_particle(sc.extras["target_log_E"], sc.batch_offsets)
    tn = BT.per_particle(sc.extras["target_nu"], sc.batch_offsets)
    xt = BT.target_positions(sc, steps, tl, tn)
    ev = BT.Evaluation(sc, steps, K, xt)
    ev.run_eager()
    torch.cuda.synchronize()
    gl_e, gn_e = ev.gradients()
    loss_e = ev.losses()
    assert np.all(loss_e > 0) and np.all(np.isfinite(gl_e))
    ev.capture()
    for rep in range(3):  # replays with eager work and synchronisation in between
        ev.run_graph()
        torch.cuda.synchronize()
        gl, gn = ev.gradients()
        print("replay", rep, rel_err(gl, gl_e, 0.0), rel_err(gn, gn_e, 0.0), flush=True)
        assert rel_err(gl, gl_e, 0.0) < 1e-3 and rel_err(gn, gn_e, 0.0) < 1e-3
        assert np.allclose(ev.losses(), loss_e, rtol=1e-4)
        _ = torch.ones(1000, device="cuda").sum().item()
    plain = BT.plain_evaluations(sc, steps, K, xt)
    for b, pe in enumerate(plain):
        pe.run_eager()
        torch.cuda.synchronize()
        lo, hi = sc.batch_offsets[b], sc.batch_offsets[b + 1]
        g1, n1 = pe.gradients()
        print("candidate", b, g1.sum(), gl_e[lo:hi].sum(), flush=True)
        assert rel_err(g1, gl_e[lo:hi], 0.0) < 1e-3
        assert rel_err(n1, gn_e[lo:hi], 0.0) < 1e-3
        assert abs(pe.losses()[0] - loss_e[b]) <= 1e-4 * loss_e[b]


def test_autotune_keeps_caller_state_and_parity():
    sc = scenes.make_scene("gaussian_cloud", n_total=20_000)
    ctx = B.init_from_scene(sc)
    p = B.Particles.from_scene(sc)
    before = p.state_numpy()
    best = B.mpm_autotune(ctx, p, trial_steps=4)
    torch.cuda.synchronize()
    after = p.state_numpy()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    assert best["chunk"] in (256, 512, 768, 1024, 1536, 2048) and best["workgroups"] > 0
    assert best["sort_every"] in (2, 4, 8)  # candidates below 2 x trial_steps, or the default 8 kept
    assert best["ms_per_substep"] > 0
    assert B.mpm_get_tuning(ctx)["chunk"] == best["chunk"]
    state0 = p.state_numpy()
    B.mpm_substep(ctx, p)
    torch.cuda.synchronize()
    m, mv, v = (t.cpu().numpy() for t in B.grid_state(ctx))
    errs, _ = compare_substep(state0, p.state_numpy(), (m, mv, v), O.Params.from_scene(sc), sc.mass)
    assert max(errs[k] for k in ("x", "v", "C", "F", "m", "mv", "grid_v")) < 1e-5, errs
