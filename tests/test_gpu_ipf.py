"""Candidate generation of the interior fill (Sec. 4.1) through the C ABI
against the oracle: candidates uniform in the box of each instance's hull,
kept where the six-ray parity occupancy of the hull mesh exceeds 0.6.

Kept/dropped is integer work decided by float64 arithmetic that both sides
evaluate in the same order without contraction, so the bar is bit-exact:
the kept raw indices, the offsets and every coordinate.  At the full size
(four instances of 37,500 hull points, 600,000 raw candidates) the oracle
decides a sample of raw candidates one by one and the kept fraction is
checked against each hull's volume."""
import math

import numpy as np
import pytest
import torch

from oracle import mpm_oracle as O
from paper_2602_01723_amd import binding as B
from paper_2602_01723_amd import scenes

pytestmark = pytest.mark.gpu


def dev_planes(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype).reshape(-1, 3).T)).cuda()


def run_gpu(d, threshold=0.6):
    print(f"ipf: K={len(d['raw_offsets']) - 1} V={int(d['hull_vertex_offsets'][-1])} "
          f"T={int(d['hull_triangle_offsets'][-1])} R={int(d['raw_offsets'][-1])}", flush=True)
    cand, offs, src = B.mpm_ipf_candidates(dev_planes(d["hull_vertices"], np.float32),
                                           d["hull_vertex_offsets"], dev_planes(d["hull_triangles"], np.int32),
                                           d["hull_triangle_offsets"], dev_planes(d["u"], np.float64),
                                           d["raw_offsets"], threshold, want_source=True)
    torch.cuda.synchronize()
    return cand.cpu().numpy().T.copy(), np.array(offs, np.int64), src.cpu().numpy()


def run_oracle(d, threshold=0.6):
    return O.ipf_candidates(d["hull_vertices"], d["hull_vertex_offsets"], d["hull_triangles"],
                            d["hull_triangle_offsets"], d["u"], d["raw_offsets"], threshold)


def grid_uniforms(n):
    """Uniforms on the grid {0, 1/n, ..., 1}^3: with a dyadic box they put
    candidates exactly on projected edges and vertices of dyadic meshes."""
    g = np.arange(n + 1) / n
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)


def mixed_inputs(seed=8):
    """Ellipsoid hulls, then a hollow box, two open boxes (one with an extra
    vertex that no triangle uses, which must not widen its box), an
    octahedron and an instance without triangles; the box and octahedron
    instances take grid uniforms (ties), the rest random ones."""
    hollow = scenes.merge_meshes(scenes.box_mesh(0.25, 0.75), scenes.box_mesh(0.375, 0.625))
    open_z = scenes.box_mesh(0.25, 0.75, drop=("+z",))
    open_z = (np.concatenate([open_z[0], [[0.05, 0.9, 0.5]]]).astype(np.float32), open_z[1])
    meshes = [hollow, open_z, scenes.box_mesh(0.25, 0.75, drop=("+x", "+y", "+z")),
              scenes.octahedron_mesh((0.5, 0.5, 0.5), 0.25),
              (np.array([[0.5, 0.5, 0.5]], np.float32), np.zeros((0, 3), np.int32))]
    d = scenes.ipf_inputs(seed=seed, n_shell=(600, 1000, 400), raw_per_point=4.0, meshes=meshes, raw_per_mesh=729)
    # grid uniforms for the four dyadic meshes (their raw slots hold 729 = 9^3 each)
    ro = d["raw_offsets"]
    for k in range(3, 7):
        d["u"][ro[k]:ro[k + 1]] = grid_uniforms(8)
    return d


def assert_bit_exact(got, ref):
    cand, offs, src = got
    rp, ridx, roffs, _ = ref
    assert np.array_equal(offs, roffs), (offs, roffs)
    assert np.array_equal(src, ridx)
    assert cand.shape == rp.shape and np.array_equal(cand.view(np.uint32), rp.view(np.uint32))


def test_candidates_bit_exact_against_the_oracle():
    d = mixed_inputs()
    ref = run_oracle(d)
    got = run_gpu(d)
    assert_bit_exact(got, ref)
    counts = np.diff(ref[2])
    assert np.all(counts[[0, 1, 2, 3, 4, 6]] > 0)
    assert counts[7] == 0  # the instance without triangles keeps nothing
    # the open box without three faces votes 3 of 6 inside: only surface points can be kept
    assert counts[5] < 729 // 4
    # twice: the same result (the binning order does not matter)
    assert_bit_exact(run_gpu(d), ref)


@pytest.mark.parametrize("threshold", [0.0, 0.49, 0.5, 0.99])
def test_thresholds_bit_exact(threshold):
    d = mixed_inputs(seed=9)
    assert_bit_exact(run_gpu(d, threshold), run_oracle(d, threshold))


def test_grids_with_many_references_per_triangle():
    """Long thin triangles (a box cut into slivers) span many cells of the
    triangle grid: the side of a grid is halved until its references fit,
    which must leave the result unchanged."""
    n = 400  # slivers: the -x face as a fan of 2n triangles from one corner
    v, t = scenes.box_mesh(0.2, 0.8)
    edge = np.stack([np.full(n + 1, 0.2), np.linspace(0.2, 0.8, n + 1), np.full(n + 1, 0.8)], -1)
    edge2 = np.stack([np.full(n + 1, 0.2), np.full(n + 1, 0.8), np.linspace(0.8, 0.2, n + 1)], -1)
    fan = np.concatenate([[[0.2, 0.2, 0.2]], edge, edge2[1:]]).astype(np.float32)
    # -x face: corner (0.2, 0.2, 0.2), then (y, 0.8) for y up, then (0.8, z) for z down
    ft = np.array([[0, i, i + 1] for i in range(1, 2 * n + 1)], np.int32)
    mesh = scenes.merge_meshes((v, t[2:]), (fan, ft))  # t[2:]: every face but -x
    d = scenes.ipf_inputs(seed=11, n_shell=(), meshes=[mesh], raw_per_mesh=5000)
    ref = run_oracle(d)
    assert np.diff(ref[2])[0] > 3000
    assert_bit_exact(run_gpu(d), ref)


def test_ipf_then_mcis_matches_the_oracle():
    """The kept candidates feed the MCIS selection unchanged (layout and
    offsets): GPU candidates -> GPU selection against oracle candidates ->
    oracle selection, with the same selection uniforms."""
    d = scenes.ipf_inputs(seed=12, n_shell=(800, 1200), raw_per_point=4.0)
    ref = run_oracle(d)
    cand, offs, src = run_gpu(d)
    assert_bit_exact((cand, offs, src), ref)
    M = int(offs[-1])
    rng = np.random.default_rng(13)
    u_sel = 1.0 - rng.uniform(0.0, 1.0, M)
    n_sel = (np.diff(offs) // 2).astype(np.int64)
    surf = dev_planes(d["surface"], np.float32)
    idx, dist = B.mpm_mcis_select(surf, d["surface_offsets"], dev_planes(cand, np.float32), offs,
                                  torch.as_tensor(u_sel).cuda(), n_sel, want_distance=True)
    torch.cuda.synchronize()
    got = idx.cpu().numpy()
    sel, rd = O.mcis(ref[0], ref[2], d["surface"], d["surface_offsets"], u_sel, n_sel)
    ref_sel = sel.numpy()
    assert len(got) == len(ref_sel) == int(n_sel.sum())
    diff = set(got.tolist()) ^ set(ref_sel.tolist())
    if diff:  # only near-ties of keys may differ (exp and log may differ in the last bit)
        rd = rd.numpy()
        w = np.maximum(np.exp(-rd ** 2 / (2 * 0.02 ** 2)), 1e-6)
        keys = np.log(u_sel) / w
        for j in diff:
            k = int(np.searchsorted(offs, j, side="right") - 1)
            kk = np.sort(keys[offs[k]:offs[k + 1]])[::-1]
            T = kk[int(n_sel[k]) - 1]
            assert abs(keys[j] - T) <= 1e-12 * abs(T), (j, keys[j], T)


def test_full_size_sampled_against_the_oracle():
    """Four instances of 37,500 hull points (the shell half of the
    300,000-particle Gaussian-cloud scene), four raw candidates per point:
    the oracle decides 150 sampled raw candidates per instance one by one,
    and each instance's kept fraction estimates its hull's volume share of
    the box."""
    d = scenes.ipf_inputs(seed=14, n_shell=(37_500,) * 4, raw_per_point=4.0, r_range=(0.05, 0.195))
    cand, offs, src = run_gpu(d)
    ro = d["raw_offsets"]
    kept = np.zeros(int(ro[-1]), bool)
    kept[src] = True
    assert np.all(np.diff(src) > 0)
    rng = np.random.default_rng(15)
    for k in range(4):
        r0, r1 = int(ro[k]), int(ro[k + 1])
        v0, v1 = d["hull_vertex_offsets"][k:k + 2]
        t0, t1 = d["hull_triangle_offsets"][k:k + 2]
        lo, hi = O.ipf_box(d["hull_vertices"][v0:v1])
        pick = np.sort(rng.choice(np.arange(r0, r1), 150, replace=False))
        q = O.ipf_points(d["u"][pick], lo, hi)
        tri = d["hull_vertices"][v0:v1][d["hull_triangles"][t0:t1]]
        want = O.ipf_ray_votes(q, tri) / 6.0 > 0.6
        assert np.array_equal(kept[pick], want), k
        # coordinates of the sampled kept ones
        pos = np.searchsorted(src, pick[want])
        assert np.array_equal(cand[pos].view(np.uint32), q[want].view(np.uint32))
        # kept fraction vs vol(hull) / vol(box), 5 binomial standard errors
        p = d["hull_volume"][k] / float(np.prod(hi.astype(np.float64) - lo))
        n = r1 - r0
        frac = (offs[k + 1] - offs[k]) / n
        assert abs(frac - p) < 5 * math.sqrt(p * (1 - p) / n), (k, frac, p)


def test_invalid_inputs_are_rejected():
    d = mixed_inputs(seed=16)
    bad = dict(d)
    bad["hull_triangles"] = d["hull_triangles"].copy()
    bad["hull_triangles"][5, 1] = 10_000  # outside its instance
    with pytest.raises(B.MPMError, match="invalid"):
        run_gpu(bad)
    bad = dict(d)
    bad["hull_vertices"] = d["hull_vertices"].copy()
    bad["hull_vertices"][3, 2] = 1.5
    with pytest.raises(B.MPMError, match="invalid"):
        run_gpu(bad)
    bad = dict(d)
    bad["u"] = d["u"].copy()
    bad["u"][17, 0] = -0.25
    with pytest.raises(B.MPMError, match="invalid"):
        run_gpu(bad)
    with pytest.raises(B.MPMError, match="invalid"):
        run_gpu(d, threshold=1.5)
    # after the errors the library still works
    assert_bit_exact(run_gpu(d), run_oracle(d))


def test_no_raw_candidates_or_no_triangles():
    box = scenes.box_mesh(0.25, 0.75)
    d = scenes.ipf_inputs(seed=17, n_shell=(), meshes=[box, box], raw_per_mesh=0)
    cand, offs, src = run_gpu(d)
    assert list(offs) == [0, 0, 0] and cand.shape == (0, 3)
    d = scenes.ipf_inputs(seed=17, n_shell=(), meshes=[(box[0], np.zeros((0, 3), np.int32))], raw_per_mesh=100)
    cand, offs, src = run_gpu(d)
    assert list(offs) == [0, 0]


def test_many_small_instances_bit_exact():
    """300 instances of 40 hull points each (grids of a few cells, waves
    spanning instances in the box reduction and the binning)."""
    d = scenes.ipf_inputs(seed=18, n_shell=(40,) * 300, raw_per_point=5.0, r_range=(0.01, 0.04))
    ref = run_oracle(d)
    assert np.all(np.diff(ref[2]) > 0)
    assert_bit_exact(run_gpu(d), ref)
