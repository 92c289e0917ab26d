"""Pins of the oracle's candidate generation (Sec. 4.1: candidates uniform in
the box of each instance's hull, kept by the ray-cast occupancy of the hull
above 0.6), against facts that do not come from the oracle itself:
SciPy's Qhull (half-space equations, bounds, volume) and Delaunay point
location, meshes whose inside is known by construction (a hollow box, boxes
with faces removed, whose vote counts follow by hand), and rays that run
exactly through shared edges and vertices of meshes with dyadic
coordinates (a double or missed count there changes the parity)."""
import math

import numpy as np
import pytest

from oracle import mpm_oracle as O
from paper_2602_01723_amd import scenes


def votes(points, mesh):
    v, t = mesh
    return O.ipf_ray_votes(np.asarray(points, np.float32), np.asarray(v, np.float32)[np.asarray(t)])


def test_convex_hull_occupancy_matches_qhull_half_spaces_and_delaunay():
    from scipy.spatial import ConvexHull, Delaunay
    rng = np.random.default_rng(0)
    pts, tris, _ = scenes.ellipsoid_hull(rng, 400)
    hull = ConvexHull(pts.astype(np.float64))
    lo, hi = O.ipf_box(pts[np.unique(tris)])
    q = O.ipf_points(rng.uniform(0, 1, (3000, 3)), lo, hi)
    s = (q.astype(np.float64) @ hull.equations[:, :3].T + hull.equations[:, 3]).max(axis=1)
    inside, outside = s < -1e-6, s > 1e-6
    assert inside.sum() > 500 and outside.sum() > 500
    vt = votes(q, (pts, tris))
    assert np.all(vt[inside] == 6) and np.all(vt[outside] == 0)
    located = Delaunay(pts.astype(np.float64)).find_simplex(q.astype(np.float64)) >= 0
    assert np.array_equal(located[inside | outside], (vt == 6)[inside | outside])


def test_hollow_box_keeps_the_shell_and_rejects_the_cavity():
    """Outer box [0.2, 0.8]^3 with a closed inner box [0.4, 0.6]^3 (a
    non-convex solid: the cavity is outside).  Every ray from a cavity point
    crosses the inner box once and the outer box once."""
    mesh = scenes.merge_meshes(scenes.box_mesh(0.2, 0.8), scenes.box_mesh(0.4, 0.6))
    rng = np.random.default_rng(1)
    q = rng.uniform(0.1, 0.9, (8000, 3)).astype(np.float32)
    in_outer = np.all((q > 0.2 + 1e-6) & (q < 0.8 - 1e-6), axis=1)
    in_inner = np.all((q > 0.4 + 1e-6) & (q < 0.6 - 1e-6), axis=1)
    outside_outer = np.any((q < 0.2 - 1e-6) | (q > 0.8 + 1e-6), axis=1)
    outside_inner = np.any((q < 0.4 - 1e-6) | (q > 0.6 + 1e-6), axis=1)
    vt = votes(q, mesh)
    shell = in_outer & outside_inner
    assert shell.sum() > 1000 and in_inner.sum() > 100
    assert np.all(vt[shell] == 6)
    assert np.all(vt[in_inner] == 0)
    assert np.all(vt[outside_outer] == 0)


@pytest.mark.parametrize("drop,expected", [((), 6), (("+z",), 5), (("+z", "-z"), 4), (("+x", "+y", "+z"), 3),
                                           (("-x", "+x", "-y", "+y", "-z", "+z"), 0)])
def test_open_boxes_vote_by_their_remaining_faces(drop, expected):
    """A point inside a box whose faces in `drop` are removed: the ray toward
    a removed face crosses nothing, every other ray crosses one face."""
    mesh = scenes.box_mesh(0.3, 0.7, drop=drop)
    rng = np.random.default_rng(2)
    q = rng.uniform(0.31, 0.69, (500, 3)).astype(np.float32)
    assert np.all(votes(q, mesh) == expected)


def test_threshold_keeps_four_of_six_rays_and_more():
    """occ > 0.6 keeps 4, 5 and 6 votes and drops 3; a lower threshold
    (0.49) keeps 3 as well."""
    meshes = [scenes.box_mesh(0.3, 0.7, drop=d) for d in ((), ("+z",), ("+z", "-z"), ("+x", "+y", "+z"))]
    v, t = zip(*meshes)
    vo = np.concatenate([[0], np.cumsum([len(a) for a in v])])
    to = np.concatenate([[0], np.cumsum([len(a) for a in t])])
    # uniforms inside the central part of the box (B_k = [0.3, 0.7]^3)
    rng = np.random.default_rng(3)
    u = rng.uniform(0.05, 0.95, (4 * 100, 3))
    ro = np.arange(0, 401, 100)
    pts, idx, offs, vt = O.ipf_candidates(np.concatenate(v), vo, np.concatenate(t), to, u, ro)
    assert list(np.diff(offs)) == [100, 100, 100, 0]
    assert np.array_equal(idx, np.arange(300))
    assert np.array_equal(np.bincount(vt, minlength=7)[3:], [100, 100, 100, 100])  # 3, 4, 5, 6 votes
    _, _, offs2, _ = O.ipf_candidates(np.concatenate(v), vo, np.concatenate(t), to, u, ro, threshold=0.49)
    assert list(np.diff(offs2)) == [100, 100, 100, 100]


def test_rays_through_shared_edges_and_vertices_cross_once():
    """Dyadic meshes and query points, so the edge functions are exact and
    hit zero where a ray runs through an edge or a vertex.

    Box [0.25, 0.75]^3: each face is split along the diagonal from its lowest
    corner, so a point inside with y == z sends its x rays through the
    diagonals of both x faces (likewise z == x for y rays, x == y for z
    rays); the centre does all three.  Outside points whose x ray grazes the
    box along an edge or a face must count an even number of crossings.
    Octahedron around (0.5, 0.5, 0.5) with radius 0.25: points on the
    coordinate axes through the centre send rays through the vertices where
    four triangles meet and along projected edges."""
    box = scenes.box_mesh(0.25, 0.75)
    inside = np.array([[0.5, 0.5, 0.5], [0.3125, 0.5, 0.5], [0.625, 0.375, 0.375], [0.5, 0.625, 0.5],
                       [0.375, 0.4375, 0.375], [0.4375, 0.4375, 0.6875]], np.float32)
    assert np.all(votes(inside, box) == 6)
    outside = np.array([[0.125, 0.25, 0.25], [0.125, 0.75, 0.75], [0.125, 0.25, 0.5], [0.125, 0.75, 0.5],
                        [0.875, 0.5, 0.25], [0.5, 0.875, 0.75], [0.5, 0.125, 0.25]], np.float32)
    assert np.all(votes(outside, box) == 0)
    octa = scenes.octahedron_mesh((0.5, 0.5, 0.5), 0.25)
    on_axes = np.array([[0.375, 0.5, 0.5], [0.5, 0.625, 0.5], [0.5, 0.5, 0.3125], [0.5, 0.5, 0.5],
                        [0.5625, 0.5, 0.5]], np.float32)
    assert np.all(votes(on_axes, octa) == 6)
    beyond = np.array([[0.125, 0.5, 0.5], [0.5, 0.875, 0.5], [0.5, 0.5, 0.0625]], np.float32)
    assert np.all(votes(beyond, octa) == 0)


def test_votes_do_not_depend_on_triangle_orientation_or_order():
    rng = np.random.default_rng(4)
    pts, tris, _ = scenes.ellipsoid_hull(rng, 300)
    q = O.ipf_points(rng.uniform(0, 1, (1500, 3)), *O.ipf_box(pts))
    ref = votes(q, (pts, tris))
    t2 = tris.copy()
    flip = rng.uniform(size=len(t2)) < 0.5
    t2[flip] = t2[flip][:, ::-1]
    t2 = t2[rng.permutation(len(t2))]
    assert np.array_equal(votes(q, (pts, t2)), ref)


def test_box_comes_from_the_hull_and_points_span_it():
    from scipy.spatial import ConvexHull
    rng = np.random.default_rng(5)
    pts, tris, _ = scenes.ellipsoid_hull(rng, 500)
    hull = ConvexHull(pts.astype(np.float64))
    lo, hi = O.ipf_box(pts[np.unique(tris)])
    assert np.array_equal(lo.astype(np.float64), hull.min_bound)
    assert np.array_equal(hi.astype(np.float64), hull.max_bound)
    corners = O.ipf_points(np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.0, 1.0, 0.0]]), lo, hi)
    assert np.array_equal(corners[0], lo) and np.array_equal(corners[1], hi)
    assert np.array_equal(corners[2], [lo[0], hi[1], lo[2]])
    q = O.ipf_points(rng.uniform(0, 1, (20000, 3)), lo, hi)
    assert np.all((q >= lo) & (q <= hi))
    # uniform in the box: per-axis mean at the centre within 5 standard errors
    se = (hi - lo) / math.sqrt(12 * len(q))
    assert np.all(np.abs(q.mean(0) - 0.5 * (lo + hi)) < 5 * se)


def test_kept_fraction_estimates_the_hull_volume():
    """For the convex hull the kept fraction of uniform box candidates is a
    binomial estimate of vol(hull) / vol(box) (Qhull's volume)."""
    d = scenes.ipf_inputs(seed=6, n_shell=(600, 900), raw_per_point=6.0)
    pts, idx, offs, _ = O.ipf_candidates(d["hull_vertices"], d["hull_vertex_offsets"], d["hull_triangles"],
                                         d["hull_triangle_offsets"], d["u"], d["raw_offsets"])
    for k in range(2):
        v0, v1 = d["hull_vertex_offsets"][k:k + 2]
        lo, hi = O.ipf_box(d["hull_vertices"][v0:v1])
        p = d["hull_volume"][k] / float(np.prod(hi.astype(np.float64) - lo))
        n = int(d["raw_offsets"][k + 1] - d["raw_offsets"][k])
        kept = int(offs[k + 1] - offs[k])
        assert abs(kept / n - p) < 5 * math.sqrt(p * (1 - p) / n)


def test_candidates_bookkeeping_and_degenerate_instances():
    """Offsets are prefix sums of per-instance kept counts, indices ascend
    and point into their own instance, an instance without triangles or
    without raw candidates keeps nothing, and bad inputs raise."""
    box = scenes.box_mesh(0.3, 0.7)
    v = np.concatenate([box[0], box[0], box[0]])
    t = np.concatenate([box[1], np.zeros((0, 3), np.int32), box[1]])
    vo, to = [0, 8, 16, 24], [0, 12, 12, 24]
    rng = np.random.default_rng(7)
    ro = [0, 50, 80, 80]
    u = rng.uniform(0, 1, (80, 3))
    pts, idx, offs, vt = O.ipf_candidates(v, vo, t, to, u, ro)
    assert list(offs) == [0, 50, 50, 50]
    assert np.array_equal(idx, np.arange(50)) and np.all(vt[50:] == 0)
    assert pts.dtype == np.float32 and pts.shape == (50, 3)
    with pytest.raises(ValueError):
        O.ipf_candidates(v, vo, np.where(t == 7, 8, t), to, u, ro)
    with pytest.raises(ValueError):
        O.ipf_candidates(v + 0.5, vo, t, to, u, ro)
    with pytest.raises(ValueError):
        O.ipf_candidates(v, vo, t, to, u * 1.5, ro)


def _cycle(points, shift):
    """Cyclic relabelling of the axes: new axis a takes old axis (a - shift) mod 3."""
    return np.roll(np.asarray(points, np.float32), shift, axis=-1)


@pytest.mark.parametrize("shift", [0, 1, 2])
def test_perturbation_convention_on_an_open_triangle(shift):
    """The zero of an edge function is resolved by moving q by (e, e^2) in
    the two axes that follow the ray's axis cyclically.  A triangle below
    the diagonal of its plane (b > c) claims a query on the diagonal, the
    triangle above it does not, and the closed square of both claims it
    once.  The other order of the two axes would flip the first two."""
    below = (np.array([[0.25, 0.25, 0.5], [0.75, 0.75, 0.5], [0.75, 0.25, 0.5]], np.float32), [[0, 1, 2]])
    above = (np.array([[0.25, 0.25, 0.5], [0.25, 0.75, 0.5], [0.75, 0.75, 0.5]], np.float32), [[0, 1, 2]])
    q = np.array([[0.5, 0.5, 0.25], [0.5, 0.5, 0.75]], np.float32)  # rays along the third axis cross z = 0.5
    cyc = lambda m: (_cycle(m[0], shift), m[1])
    assert list(votes(_cycle(q, shift), cyc(below))) == [1, 1]
    assert list(votes(_cycle(q, shift), cyc(above))) == [0, 0]
    assert list(votes(_cycle(q, shift), cyc(scenes.merge_meshes(below, above)))) == [1, 1]


def test_points_on_the_surface():
    """A point on a face: the crossing at t = 0 counts for both rays of the
    face's axis, and the (e, e^2) move decides the other four rays.  On the
    -x face of [0.25, 0.75]^3: + ray 2 crossings, - ray 1, y and z rays 1
    each (moved inside) -> 5 votes, kept.  On the +x face: + ray 1,
    - ray 2, y and z rays moved outside -> 1 vote."""
    box = scenes.box_mesh(0.25, 0.75)
    q = np.array([[0.25, 0.5, 0.375], [0.75, 0.5, 0.375]], np.float32)
    assert list(votes(q, box)) == [5, 1]


def test_threshold_is_strict():
    """occ > threshold: at 0.5 three votes of six are not enough."""
    v, t = scenes.box_mesh(0.3, 0.7, drop=("+x", "+y", "+z"))
    rng = np.random.default_rng(8)
    u = rng.uniform(0.05, 0.95, (100, 3))
    _, _, offs, vt = O.ipf_candidates(v, [0, 8], t, [0, len(t)], u, [0, 100], threshold=0.5)
    assert np.all(vt == 3) and list(offs) == [0, 0]


def test_box_ignores_vertices_no_triangle_uses():
    """B_k is the box of the hull H_k: a vertex that no triangle uses (a point
    inside the hull, or a stray one) does not widen it."""
    v, t = scenes.box_mesh(0.3, 0.7)
    v2 = np.concatenate([v, [[0.05, 0.95, 0.5]]]).astype(np.float32)
    u = np.random.default_rng(9).uniform(0, 1, (200, 3))
    a = O.ipf_candidates(v, [0, 8], t, [0, 12], u, [0, 200])
    b = O.ipf_candidates(v2, [0, 9], t, [0, 12], u, [0, 200])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and len(a[1]) == 200
