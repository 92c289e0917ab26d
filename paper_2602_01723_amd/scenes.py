"""Seeded synthetic particle scenes for the MLS-MPM substep.

This module only *builds inputs*: positions, velocities, initial affine and
deformation state, per-particle mass / volume / material parameters.  It holds
none of the simulation arithmetic, and both the HIP path and the FP64 oracle
consume what it returns.  It imports nothing but NumPy (and SciPy's KD-tree
when present).

The scenes stand in for the paper's 3DGS scenes (not available here): every
object is normalised into the unit cube (App. C, setup details), Gaussian
centres are placed on ellipsoid shells and the interior is filled by the
instance-aware Monte Carlo importance sampling of Sec. 4.1 (MCIS steps 1-5:
nearest-surface distance, Gaussian importance weight with sigma = 0.02 and
floor 1e-6, normalisation, sampling of n_k points, union with the shell set),
with the analytic ellipsoid inside test replacing the convex hull and
ray-cast occupancy field.

Array conventions (all NumPy, particle-major):
  x, v        float32 [N, 3]
  C, F        float32 [N, 3, 3]   (row-major 3x3)
  mass, vol0  float32 [N]
  log_E, nu   float32 [N]
  mat_id      int32   [N]         index into ``materials``
  inst_id     int32   [N]         instance label (label memory of Sec. 4.1)
  is_shell    bool    [N]         True for Gaussian centres (shell points)
  cov0        float32 [N, 6]      rest covariance (xx, xy, xz, yy, yz, zz)
  batch_offsets int64 [B + 1]     particles of scene b are [off[b], off[b+1])
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

# Material codes shared with include/fastmpm.h (MPM_ELASTIC_*, MPM_PLASTIC_*).
ELASTIC_FCR = 0
ELASTIC_HENCKY = 1
ELASTIC_NEO_HOOKEAN = 2
ELASTIC_STVK = 3
ELASTIC_FLUID = 4
ELASTIC_VOLUME = 5
PLASTIC_NONE = 0
PLASTIC_VON_MISES = 1
PLASTIC_DRUCKER_PRAGER = 2
PLASTIC_FLUID = 3
PLASTIC_SIGMA = 4

RHO = 1000.0
GRAVITY = (0.0, -9.8, 0.0)
BOUND = 3


@dataclass
class Scene:
    name: str
    grid_res: int
    dt: float
    n_substeps: int
    materials: List[Dict]
    x: np.ndarray
    v: np.ndarray
    C: np.ndarray
    F: np.ndarray
    mass: np.ndarray
    vol0: np.ndarray
    log_E: np.ndarray
    nu: np.ndarray
    mat_id: np.ndarray
    inst_id: np.ndarray
    is_shell: np.ndarray
    cov0: np.ndarray
    batch_offsets: np.ndarray
    gravity: tuple = GRAVITY
    bound: int = BOUND
    checkpoint_every: int = 0
    extras: Dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_batch(self) -> int:
        return int(self.batch_offsets.shape[0] - 1)

    def copy(self) -> "Scene":
        out = Scene(**{k: (v.copy() if isinstance(v, np.ndarray) else v)
                       for k, v in self.__dict__.items() if k != "extras"})
        out.extras = dict(self.extras)
        return out

    def subset(self, b: int) -> "Scene":
        """Scene b of a batched scene as a one-scene Scene (same grid, dt)."""
        lo, hi = int(self.batch_offsets[b]), int(self.batch_offsets[b + 1])
        kw = {}
        for k, v in self.__dict__.items():
            if isinstance(v, np.ndarray) and v.ndim >= 1 and v.shape[0] == self.n and k != "batch_offsets":
                kw[k] = v[lo:hi].copy()
            elif k == "batch_offsets":
                kw[k] = np.array([0, hi - lo], dtype=np.int64)
            elif k == "extras":
                continue
            else:
                kw[k] = v
        s = Scene(**kw)
        s.name = f"{self.name}[{b}]"
        return s


def _material(elastic, plastic=PLASTIC_NONE, yield_stress=0.0, friction_deg=0.0):
    return dict(elastic=int(elastic), plastic=int(plastic),
                yield_stress=float(yield_stress), friction_deg=float(friction_deg))


def haar_rotation(rng) -> np.ndarray:
    """Uniformly random rotation: QR of a Gaussian matrix with the sign fix."""
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _nearest_distance(queries: np.ndarray, points: np.ndarray, cutoff=np.inf) -> np.ndarray:
    """Distance to the nearest point; beyond ``cutoff`` the result is inf."""
    try:
        from scipy.spatial import cKDTree
        # sliding-midpoint tree: much faster than median splits on surface points
        tree = cKDTree(points, balanced_tree=False, compact_nodes=False)
        d, _ = tree.query(queries, k=1, distance_upper_bound=cutoff, workers=-1)
        return d
    except ImportError:  # pragma: no cover - brute force, chunked
        out = np.empty(len(queries))
        for s in range(0, len(queries), 4096):
            q = queries[s:s + 4096]
            d2 = ((q[:, None, :] - points[None, :, :]) ** 2).sum(-1)
            out[s:s + 4096] = np.sqrt(d2.min(1))
        out[out > cutoff] = np.inf
        return out


def ellipsoid_instance(rng, centre, axes, rot, n_shell, n_interior, sigma=0.02, eps=1e-6):
    """Shell points plus an MCIS interior fill of one ellipsoid (Sec. 4.1).

    Returns (points [n_shell + n_interior, 3] float64, is_shell bool array).
    """
    centre = np.asarray(centre, np.float64)
    axes = np.asarray(axes, np.float64)
    u = rng.standard_normal((n_shell, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    shell = centre + (u * axes) @ rot.T
    if n_interior == 0:
        return shell, np.ones(n_shell, bool)
    # candidate points, uniform in the instance AABB (M >> n)
    half = np.sqrt(((rot * axes[None, :]) ** 2).sum(1))
    pts = []
    need = n_interior
    m = 8 * n_interior
    while need > 0:
        q = centre + rng.uniform(-1.0, 1.0, (m, 3)) * half
        loc = (q - centre) @ rot / axes  # ellipsoid frame, unit sphere
        r = np.sqrt((loc ** 2).sum(1))
        keep = r < 1.0
        pts.append((q[keep], r[keep]))
        need -= int(keep.sum())
    cand = np.concatenate([c for c, _ in pts])
    rad = np.concatenate([r for _, r in pts])
    # MCIS 1-3: nearest-surface distance -> Gaussian weight -> probabilities.
    # Beyond `cutoff` the Gaussian weight is below eps and the floor applies;
    # a point at normalised radius r is at least (1 - r) * min(axes) from the
    # surface (and so from every shell point), so only the rest is queried.
    cutoff = sigma * math.sqrt(-2.0 * math.log(eps)) * 1.01
    d = np.full(len(cand), np.inf)
    near = (1.0 - rad) * axes.min() <= cutoff
    d[near] = _nearest_distance(cand[near], shell, cutoff)
    w = np.maximum(np.exp(-d * d / (2.0 * sigma * sigma)), eps)
    p = w / w.sum()
    # MCIS 4: draw n_k points by p, without replacement (duplicates add
    # nothing to MPM), with the exponential-key method of Efraimidis and
    # Spirakis (2006): the n_k largest log(u)/p_j.
    keys = np.log(rng.uniform(0.0, 1.0, len(cand))) / p
    pick = np.argpartition(-keys, n_interior - 1)[:n_interior]
    interior = cand[pick]
    pts = np.concatenate([shell, interior])
    is_shell = np.zeros(len(pts), bool)
    is_shell[:n_shell] = True
    return pts, is_shell


def _rest_cov(rng, n, dx):
    s = rng.uniform(0.2, 1.0, (n, 3)) * (0.5 * dx)
    out = np.empty((n, 6), np.float32)
    q = np.stack([haar_rotation(rng) for _ in range(min(n, 64))])
    qi = q[rng.integers(0, len(q), n)]
    cov = np.einsum("nij,nj,nkj->nik", qi, s * s, qi)
    out[:, 0] = cov[:, 0, 0]
    out[:, 1] = cov[:, 0, 1]
    out[:, 2] = cov[:, 0, 2]
    out[:, 3] = cov[:, 1, 1]
    out[:, 4] = cov[:, 1, 2]
    out[:, 5] = cov[:, 2, 2]
    return out


def _finish(name, grid_res, dt, n_substeps, materials, parts, rng, offsets=None, **kw) -> Scene:
    """parts: list of dicts with pts, is_shell, vol, log_E, nu, mat, inst, v0."""
    x = np.concatenate([p["pts"] for p in parts]).astype(np.float32)
    n = len(x)
    v = np.concatenate([np.broadcast_to(np.asarray(p["v0"], np.float64), (len(p["pts"]), 3))
                        for p in parts]).astype(np.float32)
    vol0 = np.concatenate([np.full(len(p["pts"]), p["vol"]) for p in parts]).astype(np.float32)
    mass = (RHO * vol0.astype(np.float64)).astype(np.float32)
    log_E = np.concatenate([np.full(len(p["pts"]), p["log_E"]) for p in parts]).astype(np.float32)
    nu = np.concatenate([np.full(len(p["pts"]), p["nu"]) for p in parts]).astype(np.float32)
    mat_id = np.concatenate([np.full(len(p["pts"]), p["mat"]) for p in parts]).astype(np.int32)
    inst_id = np.concatenate([np.full(len(p["pts"]), p["inst"]) for p in parts]).astype(np.int32)
    is_shell = np.concatenate([p["is_shell"] for p in parts])
    C = np.zeros((n, 3, 3), np.float32)
    F = np.broadcast_to(np.eye(3, dtype=np.float32), (n, 3, 3)).copy()
    cov0 = _rest_cov(rng, n, 1.0 / grid_res)
    if offsets is None:
        offsets = np.array([0, n], np.int64)
    return Scene(name=name, grid_res=grid_res, dt=dt, n_substeps=n_substeps,
                 materials=materials, x=x, v=v, C=C, F=F, mass=mass, vol0=vol0,
                 log_E=log_E, nu=nu, mat_id=mat_id, inst_id=inst_id,
                 is_shell=is_shell, cov0=cov0, batch_offsets=np.asarray(offsets, np.int64), **kw)


def _ellipsoid_volume(axes):
    return 4.0 / 3.0 * math.pi * float(np.prod(axes))


# ----------------------------------------------------------------------------
# Configurations
# ----------------------------------------------------------------------------

def cube_lattice(seed=0, grid_res=32, per_axis=16, side=0.25, centre=(0.5, 0.6, 0.5),
                 E=1e5, nu=0.3, dt=1e-4, n_substeps=100) -> Scene:
    """Plain scene: a jittered lattice filling a cube (spacing side/per_axis,
    jitter uniform in +-0.25 spacing), fixed-corotated elastic."""
    rng = np.random.default_rng(seed)
    h = side / per_axis
    lo = np.asarray(centre) - side / 2
    idx = np.stack(np.meshgrid(*[np.arange(per_axis)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pts = lo + (idx + 0.5) * h + rng.uniform(-0.25, 0.25, idx.shape) * h
    vol = side ** 3 / len(pts)
    parts = [dict(pts=pts, is_shell=np.zeros(len(pts), bool), vol=vol, log_E=math.log(E), nu=nu,
                  mat=0, inst=0, v0=(0.0, 0.0, 0.0))]
    return _finish("cube_lattice", grid_res, dt, n_substeps, [_material(ELASTIC_FCR)], parts, rng)


def cube_uniform(seed=0, n=20480, grid_res=32, side=0.25, centre=(0.5, 0.6, 0.5),
                 E=1e5, nu=0.3, dt=1e-4, n_substeps=100) -> Scene:
    """Plain scene at the stated count: n seeded-uniform points in the cube."""
    rng = np.random.default_rng(seed)
    pts = np.asarray(centre) - side / 2 + rng.uniform(0.0, side, (n, 3))
    parts = [dict(pts=pts, is_shell=np.zeros(n, bool), vol=side ** 3 / n, log_E=math.log(E), nu=nu,
                  mat=0, inst=0, v0=(0.0, 0.0, 0.0))]
    return _finish("cube_uniform", grid_res, dt, n_substeps, [_material(ELASTIC_FCR)], parts, rng)


def gaussian_cloud(seed=1, n_total=300_000, grid_res=64, dt=1e-4, n_substeps=1000) -> Scene:
    """Four ellipsoid instances (half shell, half MCIS interior) in a 2x2
    x-z layout, materials: two fixed-corotated (E log-uniform 1e4..1e6),
    one Hencky + von Mises (yield 1e3), one Hencky + Drucker-Prager (30 deg)."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / grid_res
    mats = [_material(ELASTIC_FCR), _material(ELASTIC_FCR),
            _material(ELASTIC_HENCKY, PLASTIC_VON_MISES, yield_stress=1e3),
            _material(ELASTIC_HENCKY, PLASTIC_DRUCKER_PRAGER, friction_deg=30.0)]
    per = n_total // 4
    sizes = [per] * 3 + [n_total - 3 * per]
    parts = []
    slots = [(0.28, 0.28), (0.72, 0.28), (0.28, 0.72), (0.72, 0.72)]
    for k in range(4):
        axes = rng.uniform(0.05, 0.195, 3)
        rot = haar_rotation(rng)
        yc = 3 * dx + axes.max() + 0.02
        centre = (slots[k][0], yc, slots[k][1])
        ns = sizes[k] // 2
        pts, sh = ellipsoid_instance(rng, centre, axes, rot, ns, sizes[k] - ns)
        E = math.exp(rng.uniform(math.log(1e4), math.log(1e6))) if k < 2 else 1e5
        parts.append(dict(pts=pts, is_shell=sh, vol=_ellipsoid_volume(axes) / len(pts),
                          log_E=math.log(E), nu=0.3, mat=k, inst=k, v0=(0.0, 0.0, 0.0)))
    return _finish("gaussian_cloud", grid_res, dt, n_substeps, mats, parts, rng)


def large_scene(seed=2, n_total=2_000_000, grid_res=128, dt=5e-5, n_substeps=500) -> Scene:
    """Twelve ellipsoid instances in a 3x2x2 slot layout with uneven counts
    (log-uniform 2e4..4e5, rescaled to n_total), materials cycling
    fixed-corotated / von Mises / Drucker-Prager, per-instance v0 ~ N(0, 0.5)."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / grid_res
    lo, hi = 3 * dx, 1.0 - 3 * dx
    nslot = (3, 2, 2)
    size = [(hi - lo) / s for s in nslot]
    r_max = min(size) / 2 - 2 * dx
    n_k = np.exp(rng.uniform(math.log(2e4), math.log(4e5), 12))
    n_k = np.clip(n_k * (n_total / n_k.sum()), 1000, None)
    n_k = np.floor(n_k * (n_total / n_k.sum())).astype(np.int64)
    n_k[np.argmax(n_k)] += n_total - n_k.sum()
    mats = [_material(ELASTIC_FCR),
            _material(ELASTIC_HENCKY, PLASTIC_VON_MISES, yield_stress=1e3),
            _material(ELASTIC_HENCKY, PLASTIC_DRUCKER_PRAGER, friction_deg=30.0)]
    parts = []
    k = 0
    for ix in range(3):
        for iy in range(2):
            for iz in range(2):
                centre = (lo + (ix + 0.5) * size[0], lo + (iy + 0.5) * size[1], lo + (iz + 0.5) * size[2])
                r_k = r_max * min(1.0, (n_k[k] / 4e5)) ** (1.0 / 3.0)
                axes = r_k * np.array([1.0, rng.uniform(0.5, 1.0), rng.uniform(0.5, 1.0)])
                rot = haar_rotation(rng)
                ns = int(n_k[k]) // 2
                pts, sh = ellipsoid_instance(rng, centre, axes, rot, ns, int(n_k[k]) - ns)
                m = k % 3
                E = math.exp(rng.uniform(math.log(1e4), math.log(1e6))) if m == 0 else 1e5
                v0 = rng.normal(0.0, 0.5, 3)
                parts.append(dict(pts=pts, is_shell=sh, vol=_ellipsoid_volume(axes) / len(pts),
                                  log_E=math.log(E), nu=0.3, mat=m, inst=k, v0=v0))
                k += 1
    return _finish("large_scene", grid_res, dt, n_substeps, mats, parts, rng)


def colliding_pair(seed=3, n_total=200_000, grid_res=64, dt=1e-4, n_substeps=200,
                   checkpoint_every=20, E=(1e5, 1e5), nu=(0.3, 0.3)) -> Scene:
    """Two fixed-corotated ellipsoids (half shell, half interior) moving at
    +-1 m/s along x towards each other with a one-cell gap."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / grid_res
    per = n_total // 2
    parts = []
    axes = [rng.uniform(0.08, 0.15, 3) for _ in range(2)]
    rots = [haar_rotation(rng) for _ in range(2)]
    half = [np.sqrt(((r * a[None, :]) ** 2).sum(1)) for r, a in zip(rots, axes)]
    yc = 0.5
    xl = 0.5 - 0.5 * dx - half[0][0]
    xr = 0.5 + 0.5 * dx + half[1][0]
    for k, (cx, vx) in enumerate([(xl, 1.0), (xr, -1.0)]):
        n_k = per if k == 0 else n_total - per
        ns = n_k // 2
        pts, sh = ellipsoid_instance(rng, (cx, yc, 0.5), axes[k], rots[k], ns, n_k - ns)
        parts.append(dict(pts=pts, is_shell=sh, vol=_ellipsoid_volume(axes[k]) / len(pts),
                          log_E=math.log(E[k]), nu=nu[k], mat=0, inst=k, v0=(vx, 0.0, 0.0)))
    sc = _finish("colliding_pair", grid_res, dt, n_substeps, [_material(ELASTIC_FCR)], parts, rng,
                 checkpoint_every=checkpoint_every)
    return sc


def candidate_batch(seed=4, n_batch=64, grid_res=48, dt=1e-4, n_substeps=100,
                    n_min=10_000, n_max=100_000) -> Scene:
    """n_batch independent candidates, each a single fixed-corotated
    ellipsoid (half shell, half interior) on its own grid, falling at
    1.5 m/s with its lowest point 0.1 cell above the sticky floor band, so
    it lands within the first substeps and its deformation depends on E;
    per-candidate E (log-uniform 1e4..1e6) and nu (uniform 0.2..0.4), and
    hidden target parameters drawn alike."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / grid_res
    parts = []
    offsets = [0]
    tgt_logE, tgt_nu = [], []
    for b in range(n_batch):
        n_c = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        axes = rng.uniform(0.08, 0.2, 3)
        rot = haar_rotation(rng)
        half = np.sqrt(((rot * axes[None, :]) ** 2).sum(1))
        centre = (0.5, 3.6 * dx + half[1], 0.5)
        ns = n_c // 2
        pts, sh = ellipsoid_instance(rng, centre, axes, rot, ns, n_c - ns)
        E = math.exp(rng.uniform(math.log(1e4), math.log(1e6)))
        nu = rng.uniform(0.2, 0.4)
        tgt_logE.append(rng.uniform(math.log(1e4), math.log(1e6)))
        tgt_nu.append(rng.uniform(0.2, 0.4))
        parts.append(dict(pts=pts, is_shell=sh, vol=_ellipsoid_volume(axes) / len(pts),
                          log_E=math.log(E), nu=nu, mat=0, inst=b, v0=(0.0, -1.5, 0.0)))
        offsets.append(offsets[-1] + n_c)
    sc = _finish("candidate_batch", grid_res, dt, n_substeps, [_material(ELASTIC_FCR)], parts, rng,
                 offsets=offsets)
    sc.extras["target_log_E"] = np.asarray(tgt_logE, np.float32)
    sc.extras["target_nu"] = np.asarray(tgt_nu, np.float32)
    return sc


_CONFIGS = {
    "cube_lattice": cube_lattice,
    "cube_uniform": cube_uniform,
    "gaussian_cloud": gaussian_cloud,
    "large_scene": large_scene,
    "colliding_pair": colliding_pair,
    "candidate_batch": candidate_batch,
}


def make_scene(name: str, **kw) -> Scene:
    """Build a named scene; keyword arguments override the defaults (e.g.
    ``n_total`` for a reduced-size copy of an ellipsoid scene)."""
    return _CONFIGS[name](**kw)


def random_state(rng, n, grid_res, spread=0.3, vel=0.5, cgrad=2.0, fdev=0.05, centre=0.5):
    """Randomised particle state for unit and parity tests: positions well
    inside the wall band, random v, C and F near identity.  No physics."""
    lo = centre - spread / 2
    x = (lo + rng.uniform(0, spread, (n, 3))).astype(np.float32)
    v = rng.normal(0, vel, (n, 3)).astype(np.float32)
    C = rng.normal(0, cgrad, (n, 3, 3)).astype(np.float32)
    F = (np.eye(3) + rng.normal(0, fdev, (n, 3, 3))).astype(np.float32)
    return x, v, C, F


def mcis_inputs(seed=7, n_shell=(2000, 3000, 1500), cand_per_shell=2.0, fill_frac=0.5, r_range=(0.06, 0.16),
                empty_instances=()):
    """Inputs of the MCIS interior fill (Sec. 4.1) for ellipsoid instances:
    surface points on each shell (the Gaussian centres), candidates drawn
    uniformly in the instance's box and kept if inside the ellipsoid (the
    analytic occupancy test standing in for hull + ray casting), one uniform
    u in (0, 1] per candidate, and n_k = fill_frac x candidates.  Instances
    listed in ``empty_instances`` get no surface points.  Returns a dict of
    NumPy arrays: surface [S, 3], surface_offsets [K+1], candidates [M, 3],
    candidate_offsets [K+1], u [M], n_select [K]."""
    rng = np.random.default_rng(seed)
    surf, cand, so, co, nsel = [], [], [0], [0], []
    for k, ns in enumerate(n_shell):
        axes = rng.uniform(r_range[0], r_range[1], 3)
        rot = haar_rotation(rng)
        half = np.sqrt(((rot * axes[None, :]) ** 2).sum(1))
        centre = rng.uniform(half + 0.01, 1.0 - half - 0.01)
        d = rng.standard_normal((ns, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        shell = centre + (d * axes) @ rot.T
        want = int(cand_per_shell * ns)
        pts = []
        while sum(len(p) for p in pts) < want:
            q = centre + rng.uniform(-1.0, 1.0, (2 * want, 3)) * half
            loc = (q - centre) @ rot / axes
            pts.append(q[(loc ** 2).sum(1) < 1.0])
        c = np.concatenate(pts)[:want]
        if k not in empty_instances:
            surf.append(shell)
        cand.append(c)
        so.append(so[-1] + (0 if k in empty_instances else ns))
        co.append(co[-1] + len(c))
        nsel.append(int(fill_frac * len(c)))
    M = co[-1]
    return dict(surface=np.concatenate(surf).astype(np.float32) if surf else np.zeros((0, 3), np.float32),
                surface_offsets=np.array(so, np.int64), candidates=np.concatenate(cand).astype(np.float32),
                candidate_offsets=np.array(co, np.int64), u=1.0 - rng.uniform(0.0, 1.0, M),
                n_select=np.array(nsel, np.int64))


# ---------------------------------------------------------------------------
# Inputs of the candidate generation (Sec. 4.1): per instance a closed
# triangle mesh (the convex hull of its points) and raw uniforms
# ---------------------------------------------------------------------------

def _box_index(x, y, z):
    return x + 2 * y + 4 * z


def box_mesh(lo, hi, drop=()):
    """Triangle mesh of the axis-aligned box [lo, hi]^3 (scalars or 3-vectors):
    8 vertices (vertex x + 2y + 4z at the corner (x, y, z) in {lo, hi}), two
    triangles per face split along the diagonal from the face's lowest
    corner.  Faces named in ``drop`` ("-x", "+x", "-y", "+y", "-z", "+z") are
    left out, which opens the mesh.  Returns (vertices [8, 3] float32,
    triangles [T, 3] int32)."""
    lo = np.broadcast_to(np.asarray(lo, np.float32), (3,))
    hi = np.broadcast_to(np.asarray(hi, np.float32), (3,))
    v = np.array([[(lo, hi)[(i >> a) & 1][a] for a in range(3)] for i in range(8)], np.float32)
    quads = {}
    for s, name in ((0, "-"), (1, "+")):
        quads[name + "x"] = [_box_index(s, 0, 0), _box_index(s, 1, 0), _box_index(s, 1, 1), _box_index(s, 0, 1)]
        quads[name + "y"] = [_box_index(0, s, 0), _box_index(0, s, 1), _box_index(1, s, 1), _box_index(1, s, 0)]
        quads[name + "z"] = [_box_index(0, 0, s), _box_index(1, 0, s), _box_index(1, 1, s), _box_index(0, 1, s)]
    tris = []
    for name in ("-x", "+x", "-y", "+y", "-z", "+z"):
        if name in drop:
            continue
        q = quads[name]
        tris += [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
    return v, np.array(tris, np.int32).reshape(-1, 3)


def merge_meshes(*meshes):
    """One mesh of several (vertices, triangles) pairs (indices shifted)."""
    vs, ts, n = [], [], 0
    for v, t in meshes:
        vs.append(np.asarray(v, np.float32))
        ts.append(np.asarray(t, np.int64) + n)
        n += len(v)
    return np.concatenate(vs), np.concatenate(ts).astype(np.int32)


def octahedron_mesh(centre, r):
    """The octahedron with vertices centre +- r along each axis (8 triangles)."""
    c = np.asarray(centre, np.float32)
    v = np.array([c + s * r * e for e in np.eye(3, dtype=np.float32) for s in (-1, 1)], np.float32)
    tris = [(ix, iy, iz) for ix in (0, 1) for iy in (2, 3) for iz in (4, 5)]
    return v, np.array(tris, np.int32)


def ellipsoid_hull(rng, n_shell, r_range=(0.06, 0.16)):
    """Points on a random ellipsoid shell in the unit cube (float32) and
    their convex hull's triangles (Quickhull via SciPy's Qhull, run on the
    float32 values).  Returns (points [n, 3] float32, triangles [T, 3] int32,
    hull volume)."""
    from scipy.spatial import ConvexHull
    axes = rng.uniform(r_range[0], r_range[1], 3)
    rot = haar_rotation(rng)
    half = np.sqrt(((rot * axes[None, :]) ** 2).sum(1))
    centre = rng.uniform(half + 0.01, 1.0 - half - 0.01)
    d = rng.standard_normal((n_shell, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = (centre + (d * axes) @ rot.T).astype(np.float32)
    hull = ConvexHull(pts.astype(np.float64))
    return pts, hull.simplices.astype(np.int32), float(hull.volume)


def ipf_inputs(seed=8, n_shell=(1500, 2500, 1000), raw_per_point=4.0, meshes=(), raw_per_mesh=2000,
               r_range=(0.06, 0.16)):
    """Inputs of the candidate generation for ellipsoid instances (shell
    points and their hull) followed by the given extra meshes (each a
    (vertices, triangles) pair, one instance each).  Instance k gets
    raw_per_point x its points (ellipsoids) or raw_per_mesh (extra meshes)
    raw candidates with three uniforms each.  Returns a dict of NumPy arrays:
    hull_vertices [V, 3] float32, hull_vertex_offsets [K+1], hull_triangles
    [T, 3] int32 (local to the instance), hull_triangle_offsets [K+1], u
    [R, 3] float64 in [0, 1), raw_offsets [K+1], surface / surface_offsets
    (the instance's points, for the selection that follows) and
    hull_volume [K] (NaN for the extra meshes)."""
    rng = np.random.default_rng(seed)
    vs, ts, raws, vols = [], [], [], []
    for ns in n_shell:
        p, t, vol = ellipsoid_hull(rng, ns, r_range)
        vs.append(p)
        ts.append(t)
        raws.append(int(raw_per_point * ns))
        vols.append(vol)
    for v, t in meshes:
        vs.append(np.asarray(v, np.float32).reshape(-1, 3))
        ts.append(np.asarray(t, np.int32).reshape(-1, 3))
        raws.append(int(raw_per_mesh))
        vols.append(math.nan)
    off = lambda sizes: np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    vo = off([len(v) for v in vs])
    R = int(sum(raws))
    return dict(hull_vertices=np.concatenate(vs).astype(np.float32), hull_vertex_offsets=vo,
                hull_triangles=np.concatenate(ts).astype(np.int32), hull_triangle_offsets=off([len(t) for t in ts]),
                u=rng.uniform(0.0, 1.0, (R, 3)), raw_offsets=off(raws),
                surface=np.concatenate(vs).astype(np.float32), surface_offsets=vo.copy(),
                hull_volume=np.array(vols, np.float64))
