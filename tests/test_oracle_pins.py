"""Pins of the FP64 oracle against facts fixed outside it: brute-force node
sums, closed-form trajectories, conservation laws, energy derivatives,
textbook elasticity, objectivity and the return maps' defining properties."""
import math

import numpy as np
import pytest
import torch

from oracle import mpm_oracle as O

F64 = torch.float64


def rot(rng):
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return torch.tensor(q)


def bspline_1d(u):
    """Quadratic B-spline N(u) of the node-to-particle distance in cells."""
    u = abs(u)
    if u < 0.5:
        return 0.75 - u * u
    if u < 1.5:
        return 0.5 * (1.5 - u) ** 2
    return 0.0


# --------------------------------------------------------------------------
# B-spline weights: partition of unity, zero first moment, D_p = dx^2/4 I
# --------------------------------------------------------------------------

def test_bspline_moments_and_continuity():
    x = torch.tensor(np.random.default_rng(0).uniform(0.2, 0.8, (2000, 3)))
    n = 32
    base, fx, w = O.stencil(x, n)
    o = torch.arange(3, dtype=F64)[None, :, None]
    d = o - fx[:, None, :]
    assert torch.allclose(w.sum(1), torch.ones(2000, 3, dtype=F64), atol=1e-15)
    assert torch.allclose((w * d).sum(1), torch.zeros(2000, 3, dtype=F64), atol=1e-14)
    # second moment 1/4 cell^2: the inverse is the 4/dx^2 of the P2G / G2P formulas
    assert torch.allclose((w * d * d).sum(1), torch.full((2000, 3), 0.25, dtype=F64), atol=1e-14)
    # weights equal the brute-force kernel of the distance
    for i in range(20):
        for a in range(3):
            for ax in range(3):
                u = float(fx[i, ax]) - a
                assert abs(float(w[i, a, ax]) - bspline_1d(u)) < 1e-15
    # C0 / C1 continuity at f = 0.5 and 1.5: the dropped node has zero weight
    for f in (0.5, 1.5 - 1e-12):
        xx = torch.tensor([[(10 + f) / n] * 3], dtype=F64)
        _, fx1, w1 = O.stencil(xx, n)
        assert float(w1[0, 2 if f == 0.5 else 0, 0]) < 1e-12


# --------------------------------------------------------------------------
# P2G / G2P against brute-force sums over every node
# --------------------------------------------------------------------------

def _tiny(rng, N, n):
    x = torch.tensor(rng.uniform(0.3, 0.7, (N, 3)))
    v = torch.tensor(rng.normal(0, 1, (N, 3)))
    C = torch.tensor(rng.normal(0, 5, (N, 3, 3)))
    tau = torch.tensor(rng.normal(0, 1e3, (N, 3, 3)))
    mass = torch.tensor(rng.uniform(0.5, 2.0, N))
    vol = torch.tensor(rng.uniform(1e-4, 3e-4, N))
    return x, v, C, tau, mass, vol


@pytest.mark.parametrize("N", [2, 5, 8])
def test_p2g_bruteforce(N):
    rng = np.random.default_rng(N)
    n, dt = 8, 1e-3
    x, v, C, tau, mass, vol = _tiny(rng, N, n)
    m, mv = O.p2g(x, v, C, tau, mass, vol, n, dt)
    dx = 1.0 / n
    m_bf = np.zeros(n ** 3)
    mv_bf = np.zeros((n ** 3, 3))
    for p in range(N):
        xp = x[p].numpy()
        A = mass[p].item() * C[p].numpy() - 4 * n * n * dt * vol[p].item() * tau[p].numpy()
        for i in range(n):
            for j in range(n):
                for k in range(n):
                    xi = np.array([i, j, k]) * dx
                    w = 1.0
                    for ax in range(3):
                        w *= bspline_1d((xp[ax] - xi[ax]) / dx)
                    if w == 0.0:
                        continue
                    lin = (i * n + j) * n + k
                    m_bf[lin] += w * mass[p].item()
                    mv_bf[lin] += w * (mass[p].item() * v[p].numpy() + A @ (xi - xp))
    np.testing.assert_allclose(m.numpy(), m_bf, rtol=0, atol=1e-14 * m_bf.max())
    np.testing.assert_allclose(mv.numpy(), mv_bf, rtol=0, atol=1e-13 * np.abs(mv_bf).max())


def test_g2p_bruteforce():
    rng = np.random.default_rng(7)
    n, dt, N = 8, 1e-3, 6
    x = torch.tensor(rng.uniform(0.3, 0.7, (N, 3)))
    F = torch.tensor(np.eye(3) + rng.normal(0, 0.1, (N, 3, 3)))
    vg = torch.tensor(rng.normal(0, 1, (n ** 3, 3)))
    x1, v1, C1, F1 = O.g2p(x, F, vg, n, dt)
    dx = 1.0 / n
    for p in range(N):
        xp = x[p].numpy()
        vs = np.zeros(3)
        B = np.zeros((3, 3))
        for i in range(n):
            for j in range(n):
                for k in range(n):
                    xi = np.array([i, j, k]) * dx
                    w = np.prod([bspline_1d((xp[a] - xi[a]) / dx) for a in range(3)])
                    vi = vg[(i * n + j) * n + k].numpy()
                    vs += w * vi
                    B += w * np.outer(vi, xi - xp)
        Cp = 4 / dx ** 2 * B
        np.testing.assert_allclose(v1[p].numpy(), vs, atol=1e-14)
        np.testing.assert_allclose(C1[p].numpy(), Cp, atol=1e-11)
        np.testing.assert_allclose(x1[p].numpy(), xp + dt * vs, atol=1e-15)
        np.testing.assert_allclose(F1[p].numpy(), (np.eye(3) + dt * Cp) @ F[p].numpy(), atol=1e-13)


# --------------------------------------------------------------------------
# Conservation and closed-form trajectories
# --------------------------------------------------------------------------

def _params(N, n, dt, gravity=(0, 0, 0), bound=0, E=1e5, nu=0.3, mats=None, mat_id=None, rng=None):
    mats = mats or [dict(elastic=0, plastic=0, yield_stress=0.0, friction_deg=0.0)]
    rng = rng or np.random.default_rng(0)
    mass = rng.uniform(0.5, 2.0, N) * 1e-3
    vol = mass / 1000.0
    return O.Params(mass, vol, np.full(N, math.log(E)), np.full(N, nu),
                    np.zeros(N, np.int64) if mat_id is None else mat_id, mats, n, dt, gravity, bound)


def test_mass_and_momentum_conservation():
    rng = np.random.default_rng(1)
    N, n, dt = 300, 16, 1e-4
    x = torch.tensor(rng.uniform(0.3, 0.7, (N, 3)))
    v = torch.tensor(rng.normal(0, 1, (N, 3)))
    C = torch.tensor(rng.normal(0, 3, (N, 3, 3)))
    F = torch.tensor(np.eye(3) + rng.normal(0, 0.05, (N, 3, 3)))
    p = _params(N, n, dt, rng=rng)
    (x1, v1, C1, F1), grids = O.substep((x, v, C, F), p, return_grid=True)
    m, mv, vg = grids[0]
    assert abs(m.sum().item() - p.mass.sum().item()) < 1e-15 * p.mass.sum().item() * 10
    P0 = (p.mass[:, None] * v).sum(0)
    # stress and affine terms carry no net momentum (zero first moment)
    assert torch.allclose(mv.sum(0), P0, rtol=1e-12, atol=1e-15)
    # G2P returns it: sum_p m_p v'_p = sum_i m_i v_i
    assert torch.allclose((p.mass[:, None] * v1).sum(0), (m[:, None] * vg).sum(0), rtol=1e-12, atol=1e-15)
    assert torch.allclose((p.mass[:, None] * v1).sum(0), P0, rtol=1e-10, atol=1e-14)


def test_apic_affine_field_reproduced():
    """v_p = a + B x_p, C_p = B, F = I (tau = 0): one substep returns
    v'_p = a + B x_p and C'_p = B exactly (pins 4/dx^2, dpos sign, APIC)."""
    rng = np.random.default_rng(2)
    N, n, dt = 400, 16, 1e-4
    x = torch.tensor(rng.uniform(0.3, 0.7, (N, 3)))
    a = torch.tensor(rng.normal(0, 1, 3))
    B = torch.tensor(rng.normal(0, 2, (3, 3)))
    v = a + x @ B.T
    C = B.expand(N, 3, 3).clone()
    F = torch.eye(3, dtype=F64).expand(N, 3, 3).clone()
    p = _params(N, n, dt, rng=rng)
    x1, v1, C1, F1 = O.substep((x, v, C, F), p)
    assert torch.allclose(v1, a + x @ B.T, atol=1e-12)
    assert torch.allclose(C1, C, atol=1e-10)
    assert torch.allclose(x1, x + dt * v1, atol=1e-15)


def test_free_fall_closed_form():
    rng = np.random.default_rng(3)
    N, n, dt, steps = 200, 16, 1e-3, 25
    g = torch.tensor([0.0, -9.8, 0.0], dtype=F64)
    x0 = torch.tensor(rng.uniform(0.4, 0.6, (N, 3)))
    v = torch.zeros(N, 3, dtype=F64)
    C = torch.zeros(N, 3, 3, dtype=F64)
    F = torch.eye(3, dtype=F64).expand(N, 3, 3).clone()
    p = _params(N, n, dt, gravity=(0, -9.8, 0), bound=0, rng=rng)
    x1, v1, C1, F1 = O.step_n((x0, v, C, F), p, steps)
    assert torch.allclose(v1, (steps * dt * g).expand(N, 3), atol=1e-12)
    assert torch.allclose(x1, x0 + dt * dt * g * steps * (steps + 1) / 2, atol=1e-13)
    assert torch.allclose(C1, torch.zeros_like(C1), atol=1e-9)
    assert torch.allclose(F1, F, atol=1e-12)


def test_sticky_wall_stops_particles():
    n, dt = 32, 1e-4
    # x/dx = 1.4: base 0, stencil nodes 0..2 on x, all inside the 3-node wall band
    x = torch.tensor([[1.4 / n, 0.5, 0.5], [0.5, 0.5, 0.5]], dtype=F64)
    v = torch.tensor([[-1.0, 0.3, 0.0], [0.0, 0.0, 0.0]], dtype=F64)
    C = torch.zeros(2, 3, 3, dtype=F64)
    F = torch.eye(3, dtype=F64).expand(2, 3, 3).clone()
    p = _params(2, n, dt, gravity=(0, -9.8, 0), bound=3)
    x1, v1, C1, F1 = O.substep((x, v, C, F), p)
    assert torch.all(v1[0] == 0)
    assert torch.allclose(v1[1], torch.tensor([0, -9.8 * dt, 0], dtype=F64), atol=1e-14)


# --------------------------------------------------------------------------
# SVD convention
# --------------------------------------------------------------------------

def test_svd_rotation_convention():
    rng = np.random.default_rng(4)
    F = torch.tensor(rng.normal(0, 1, (500, 3, 3)))
    F[:3] = torch.eye(3, dtype=F64)
    F[3] = torch.diag(torch.tensor([2.0, 2.0, -0.5], dtype=F64))  # inverted
    F[4] = torch.tensor([[1.0, 2, 3], [2, 4, 6], [0, 1, 0]], dtype=F64)  # singular
    U, S, V = O.svd_rot(F)
    rec = U @ torch.diag_embed(S) @ V.transpose(-1, -2)
    assert torch.allclose(rec, F, atol=1e-13)
    assert torch.allclose(torch.linalg.det(U), torch.ones(500, dtype=F64), atol=1e-13)
    assert torch.allclose(torch.linalg.det(V), torch.ones(500, dtype=F64), atol=1e-13)
    assert torch.all(S[:, 0] >= S[:, 1]) and torch.all(S[:, 1] >= S[:, 2].abs() - 1e-14)
    assert torch.all(S[:, :2] >= 0)
    detF = torch.linalg.det(F)
    nz = detF.abs() > 1e-9
    assert torch.all(torch.sign(S[nz, 2]) == torch.sign(detF[nz]))
    # magnitudes are the eigenvalue square roots of F^T F
    ev = torch.linalg.eigvalsh(F.transpose(-1, -2) @ F).flip(-1).clamp(min=0).sqrt()
    assert torch.allclose(S.abs(), ev, atol=1e-7)


# --------------------------------------------------------------------------
# Stress models
# --------------------------------------------------------------------------

def _energy_fcr(F, mu, lam):
    U, S, V = np.linalg.svd(F)
    R = U @ V
    if np.linalg.det(R) < 0:  # rotation of the polar factor
        U[:, 2] *= -1
        R = U @ V
    J = np.linalg.det(F)
    return mu * np.sum((F - R) ** 2) + 0.5 * lam * (J - 1) ** 2


def _energy_hencky(F, mu, lam):
    s = np.linalg.svd(F, compute_uv=False)
    e = np.log(s)
    return mu * np.sum(e * e) + 0.5 * lam * e.sum() ** 2


def _energy_neo_hookean(F, mu, lam):
    lnJ = np.log(np.linalg.det(F))
    return 0.5 * mu * (np.sum(F * F) - 3.0) - mu * lnJ + 0.5 * lam * lnJ ** 2


def _energy_stvk(F, mu, lam):
    E = 0.5 * (F.T @ F - np.eye(3))
    return mu * np.sum(E * E) + 0.5 * lam * np.trace(E) ** 2


def _energy_fluid(F, mu, lam):
    return 0.5 * lam * (np.linalg.det(F) - 1.0) ** 2


def _energy_volume(F, mu, lam):
    # d/dJ of kappa (J + 1/J - 2) is kappa (1 - J^-2); times J: kappa (J - 1/J)
    J = np.linalg.det(F)
    return (2.0 / 3.0 * mu + lam) * (J + 1.0 / J - 2.0)


ENERGY_MODELS = {
    "fcr": (_energy_fcr, O.tau_fixed_corotated), "hencky": (_energy_hencky, O.tau_hencky),
    "neo_hookean": (_energy_neo_hookean, O.tau_neo_hookean), "stvk": (_energy_stvk, O.tau_stvk),
    "fluid": (_energy_fluid, O.tau_fluid), "volume": (_energy_volume, O.tau_volume)}


@pytest.mark.parametrize("model", sorted(ENERGY_MODELS))
def test_stress_is_energy_derivative(model):
    """tau = (dPsi/dF) F^T, with dPsi/dF from central differences of the
    textbook energies (fixed corotated: mu|F-R|^2 + lam/2 (J-1)^2;
    Hencky: mu|log S|^2 + lam/2 tr(log S)^2; Neo-Hookean (Bonet & Wood):
    mu/2 (|F|^2 - 3) - mu log J + lam/2 (log J)^2; StVK: mu|E|^2 + lam/2 tr(E)^2;
    fluid: lam/2 (J - 1)^2; volume: kappa (J + 1/J - 2))."""
    rng = np.random.default_rng(5)
    mu, lam = 3.0e4, 5.0e4
    energy, fn = ENERGY_MODELS[model]
    done = 0
    while done < 10:
        F = np.eye(3) + rng.normal(0, 0.2, (3, 3))
        if np.linalg.det(F) < 0.2:
            continue
        done += 1
        h = 1e-6
        P = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                d = np.zeros((3, 3))
                d[i, j] = h
                P[i, j] = (energy(F + d, mu, lam) - energy(F - d, mu, lam)) / (2 * h)
        tau = fn(torch.tensor(F)[None], torch.tensor([mu]), torch.tensor([lam]))[0].numpy()
        np.testing.assert_allclose(tau, P @ F.T, rtol=0, atol=2e-5 * np.abs(P @ F.T).max())


def test_first_piola_forms_of_appendix_A2():
    """App. A.2 writes P; App. B.1 writes tau.  P F^T must equal tau."""
    rng = np.random.default_rng(6)
    F = torch.tensor(np.eye(3) + rng.normal(0, 0.2, (50, 3, 3)))
    mu = torch.tensor(rng.uniform(1e3, 1e5, 50))
    lam = torch.tensor(rng.uniform(1e3, 1e5, 50))
    U, S, V = O.svd_rot(F)
    R = U @ V.transpose(-1, -2)
    J = torch.linalg.det(F)
    FinvT = torch.linalg.inv(F).transpose(-1, -2)
    P_fcr = 2 * mu[:, None, None] * (F - R) + (lam * J * (J - 1))[:, None, None] * FinvT
    ln = torch.log(S)
    P_h = U @ torch.diag_embed(2 * mu[:, None] * ln / S + (lam * ln.sum(-1))[:, None] / S) @ V.transpose(-1, -2)
    FT = F.transpose(-1, -2)
    assert torch.allclose(P_fcr @ FT, O.tau_fixed_corotated(F, mu, lam), rtol=1e-10, atol=1e-8)
    assert torch.allclose(P_h @ FT, O.tau_hencky(F, mu, lam), rtol=1e-10, atol=1e-8)
    P_nh = mu[:, None, None] * (F - FinvT) + (lam * torch.log(J))[:, None, None] * FinvT
    assert torch.allclose(P_nh @ FT, O.tau_neo_hookean(F, mu, lam), rtol=1e-10, atol=1e-8)


@pytest.mark.parametrize("fn", [O.tau_fixed_corotated, O.tau_hencky, O.tau_neo_hookean, O.tau_stvk, O.tau_fluid,
                                O.tau_volume])
def test_stress_rest_objectivity_linearity(fn):
    rng = np.random.default_rng(8)
    mu, lam = O.lame(torch.tensor([math.log(1e5)] * 40, dtype=F64), torch.tensor([0.3] * 40, dtype=F64))
    eye = torch.eye(3, dtype=F64).expand(40, 3, 3)
    assert torch.allclose(fn(eye.clone(), mu, lam), torch.zeros(40, 3, 3, dtype=F64), atol=1e-9)
    F = torch.tensor(np.eye(3) + rng.normal(0, 0.2, (40, 3, 3)))
    Q = torch.stack([rot(rng) for _ in range(40)])
    t = fn(F, mu, lam)
    assert torch.allclose(fn(Q @ F, mu, lam), Q @ t @ Q.transpose(-1, -2), rtol=1e-9, atol=1e-7)
    assert torch.allclose(fn(F @ Q, mu, lam), t, rtol=1e-9, atol=1e-7)  # isotropy
    assert torch.allclose(fn(F, 2.5 * mu, 2.5 * lam), 2.5 * t, rtol=1e-12, atol=1e-8)
    assert torch.allclose(t, t.transpose(-1, -2), atol=1e-8)


def test_lame_matches_uniaxial_linear_elasticity():
    """Textbook meaning of (E, nu): uniaxial stress s_xx = E e with lateral
    strain -nu e and no lateral stress; small-strain limit of both models."""
    E, nu = 2.0e5, 0.27
    mu, lam = O.lame(torch.tensor([math.log(E)]), torch.tensor([nu], dtype=F64))
    e = 1e-7
    F = torch.diag(torch.tensor([1 + e, 1 - nu * e, 1 - nu * e], dtype=F64))[None]
    for fn in (O.tau_fixed_corotated, O.tau_hencky, O.tau_neo_hookean, O.tau_stvk):
        t = fn(F, mu, lam)[0]
        assert abs(t[0, 0].item() / e - E) < 1e-5 * E
        assert abs(t[1, 1].item() / e) < 1e-5 * E
        assert abs(t[2, 2].item() / e) < 1e-5 * E


def test_diagonal_closed_forms():
    s = torch.tensor([1.2, 0.9, 0.8], dtype=F64)
    F = torch.diag(s)[None]
    mu, lam = torch.tensor([1.0e4], dtype=F64), torch.tensor([2.0e4], dtype=F64)
    J = s.prod()
    fcr = torch.diag(2 * mu * (s - 1) * s + lam * J * (J - 1))
    hen = torch.diag(2 * mu * torch.log(s) + lam * torch.log(s).sum())
    assert torch.allclose(O.tau_fixed_corotated(F, mu, lam)[0], fcr, atol=1e-9)
    assert torch.allclose(O.tau_hencky(F, mu, lam)[0], hen, atol=1e-9)
    nh = torch.diag(mu * (s * s - 1) + lam * torch.log(J))
    gl = 0.5 * (s * s - 1)
    stvk = torch.diag(s * s * (2 * mu * gl + lam * gl.sum()))
    kappa = 2.0 / 3.0 * mu + lam
    assert torch.allclose(O.tau_neo_hookean(F, mu, lam)[0], nh, atol=1e-9)
    assert torch.allclose(O.tau_stvk(F, mu, lam)[0], stvk, atol=1e-9)
    assert torch.allclose(O.tau_fluid(F, mu, lam)[0], torch.eye(3, dtype=F64) * lam * J * (J - 1), atol=1e-9)
    assert torch.allclose(O.tau_volume(F, mu, lam)[0], torch.eye(3, dtype=F64) * kappa * (J - 1 / J), atol=1e-9)


def test_volume_model_small_strain_bulk_response():
    """kappa (J - 1/J) ~ 2 kappa (J - 1) near J = 1: pressure linear in the
    volume change, no shear response, and the J floor only below 1e-4."""
    mu, lam = torch.tensor([1.0e4], dtype=F64), torch.tensor([2.0e4], dtype=F64)
    kappa = 2.0 / 3.0 * 1.0e4 + 2.0e4
    e = 1e-7
    t = O.tau_volume(torch.diag(torch.tensor([1 + e, 1.0, 1.0], dtype=F64))[None], mu, lam)[0]
    assert abs(t[0, 0].item() / e - 2 * kappa) < 1e-5 * kappa and abs(t[0, 1].item()) == 0.0
    shear = torch.tensor([[1.0, 0.3, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]], dtype=F64)[None]  # J = 1
    assert torch.allclose(O.tau_volume(shear, mu, lam), torch.zeros(1, 3, 3, dtype=F64), atol=1e-9)
    tiny = torch.diag(torch.tensor([1e-5, 1.0, 1.0], dtype=F64))[None]
    assert abs(O.tau_volume(tiny, mu, lam)[0, 0, 0].item() - kappa * (1e-5 - 1e4)) < 1e-6 * kappa * 1e4


# --------------------------------------------------------------------------
# Return maps
# --------------------------------------------------------------------------

def _logsv(F):
    s = np.linalg.svd(F.numpy(), compute_uv=False)
    return np.log(s)


def test_von_mises_return():
    rng = np.random.default_rng(9)
    N = 200
    F = torch.tensor(np.eye(3) + rng.normal(0, 0.05, (N, 3, 3)))
    F = torch.tensor(np.eye(3) + rng.normal(0, 0.05, (N, 3, 3)))
    mu = torch.full((N,), 3.0e4, dtype=F64)
    sy = 1e3
    F1 = O.return_von_mises(F, mu, sy)
    yielded = 0
    for i in range(N):
        e0, e1 = _logsv(F[i:i + 1])[0], _logsv(F1[i:i + 1])[0]
        dev0 = e0 - e0.mean()
        dev1 = e1 - e1.mean()
        assert abs(e0.sum() - e1.sum()) < 1e-12            # volume preserved
        if np.linalg.norm(dev0) > sy / (2 * 3.0e4):
            yielded += 1
            assert abs(np.linalg.norm(dev1) - sy / (2 * 3.0e4)) < 1e-12  # on the surface
        else:
            assert torch.equal(F1[i], F[i])
    assert yielded > 50
    # idempotent; equivariant under rotations on both sides
    assert torch.allclose(O.return_von_mises(F1, mu, sy), F1, atol=1e-12)
    Q = torch.stack([rot(rng) for _ in range(N)])
    W = torch.stack([rot(rng) for _ in range(N)])
    assert torch.allclose(O.return_von_mises(Q @ F @ W, mu, sy), Q @ F1 @ W, atol=1e-12)


def test_drucker_prager_return():
    rng = np.random.default_rng(10)
    N = 300
    F = torch.tensor(np.eye(3) + rng.normal(0, 0.05, (N, 3, 3)))
    mu, lam = O.lame(torch.full((N,), math.log(1e5), dtype=F64), torch.full((N,), 0.3, dtype=F64))
    phi = 30.0
    alpha = O.drucker_prager_alpha(phi)
    assert abs(alpha - math.sqrt(2 / 3) * 2 * 0.5 / 2.5) < 1e-15
    F1 = O.return_drucker_prager(F, mu, lam, phi)
    c = (3 * lam[0] + 2 * mu[0]).item() / (2 * mu[0].item())
    n_t = n_c = n_e = 0
    for i in range(N):
        e0 = _logsv(F[i:i + 1])[0]
        if e0.sum() > 0:   # tension: projected to the tip, F' = U V^T (a rotation)
            n_t += 1
            assert abs(np.linalg.det(F1[i].numpy()) - 1) < 1e-12
            np.testing.assert_allclose(F1[i].numpy() @ F1[i].numpy().T, np.eye(3), atol=1e-12)
            continue
        dev0 = e0 - e0.mean()
        dg = np.linalg.norm(dev0) + c * e0.sum() * alpha
        e1 = _logsv(F1[i:i + 1])[0]
        if dg <= 0:
            n_e += 1
            assert torch.equal(F1[i], F[i])
        else:      # lands on the cone, same trace
            n_c += 1
            assert abs(e1.sum() - e0.sum()) < 1e-12
            assert abs(np.linalg.norm(e1 - e1.mean()) + c * e1.sum() * alpha) < 1e-12
    assert n_t > 10 and n_c > 10 and n_e > 10
    assert torch.allclose(O.return_drucker_prager(F1, mu, lam, phi), F1, atol=1e-12)


def test_fluid_and_sigma_return_maps():
    """Fluid plasticity keeps det F and drops every deviatoric part; sigma
    plasticity does the same with det F clamped to [0.05, 1.2]."""
    rng = np.random.default_rng(13)
    F = torch.tensor(np.eye(3) + rng.normal(0, 0.4, (300, 3, 3)))
    J = torch.linalg.det(F)
    assert bool((J < 0).any()) and bool((J > 1.2).any()) and bool(((J > 0) & (J < 0.05)).any())
    eye = torch.eye(3, dtype=F64)
    f = O.return_fluid(F)
    assert torch.allclose(torch.linalg.det(f), J, rtol=1e-12, atol=1e-15)
    assert torch.allclose(f - f[:, :1, :1] * eye, torch.zeros_like(f), atol=0)
    s = O.return_sigma(F)
    Jc = torch.clamp(J, 0.05, 1.2)
    assert torch.allclose(torch.linalg.det(s), Jc, rtol=1e-12)
    inside = (J >= 0.05) & (J <= 1.2)
    assert torch.equal(s[inside], f[inside])
    mats = [dict(elastic=0, plastic=O.PLASTIC_FLUID, yield_stress=0.0, friction_deg=0.0),
            dict(elastic=0, plastic=O.PLASTIC_SIGMA, yield_stress=0.0, friction_deg=0.0)]
    mid = torch.tensor(rng.integers(0, 2, 300))
    mu = torch.full((300,), 1e4, dtype=F64)
    out = O.plasticity(F, mu, mu, mid, mats)
    assert torch.equal(out[mid == 0], f[mid == 0]) and torch.equal(out[mid == 1], s[mid == 1])


# --------------------------------------------------------------------------
# Adjoint oracle: differentiable pieces and finite differences
# --------------------------------------------------------------------------

def test_differentiable_stress_matches_svd_stress():
    rng = np.random.default_rng(11)
    F = torch.tensor(np.eye(3) + rng.normal(0, 0.15, (64, 3, 3)))
    assert bool((torch.linalg.det(F) > 0).all())
    mu = torch.tensor(rng.uniform(1e3, 1e5, 64))
    lam = torch.tensor(rng.uniform(1e3, 1e5, 64))
    a = O._tau_fcr_differentiable(F, mu, lam)
    assert torch.allclose(a, O.tau_fixed_corotated(F, mu, lam), rtol=1e-11, atol=1e-8)
    b = O._tau_hencky_differentiable(F, mu, lam)
    assert torch.allclose(b, O.tau_hencky(F, mu, lam), rtol=1e-9, atol=1e-6)


def _small_elastic_scene(rng, N=150, n=16, dt=2e-4, mats=None, mat_id=None):
    x = torch.tensor(rng.uniform(0.35, 0.65, (N, 3)))
    v = torch.tensor(rng.normal(0, 0.5, (N, 3)))
    C = torch.tensor(rng.normal(0, 2.0, (N, 3, 3)))
    F = torch.tensor(np.eye(3) + rng.normal(0, 0.03, (N, 3, 3)))
    p = _params(N, n, dt, gravity=(0, -9.8, 0), bound=3, E=1e4, nu=0.3, mats=mats, mat_id=mat_id, rng=rng)
    p.log_E = p.log_E + torch.tensor(rng.normal(0, 0.3, N))
    p.nu = p.nu + torch.tensor(rng.uniform(-0.05, 0.05, N))
    return (x, v, C, F), p


PLASTIC_CASES = [
    [dict(elastic=1, plastic=O.PLASTIC_VON_MISES, yield_stress=100.0, friction_deg=0.0)],
    [dict(elastic=0, plastic=O.PLASTIC_VON_MISES, yield_stress=200.0, friction_deg=0.0)],
    [dict(elastic=1, plastic=O.PLASTIC_DRUCKER_PRAGER, yield_stress=0.0, friction_deg=30.0)],
    [dict(elastic=0, plastic=O.PLASTIC_FLUID, yield_stress=0.0, friction_deg=0.0)],
    [dict(elastic=1, plastic=O.PLASTIC_SIGMA, yield_stress=0.0, friction_deg=0.0)],
    [dict(elastic=0, plastic=0, yield_stress=0.0, friction_deg=0.0),
     dict(elastic=1, plastic=O.PLASTIC_VON_MISES, yield_stress=100.0, friction_deg=0.0),
     dict(elastic=1, plastic=O.PLASTIC_DRUCKER_PRAGER, yield_stress=0.0, friction_deg=25.0),
     dict(elastic=2, plastic=O.PLASTIC_SIGMA, yield_stress=0.0, friction_deg=0.0)],
]


def test_differentiable_return_maps_match_svd_return_maps():
    """The matrix-function forms of the von Mises and Drucker-Prager return
    maps equal the SVD forms (App. A.2), in yield, tension and elastic cases."""
    rng = np.random.default_rng(13)
    N = 400
    F = torch.tensor(np.eye(3) + rng.normal(0, 0.1, (N, 3, 3)))
    assert bool((torch.linalg.det(F) > 0).all())
    mu = torch.tensor(rng.uniform(1e4, 1e5, N))
    lam = torch.tensor(rng.uniform(1e4, 1e5, N))
    vm = O.return_von_mises(F, mu, 8e3)
    moved = (vm - F).abs().amax((1, 2)) > 0
    assert 0 < int(moved.sum()) < N  # both branches present
    assert torch.allclose(O._return_von_mises_differentiable(F, mu, 8e3), vm, rtol=0, atol=1e-12)
    dp = O.return_drucker_prager(F, mu, lam, 30.0)
    tr = torch.log(torch.linalg.svdvals(F)).sum(-1)
    assert bool((tr > 0).any()) and bool((tr < 0).any())
    assert torch.allclose(O._return_drucker_prager_differentiable(F, mu, lam, 30.0), dp, rtol=0, atol=1e-12)


@pytest.mark.parametrize("mats", [[dict(elastic=e, plastic=0, yield_stress=0.0, friction_deg=0.0)]
                                  for e in range(6)] + PLASTIC_CASES,
                         ids=[f"elastic{e}" for e in range(6)] + ["vm_hencky", "vm_fcr", "dp", "fluid", "sigma",
                                                                  "mixed"])
def test_adjoint_matches_central_differences(mats):
    """The oracle's autograd adjoint against central differences of its SVD
    forward, along random +-1 directions of log E and nu and a random x0
    direction.  Plastic cases use small steps so that no particle crosses a
    yield surface between the two evaluations."""
    rng = np.random.default_rng(12)
    plastic = any(m["plastic"] for m in mats)
    mat_id = rng.integers(0, len(mats), 150) if len(mats) > 1 else None
    state0, p = _small_elastic_scene(rng, mats=mats, mat_id=mat_id)
    steps = 6
    if plastic:  # larger strains, so the return maps act
        state0 = state0[:3] + (torch.tensor(np.eye(3) + rng.normal(0, 0.06, (150, 3, 3))),)
    xt = state0[0] + 0.01 * torch.tensor(rng.normal(0, 1, state0[0].shape))
    # forward agrees with the SVD-based oracle
    ref = O.step_n(state0, p, steps)
    fwd = O.forward_differentiable(state0, p, steps)
    for a, b in zip(ref, fwd):
        assert torch.allclose(a, b, rtol=1e-9, atol=1e-12)
    N = state0[0].shape[0]
    gx = 2.0 * (ref[0] - xt) / (3 * N)
    res = O.adjoint(state0, p, steps, (gx, None, None, None), want_state0=True)

    def loss(logE, nu, x0=None):
        q = O.Params(p.mass, p.vol0, logE, nu, p.mat_id, p.materials, p.n, p.dt, p.gravity, p.bound)
        s0 = state0 if x0 is None else (x0,) + tuple(state0[1:])
        return O.position_mse(O.step_n(s0, q, steps)[0], xt).item()

    d = torch.tensor(rng.choice([-1.0, 1.0], N))
    for name, g in (("logE", res["g_logE"]), ("nu", res["g_nu"])):
        h = (1e-3 if name == "logE" else 1e-4) * (1e-1 if plastic else 1.0)
        base_l, base_n = p.log_E, p.nu
        if name == "logE":
            fd = (loss(base_l + h * d, base_n) - loss(base_l - h * d, base_n)) / (2 * h)
        else:
            fd = (loss(base_l, base_n + h * d) - loss(base_l, base_n - h * d)) / (2 * h)
        an = float((g * d).sum())
        assert abs(fd - an) <= 1e-4 * abs(an) + 1e-14, (name, fd, an)
    h = 1e-6
    dx = torch.tensor(rng.normal(0, 1, state0[0].shape))
    fd = (loss(p.log_E, p.nu, state0[0] + h * dx) - loss(p.log_E, p.nu, state0[0] - h * dx)) / (2 * h)
    an = float((res["g_x0"] * dx).sum())
    assert abs(fd - an) <= 1e-4 * abs(an) + 1e-12, (fd, an)


# --------------------------------------------------------------------------
# BGDO (Alg. 1, Sec. 4.2, App. B.3-B.4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("elastic", [0, 1, 2, 3, 4, 5])
def test_bgdo_stress_gradient_is_stress_norm(elastic):
    """Every model's tau is linear in (mu, lam), both proportional to E, so
    d|tau|/d log E = |tau|: the autograd derivative must reproduce it."""
    rng = np.random.default_rng(20 + elastic)
    N = 64
    F = np.eye(3) + rng.normal(0, 0.15, (N, 3, 3))
    F[np.linalg.det(F) < 0.2] = np.eye(3) * 1.05
    mats = [dict(elastic=elastic, plastic=0, yield_stress=0.0, friction_deg=0.0)]
    p = _params(N, 16, 1e-4, mats=mats, rng=rng)
    p.log_E = torch.tensor(np.log(rng.uniform(1e3, 1e6, N)))
    x = torch.tensor(rng.uniform(0.4, 0.6, (N, 3)))
    state = (x, torch.zeros(N, 3, dtype=F64), torch.zeros(N, 3, 3, dtype=F64), torch.tensor(F))
    g, delta, term = O.bgdo_key_frame(state, p)
    mu, lam = O.lame(p.log_E, p.nu)
    s = torch.linalg.matrix_norm(O.kirchhoff_stress(torch.tensor(F), mu, lam, p.mat_id, mats))
    assert torch.allclose(g, s, rtol=1e-10, atol=1e-9)
    eta = torch.clamp(0.1 * torch.log(1.0 + torch.exp(p.log_E)), max=1.0)
    assert torch.allclose(term, eta * torch.log(1.0 + s) - (1 - eta) * (delta - 0.1), rtol=1e-12, atol=1e-12)


def test_bgdo_rest_state_closed_form():
    """At rest (F = I, v = C = 0, no gravity) tau = 0 and F' = I, so each key
    frame contributes 0.1 (1 - eta); E = 1e3 gives eta = 0.1 ln(1001)."""
    rng = np.random.default_rng(30)
    N = 200
    p = _params(N, 16, 1e-4, E=1e3, rng=rng)
    state0 = (torch.tensor(rng.uniform(0.4, 0.6, (N, 3))), torch.zeros(N, 3, dtype=F64),
              torch.zeros(N, 3, 3, dtype=F64), torch.eye(3, dtype=F64).expand(N, 3, 3).clone())
    out = O.bgdo(state0, p, frames=3, substeps_per_frame=2, key_frames=[0, 1, 2])
    eta = 0.1 * math.log(1001.0)
    assert torch.allclose(out, torch.full((N,), math.log(1e3) - 0.1 * (1 - eta), dtype=F64), atol=1e-12)


def test_bgdo_deformation_of_an_affine_field():
    """v = a + B x, C = B, F = I: tau = 0 in the first substep and APIC moves
    the affine field exactly, so F' = I + dt B and delta = dt |B|_F."""
    rng = np.random.default_rng(31)
    N, n, dt = 300, 16, 1e-4
    x = torch.tensor(rng.uniform(0.3, 0.7, (N, 3)))
    a = torch.tensor(rng.normal(0, 1, 3))
    B = torch.tensor(rng.normal(0, 2, (3, 3)))
    state = (x, a + x @ B.T, B.expand(N, 3, 3).clone(), torch.eye(3, dtype=F64).expand(N, 3, 3).clone())
    p = _params(N, n, dt, rng=rng)
    g, delta, _ = O.bgdo_key_frame(state, p)
    assert torch.allclose(g, torch.zeros(N, dtype=F64), atol=1e-9)
    assert torch.allclose(delta, torch.full((N,), dt * float(torch.linalg.norm(B)), dtype=F64), rtol=1e-9)


def test_bgdo_key_frames_are_stored_before_their_substeps():
    """Key frame k holds the state after k frames (k S substeps), and the
    update is the mean of the key-frame terms."""
    rng = np.random.default_rng(32)
    N, S = 150, 3
    state0, p = _small_elastic_scene(rng, N=N)
    out = O.bgdo(state0, p, frames=4, substeps_per_frame=S, key_frames=[0, 2, 3])
    terms = [O.bgdo_key_frame(O.step_n(state0, p, k * S), p)[2] for k in (0, 2, 3)]
    assert torch.allclose(out, p.log_E - sum(terms) / 3, rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# MCIS interior filling (Sec. 4.1)
# --------------------------------------------------------------------------

def test_mcis_distance_matches_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(40)
    surf = rng.uniform(0.2, 0.8, (3000, 3))
    cand = rng.uniform(0.1, 0.9, (5000, 3))
    d = O.mcis_distance(torch.tensor(cand), torch.tensor(surf)).numpy()
    ref, _ = cKDTree(surf).query(cand, k=1)
    np.testing.assert_allclose(d, ref, rtol=1e-12, atol=1e-15)


def test_mcis_weight_closed_forms():
    s = O.MCIS_SIGMA
    d = torch.tensor([0.0, s, 2 * s, 1.0], dtype=F64)
    w = O.mcis_weight(d)
    expect = torch.tensor([1.0, math.exp(-0.5), math.exp(-2.0), 1e-6], dtype=F64)
    assert torch.allclose(w, expect, rtol=1e-15, atol=0)


def _mcis_toy(rng, dists):
    """Candidates on the x axis at the given distances from one surface point."""
    surf = torch.tensor([[0.5, 0.5, 0.5]], dtype=F64)
    cand = torch.tensor([[0.5 + d, 0.5, 0.5] for d in dists], dtype=F64)
    w = O.mcis_weight(torch.tensor(dists, dtype=F64))
    return surf, cand, (w / w.sum()).numpy()


def test_mcis_single_draw_follows_p():
    """n = 1: the exponential-key race picks candidate j with probability p_j."""
    rng = np.random.default_rng(41)
    surf, cand, p = _mcis_toy(rng, [0.0, 0.01, 0.02, 0.03, 0.2])
    T = 20000
    counts = np.zeros(len(p))
    for _ in range(T):
        idx, _ = O.mcis_select_instance(cand, surf, torch.tensor(rng.uniform(0, 1, len(p))), 1)
        counts[int(idx[0])] += 1
    sd = np.sqrt(T * p * (1 - p))
    assert np.all(np.abs(counts - T * p) <= 4.5 * sd + 1), (counts, T * p)


def test_mcis_two_draws_without_replacement_inclusion():
    """n = 2 of 3: successive sampling without replacement includes j with
    probability p_j + sum_{i != j} p_i p_j / (1 - p_i)."""
    rng = np.random.default_rng(42)
    surf, cand, p = _mcis_toy(rng, [0.0, 0.015, 0.03])
    incl = np.array([p[j] + sum(p[i] * p[j] / (1 - p[i]) for i in range(3) if i != j) for j in range(3)])
    T = 20000
    counts = np.zeros(3)
    for _ in range(T):
        idx, _ = O.mcis_select_instance(cand, surf, torch.tensor(rng.uniform(0, 1, 3)), 2)
        assert len(set(idx.tolist())) == 2
        counts[idx.numpy()] += 1
    sd = np.sqrt(T * incl * (1 - incl))
    assert np.all(np.abs(counts - T * incl) <= 4.5 * sd + 1), (counts, T * incl)


def test_mcis_instances_union_and_limits():
    rng = np.random.default_rng(43)
    surf = torch.tensor(rng.uniform(0.3, 0.7, (400, 3)))
    cand = torch.tensor(rng.uniform(0.3, 0.7, (900, 3)))
    u = torch.tensor(rng.uniform(0, 1, 900))
    surf_off, cand_off = [0, 150, 150, 400], [0, 300, 300, 900]
    sel, d = O.mcis(cand, cand_off, surf, surf_off, u, [300, 0, 17])
    assert sel[:300].tolist() == list(range(300))          # n_k = all candidates
    assert len(sel) == 317 and len(set(sel.tolist())) == 317
    assert all(300 <= j < 900 for j in sel[300:].tolist())
    # the instance's own surface sets the distance
    assert torch.allclose(d[300:], O.mcis_distance(cand[300:], surf[150:]))


# --------------------------------------------------------------------------
# Gaussian covariance at a frame boundary (Sec. 3.2): Sigma = F Sigma0 F^T,
# stored as (xx, xy, xz, yy, yz, zz)
# --------------------------------------------------------------------------

def _sym6(S):
    return np.stack([S[:, 0, 0], S[:, 0, 1], S[:, 0, 2], S[:, 1, 1], S[:, 1, 2], S[:, 2, 2]], -1)


def _full(c):
    return np.stack([np.stack([c[:, 0], c[:, 1], c[:, 2]], -1), np.stack([c[:, 1], c[:, 3], c[:, 4]], -1),
                     np.stack([c[:, 2], c[:, 4], c[:, 5]], -1)], 1)


def test_covariance_closed_forms():
    rng = np.random.default_rng(31)
    N = 64
    q = rng.normal(0, 1, (N, 3, 3))
    S0 = q @ q.transpose(0, 2, 1) + 0.1 * np.eye(3)
    c0 = _sym6(S0)
    # identity: unchanged
    out = O.covariance(torch.eye(3, dtype=F64).expand(N, 3, 3), c0).numpy()
    assert np.allclose(out, c0, rtol=0, atol=1e-15)
    # diagonal stretch s: every entry (i, j) scales by s_i s_j (catches a
    # swapped component or a transposed product)
    s = rng.uniform(0.5, 2.0, (N, 3))
    out = _full(O.covariance(torch.tensor(np.einsum("ni,ij->nij", s, np.eye(3))), c0).numpy())
    assert np.allclose(out, S0 * s[:, :, None] * s[:, None, :], rtol=1e-14, atol=0)
    # rotation: the spectrum is kept, and the axes turn with F
    for k in range(8):
        Q = rot(rng).numpy()
        d = np.sort(rng.uniform(0.1, 3.0, 3))
        out = _full(O.covariance(torch.tensor(Q[None]), _sym6(np.diag(d)[None])).numpy())[0]
        assert np.allclose(np.linalg.eigvalsh(out), d, rtol=1e-13)
        assert np.allclose(out @ Q[:, 0], d[0] * Q[:, 0], atol=1e-12)


def test_covariance_pushes_the_level_set_forward():
    """Points on the unit level set x^T Sigma0^-1 x = 1, mapped by F, lie on
    y^T Sigma^-1 y = 1; det Sigma = det(F)^2 det Sigma0."""
    rng = np.random.default_rng(32)
    for k in range(10):
        q = rng.normal(0, 1, (3, 3))
        S0 = q @ q.T + 0.2 * np.eye(3)
        F = np.eye(3) + rng.normal(0, 0.3, (3, 3))
        S = _full(O.covariance(torch.tensor(F[None]), _sym6(S0[None])).numpy())[0]
        L = np.linalg.cholesky(S0)
        u = rng.normal(0, 1, (3, 200))
        x = L @ (u / np.linalg.norm(u, axis=0))  # x^T S0^-1 x = 1
        y = F @ x
        lvl = np.einsum("ip,ij,jp->p", y, np.linalg.inv(S), y)
        assert np.allclose(lvl, 1.0, rtol=1e-11)
        assert math.isclose(np.linalg.det(S), np.linalg.det(F) ** 2 * np.linalg.det(S0), rel_tol=1e-11)


def test_covariance_of_mapped_samples():
    """The covariance of F z for z ~ N(0, Sigma0) (200,000 samples) is
    Sigma to sampling accuracy."""
    rng = np.random.default_rng(33)
    q = rng.normal(0, 1, (3, 3))
    S0 = q @ q.T + 0.3 * np.eye(3)
    F = np.eye(3) + rng.normal(0, 0.4, (3, 3))
    z = rng.multivariate_normal(np.zeros(3), S0, 200_000)
    emp = np.cov((z @ F.T).T)
    S = _full(O.covariance(torch.tensor(F[None]), _sym6(S0[None])).numpy())[0]
    assert np.abs(emp - S).max() <= 0.02 * np.abs(S).max()
