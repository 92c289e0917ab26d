"""The adjoint through torch.autograd (paper_2602_01723_amd.autograd) against
the FP64 oracle's autograd adjoint and against direct C-ABI calls."""
import numpy as np
import pytest
import torch

from oracle import mpm_oracle as O
from paper_2602_01723_amd import autograd as AG
from paper_2602_01723_amd import binding as B
from tests.parity import rel_err
from tests.test_gpu_adjoint import ALL_ELASTIC, elastic_case

pytestmark = pytest.mark.gpu


def _setup(d, mats, steps, K):
    N = len(d["mass"])
    ctx = B.mpm_init(d["n"], d["dt"], mats, N)
    dev = lambda a, c: torch.tensor(np.ascontiguousarray(np.asarray(a, np.float32).reshape(N, c).T)).cuda()
    sim = AG.Simulation(ctx, torch.tensor(d["mass"]).cuda(), torch.tensor(d["vol0"]).cuda(),
                        torch.tensor(d["mat_id"]).cuda(), steps, K)
    state = [dev(d["x"], 3), dev(d["v"], 3), dev(d["C"], 9), dev(d["F"], 9)]
    return N, ctx, sim, state


def test_autograd_matches_oracle_adjoint():
    steps, K = 8, 3
    d = elastic_case(21, N=1200, n_mat=len(ALL_ELASTIC))
    N, ctx, sim, state = _setup(d, ALL_ELASTIC, steps, K)
    log_E = torch.tensor(d["log_E"]).cuda().requires_grad_(True)
    nu = torch.tensor(d["nu"]).cuda().requires_grad_(True)
    x0 = state[0].clone().requires_grad_(True)
    rng = np.random.default_rng(22)
    xt = torch.tensor(np.ascontiguousarray((d["x"] + rng.normal(0, 0.01, d["x"].shape)).T.astype(np.float32))).cuda()
    x, v, C, F = AG.simulate(sim, log_E, nu, x0, state[1], state[2], state[3])
    loss = ((x - xt) ** 2).mean() + 0.1 * (v ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    # the same cotangents through the oracle
    gx = (2.0 * (x - xt) / (3 * N)).detach().cpu().numpy().T
    gv = (0.2 * v / (3 * N)).detach().cpu().numpy().T
    params = O.Params(d["mass"], d["vol0"], d["log_E"], d["nu"], d["mat_id"], ALL_ELASTIC, d["n"], d["dt"])
    s0 = tuple(torch.as_tensor(np.asarray(a, np.float64)) for a in (d["x"], d["v"], d["C"], d["F"]))
    ref = O.adjoint(s0, params, steps, (gx, gv, None, None), want_state0=True)
    errs = dict(g_log_E=rel_err(log_E.grad.cpu().numpy(), ref["g_logE"].numpy(), 0.0),
                g_nu=rel_err(nu.grad.cpu().numpy(), ref["g_nu"].numpy(), 0.0),
                g_x0=rel_err(x0.grad.cpu().numpy().T, ref["g_x0"].numpy(), 0.0))
    print(errs, flush=True)
    assert max(errs.values()) <= 2e-3, errs


def test_autograd_chain_to_E_and_direct_call():
    steps, K = 6, 6
    d = elastic_case(23, N=800)
    mats = ALL_ELASTIC[:1]
    N, ctx, sim, state = _setup(d, mats, steps, K)
    E = torch.exp(torch.tensor(d["log_E"], dtype=torch.float32)).cuda().requires_grad_(True)
    nu = torch.tensor(d["nu"]).cuda()
    x, v, C, F = AG.simulate(sim, torch.log(E), nu, *state)
    w = torch.tensor(np.random.default_rng(24).normal(0, 1, (3, N)).astype(np.float32)).cuda()
    (x * w).sum().backward()
    # direct C-ABI reverse with the same cotangent
    p = B.Particles(x=state[0].clone(), v=state[1].clone(), C=state[2].clone(), F=state[3].clone(),
                    mass=sim.mass, vol0=sim.vol0, log_E=torch.tensor(d["log_E"]).cuda(), nu=nu, mat_id=sim.mat_id)
    tape = torch.empty(B.mpm_tape_size(ctx, steps, K) // 4 + 64, device="cuda")
    B.mpm_step_n(ctx, p, steps, tape=tape, checkpoint_every=K)
    gl = torch.empty(N, device="cuda")
    gn = torch.empty(N, device="cuda")
    B.mpm_backward(ctx, p, tape, steps, g_x=w, g_log_E=gl, g_nu=gn)
    torch.cuda.synchronize()
    assert torch.allclose(p.x, x.detach())
    assert rel_err((E.grad * E).detach().cpu().numpy(), gl.cpu().numpy(), 0.0) <= 1e-5


def test_autograd_one_tape_per_context():
    d = elastic_case(25, N=200)
    N, ctx, sim, state = _setup(d, ALL_ELASTIC[:1], 4, 2)
    log_E = torch.tensor(d["log_E"]).cuda().requires_grad_(True)
    nu = torch.tensor(d["nu"]).cuda()
    out1 = AG.simulate(sim, log_E, nu, *state)
    out2 = AG.simulate(sim, log_E, nu, *state)  # overwrites the context's tape
    out2[0].sum().backward()                  # the latest forward: fine
    with pytest.raises(B.MPMError) as e:
        out1[0].sum().backward()
    assert e.value.status == B.MPM_ESTATE
