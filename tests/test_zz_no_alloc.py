"""The allocation-free MCIS entry point (mpm_mcis_select_static) against
mpm_mcis_select with a caller workspace, through the C ABI: two calls in a
row on the library's fixed scratch, the second with a smaller input (the
scratch keeps the first call's contents), must give the same selected
indices and the same distances bit for bit (integer work; the distances are
float64 minima of the same float64 sums).  Inputs beyond the fixed scratch
are refused with MPM_ENOMEM before any device work."""
import numpy as np
import pytest
import torch

from paper_2602_01723_amd import binding as B
from paper_2602_01723_amd import scenes

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, np.float32).T)).cuda()


def _both(d):
    surf, cand, u = _dev(d["surface"]), _dev(d["candidates"]), torch.as_tensor(d["u"]).cuda()
    ref_idx, ref_d = B.mpm_mcis_select(surf, d["surface_offsets"], cand, d["candidate_offsets"], u, d["n_select"],
                                       want_distance=True)
    total = int(d["n_select"].sum())
    out = torch.full((max(total, 1),), -1, dtype=torch.int64, device="cuda")
    dist = torch.full((len(d["u"]),), -1.0, dtype=torch.float64, device="cuda")
    B.mpm_mcis_select_static(surf, d["surface_offsets"], cand, d["candidate_offsets"], u, d["n_select"], out, d=dist)
    torch.cuda.synchronize()
    return ref_idx.cpu().numpy(), ref_d.cpu().numpy(), out[:total].cpu().numpy(), dist.cpu().numpy()


def test_static_mcis_matches_workspace_mcis_twice():
    big = scenes.mcis_inputs(seed=21, n_shell=(3000, 2500, 4000, 1200), cand_per_shell=3.0)
    small = scenes.mcis_inputs(seed=22, n_shell=(900, 700), cand_per_shell=2.0, empty_instances=(1,))
    for name, d in (("first, larger", big), ("second, smaller", small)):
        ri, rd, si, sd = _both(d)
        print(name, "candidates", len(rd), "selected", len(ri), flush=True)
        assert len(si) == len(ri) and np.array_equal(si, ri), name
        assert np.array_equal(sd, rd), name  # inf (no surface point within reach) included


def test_static_mcis_refuses_inputs_beyond_its_scratch():
    K = 2
    M = 4_000_000  # 28 B per candidate alone exceeds the 64 MiB scratch
    so = np.array([0, 10, 20], np.int64)
    co = np.array([0, M // 2, M], np.int64)
    ns = np.array([5, 5], np.int64)
    # full-size, valid buffers, although the size check refuses the call first
    surf = torch.full((3, 20), 0.5, device="cuda")
    cand = torch.full((3, M), 0.5, device="cuda")
    u = torch.ones(M, dtype=torch.float64, device="cuda")
    out = torch.empty(10, dtype=torch.int64, device="cuda")
    with pytest.raises(B.MPMError) as e:
        B.mpm_mcis_select_static(surf, so, cand, co, u, ns, out)
    assert e.value.status == B.MPM_ENOMEM
    assert K == len(ns) == len(so) - 1
