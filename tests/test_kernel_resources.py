"""Register and scratch budget of the hot kernels (CPU: compiler remarks).

The fused substep kernel and the adjoint P2G sit at the 256-VGPR limit of
two waves per SIMD, the default-mode adjoint G2P at the 168-VGPR limit of
three.  A change that makes the compiler spill into AGPRs lowers occupancy
without any error, and one that spills to scratch adds memory traffic; both
were seen to cost 40-50% of the kernel's speed.  This test compiles the
device code with the library's flags and checks, from the compiler's
resource-usage remarks, that each hot kernel keeps the waves per SIMD listed
in OCCUPANCY (two unless listed), uses no AGPRs and at most the scratch
listed in SCRATCH_OK (the adjoint kernels are allowed 16 bytes per lane:
some builds keep a few registers there).  The caller-order permutation passes, which hold a plane's loads in
registers across their LDS round trip, are checked the same way."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2602_01723_amd import build as Bd

HOT = ("k_substepILi1E", "k_substepILi0E", "k_substepILi2E", "k_adj_g2pILb0", "k_adj_g2pILb1", "k_adj_p2g",
       "k_perm_pass1_staged", "k_perm_pass2")
SCRATCH_OK = {"k_adj_p2g": 16, "k_adj_g2pILb0": 16}  # bytes per lane
OCCUPANCY = {"k_adj_g2pILb0": 3}  # waves per SIMD


def _remarks():
    hipcc = None
    try:
        hipcc = Bd.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    flags = [f for f in Bd.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    with tempfile.TemporaryDirectory() as td:
        out = os.path.join(td, "k.co")
        cmd = [hipcc] + flags + ["-I", Bd.INCLUDE, "-I", Bd.CSRC, "--offload-device-only",
                                 "--no-gpu-bundle-output", "-Rpass-analysis=kernel-resource-usage",
                                 os.path.join(Bd.CSRC, "fastmpm.hip"), "-o", out]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-2000:]
        return res.stderr


def test_hot_kernels_keep_their_waves_and_no_scratch():
    text = _remarks()
    usage, name = {}, None
    for line in text.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            usage[name] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+)", line)
        if m and name:
            usage[name][m.group(1).strip()] = int(m.group(2))
    for key in HOT:
        names = [n for n in usage if key in n]
        assert names, f"{key} not found in the compiler remarks"
        for n in names:
            u = usage[n]
            assert u.get("Occupancy", 0) >= OCCUPANCY.get(key, 2), (n, u)
            assert u.get("ScratchSize", 0) <= SCRATCH_OK.get(key, 0), (n, u)
            assert u.get("AGPRs", 0) == 0, (n, u)
