"""Build libfastmpm.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfastmpm.so")
PROBES = os.path.join(PKG, "libmpm_probes.so")

ARCH = os.environ.get("FASTMPM_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-munsafe-fp-atomics",            # hardware FP32 atomics (no CAS loops)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, out: str, verbose: bool, extra=()) -> str:
    tmp = out + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra) + ["-I", INCLUDE, "-I", CSRC, src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, extra=()) -> str:
    """Compile every HIP source: the library (libfastmpm.so, whose path is
    returned) and the measurement probes bench.py uses (libmpm_probes.so)."""
    _compile(os.path.join(CSRC, "probes.hip"), PROBES, verbose)
    return _compile(os.path.join(CSRC, "fastmpm.hip"), LIB, verbose, extra)


if __name__ == "__main__":
    print(build(verbose=True))
