"""Binding of libmpm_probes.so: atomic-throughput probes for bench.py.

The probes time, on the current device, the two atomic operations the
substep kernel is built on (LDS 64-bit integer adds of the P2G tile, global
FP32 adds of the tile flush), so the benchmark can set the kernel's achieved
atomic rates against what the chip delivers in the same run.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
PROBES_PATH = os.path.join(_PKG, "libmpm_probes.so")
_lib = None


def load(path: str = PROBES_PATH):
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2602_01723_amd.build`")
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
        lib = ctypes.CDLL(path)
        fp, dp = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
        for word in ("u64", "u32", "f32"):
            fn = getattr(lib, f"probe_lds_add_{word}")
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, fp, dp]
        lib.probe_global_add_f32.restype = ctypes.c_int
        lib.probe_global_add_f32.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_int64, fp, dp]
        _lib = lib
    return _lib


def lds_add(pattern: int, word: str = "u64", reps: int = 200) -> dict:
    """Rate of LDS atomic adds (lane operations per second) of one word type
    ("u64": ds_add_u64, "u32": ds_add_u32, "f32": ds_add_f32): pattern 0
    lane-consecutive words, 1 the P2G scatter's node order."""
    import torch
    sink = torch.empty(4096, dtype=torch.int64, device="cuda")
    ms, ops = ctypes.c_float(), ctypes.c_double()
    fn = getattr(load(), f"probe_lds_add_{word}")
    rc = fn(int(pattern), int(reps), sink.data_ptr(), ctypes.byref(ms), ctypes.byref(ops))
    if rc:
        raise RuntimeError(f"probe_lds_add_{word} failed ({rc})")
    return dict(lane_ops_per_s=ops.value / (ms.value * 1e-3), ms=ms.value, lane_ops=ops.value)


def lds_add_u64(pattern: int, reps: int = 200) -> dict:
    return lds_add(pattern, "u64", reps)


def global_add_f32(pattern: int, reps: int = 8, mib: int = 256) -> dict:
    """Rate of global FP32 atomic adds (lane operations per second) over a
    `mib` MiB array: pattern 0 lane-distinct, 1 the 4 channels of a node."""
    import torch
    floats = mib * (1 << 20) // 4
    grid = torch.zeros(floats, dtype=torch.float32, device="cuda")
    props = torch.cuda.get_device_properties(0)
    blocks = 16 * props.multi_processor_count
    ms, ops = ctypes.c_float(), ctypes.c_double()
    rc = load().probe_global_add_f32(int(pattern), int(reps), int(blocks), grid.data_ptr(), floats,
                                     ctypes.byref(ms), ctypes.byref(ops))
    if rc:
        raise RuntimeError(f"probe_global_add_f32 failed ({rc})")
    return dict(lane_ops_per_s=ops.value / (ms.value * 1e-3), ms=ms.value, lane_ops=ops.value)
