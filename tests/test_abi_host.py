"""Host-side checks of the C ABI: the library loads, exports every symbol
declared in include/fastmpm.h, and rejects invalid input on the host
(MPM_EINVAL) before touching a device.  No compute runs here."""
import ctypes
import os
import re

import pytest

from paper_2602_01723_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2602_01723_amd import build
        build.build()
    return B.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fastmpm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(mpm_\w+)\(", src, re.M)))


def test_header_and_binding_agree():
    assert sorted(B.EXPORTED) == declared_functions()


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    assert lib.mpm_status_string(0) == b"ok"
    assert lib.mpm_status_string(B.MPM_EINVAL) == b"invalid argument"
    assert lib.mpm_status_string(-99) == b"unknown status"


def _cfg(**kw):
    base = dict(abi_version=1, grid_res=32, bound=3, n_batch=1, dt=1e-4, sort_every=0, flags=0)
    base.update(kw)
    g = (ctypes.c_float * 3)(0.0, -9.8, 0.0)
    return B.mpm_config(base["abi_version"], base["grid_res"], base["bound"], base["n_batch"], base["dt"], g,
                        base["sort_every"], base["flags"])


def _init(lib, cfg, mats=None, n=10, offsets=None):
    mats = mats or [B.mpm_material(0, 0, 0.0, 0.0)]
    arr = (B.mpm_material * len(mats))(*mats)
    h = ctypes.c_void_p()
    offs = None if offsets is None else (ctypes.c_int64 * len(offsets))(*offsets)
    rc = lib.mpm_init(ctypes.byref(cfg), arr, len(mats), n, offs, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("kw", [dict(abi_version=2), dict(grid_res=4), dict(grid_res=4096), dict(bound=-1),
                                dict(bound=15), dict(n_batch=0), dict(dt=0.0), dict(dt=float("nan")),
                                dict(flags=1), dict(sort_every=-1)])
def test_invalid_config_rejected_on_host(lib, kw):
    rc, h = _init(lib, _cfg(**kw))
    assert rc == B.MPM_EINVAL and not h.value


def test_invalid_materials_and_offsets(lib):
    assert _init(lib, _cfg(), mats=[B.mpm_material(6, 0, 0.0, 0.0)])[0] == B.MPM_EINVAL   # elastic code
    assert _init(lib, _cfg(), mats=[B.mpm_material(-1, 0, 0.0, 0.0)])[0] == B.MPM_EINVAL
    assert _init(lib, _cfg(), mats=[B.mpm_material(1, 1, 0.0, 0.0)])[0] == B.MPM_EINVAL   # yield 0
    assert _init(lib, _cfg(), mats=[B.mpm_material(1, 2, 0.0, 95.0)])[0] == B.MPM_EINVAL  # friction
    assert _init(lib, _cfg(), mats=[B.mpm_material(1, 5, 0.0, 0.0)])[0] == B.MPM_EINVAL   # plastic code
    assert _init(lib, _cfg(), n=-1)[0] == B.MPM_EINVAL
    assert _init(lib, _cfg(n_batch=2), n=10, offsets=None)[0] == B.MPM_EINVAL
    assert _init(lib, _cfg(n_batch=2), n=10, offsets=[0, 6, 5])[0] == B.MPM_EINVAL
    assert _init(lib, _cfg(n_batch=2), n=10, offsets=[0, 7, 3])[0] == B.MPM_EINVAL
    assert _init(lib, _cfg(n_batch=2), n=10, offsets=[1, 5, 10])[0] == B.MPM_EINVAL


def test_null_arguments(lib):
    assert lib.mpm_init(None, None, 0, 0, None, None) == B.MPM_EINVAL
    assert lib.mpm_step_n(None, None, 1, None, 0, None) == B.MPM_EINVAL
    assert lib.mpm_load(None, None, None) == B.MPM_EINVAL
    assert lib.mpm_advance(None, 1, None) == B.MPM_EINVAL
    assert lib.mpm_store(None, None, None) == B.MPM_EINVAL
    assert lib.mpm_export_frame(None, None, None, None, None) == B.MPM_EINVAL
    assert lib.mpm_destroy(None) == B.MPM_EINVAL
    assert lib.mpm_get_diagnostics(None, None) == B.MPM_EINVAL
    assert lib.mpm_last_error(None) == b"NULL context"
