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


def _init(lib, cfg, mats=None, n=10, offsets=None, workspace=None, nbytes=0):
    mats = mats or [B.mpm_material(0, 0, 0.0, 0.0)]
    arr = (B.mpm_material * len(mats))(*mats)
    h = ctypes.c_void_p()
    offs = None if offsets is None else (ctypes.c_int64 * len(offsets))(*offsets)
    rc = lib.mpm_init(ctypes.byref(cfg), arr, len(mats), n, offs, workspace, nbytes, ctypes.byref(h))
    return rc, h


def _ws_size(lib, cfg, n):
    out = ctypes.c_size_t()
    rc = lib.mpm_workspace_size(ctypes.byref(cfg), n, ctypes.byref(out))
    return rc, out.value


def test_workspace_size(lib):
    """The workspace grows with the particle count and the grid; invalid
    configurations are refused on the host."""
    rc, small = _ws_size(lib, _cfg(), 1000)
    assert rc == B.MPM_OK and small > 0 and small % 256 == 0
    rc, big = _ws_size(lib, _cfg(), 100_000)
    assert rc == B.MPM_OK and big > small + 100_000 * 300  # >= 332 B per particle of buffers
    rc, grid = _ws_size(lib, _cfg(grid_res=64), 1000)
    assert rc == B.MPM_OK and grid > small + 3 * 16 * (64 ** 3 - 32 ** 3)  # three float4 grids
    assert _ws_size(lib, _cfg(grid_res=4), 10)[0] == B.MPM_EINVAL
    assert _ws_size(lib, _cfg(), -1)[0] == B.MPM_EINVAL
    assert lib.mpm_workspace_size(ctypes.byref(_cfg()), 10, None) == B.MPM_EINVAL


def test_workspace_checks_before_any_device_work(lib):
    """NULL or misaligned workspaces are invalid; one byte short is MPM_ENOMEM.
    The addresses below are never dereferenced: the checks run on the host."""
    cfg = _cfg()
    _, need = _ws_size(lib, cfg, 10)
    assert _init(lib, cfg, workspace=None, nbytes=need)[0] == B.MPM_EINVAL
    assert _init(lib, cfg, workspace=0x100001, nbytes=need)[0] == B.MPM_EINVAL
    rc, h = _init(lib, cfg, workspace=0x100000, nbytes=need - 1)
    assert rc == B.MPM_ENOMEM and not h.value


@pytest.mark.parametrize("kw", [dict(abi_version=2), dict(grid_res=4), dict(grid_res=4096), dict(bound=-1),
                                dict(bound=15), dict(n_batch=0), dict(dt=0.0), dict(dt=float("nan")),
                                dict(flags=8), dict(flags=2 | 4), dict(flags=2 | 1), dict(sort_every=-1)])
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
    assert lib.mpm_init(None, None, 0, 0, None, None, 0, None) == B.MPM_EINVAL
    assert lib.mpm_step_n(None, None, 1, None, 0, None) == B.MPM_EINVAL
    assert lib.mpm_load(None, None, None) == B.MPM_EINVAL
    assert lib.mpm_advance(None, 1, None) == B.MPM_EINVAL
    assert lib.mpm_store(None, None, None) == B.MPM_EINVAL
    assert lib.mpm_export_frame(None, None, None, None, None) == B.MPM_EINVAL
    assert lib.mpm_destroy(None) == B.MPM_EINVAL
    assert lib.mpm_get_diagnostics(None, None) == B.MPM_EINVAL
    assert lib.mpm_last_error(None) == b"NULL context"


def test_ipf_workspace_size_and_host_checks(lib):
    """Candidate generation: sizes and offsets are checked on the host;
    no raw candidates or no triangles return at once with zero offsets."""
    out = ctypes.c_size_t()
    assert lib.mpm_ipf_workspace_size(2, 100, 200, 1000, ctypes.byref(out)) == B.MPM_OK and out.value > 0
    small = out.value
    assert lib.mpm_ipf_workspace_size(2, 100, 2000, 100000, ctypes.byref(out)) == B.MPM_OK
    assert out.value > small + 100000 * 4 + 1800 * (48 + 24 * 4)
    for args in ((0, 1, 1, 1), (2, -1, 1, 1), (2, 1, 1 << 28, 1), (2, 1, 1, 1 << 30)):
        assert lib.mpm_ipf_workspace_size(*args, ctypes.byref(out)) == B.MPM_EINVAL
    assert lib.mpm_ipf_workspace_size(1, 1, 1, 1, None) == B.MPM_EINVAL
    I64 = lambda *v: (ctypes.c_int64 * len(v))(*v)
    co = (ctypes.c_int64 * 3)(7, 7, 7)
    # no raw candidates: OK, offsets zero, nothing touched
    assert lib.mpm_ipf_candidates(2, None, I64(0, 3, 6), None, I64(0, 1, 2), None, I64(0, 0, 0), 0.6, None, 0,
                                  None, None, co, None) == B.MPM_OK
    assert list(co) == [0, 0, 0]
    # no triangles
    co = (ctypes.c_int64 * 3)(7, 7, 7)
    assert lib.mpm_ipf_candidates(2, None, I64(0, 3, 6), None, I64(0, 0, 0), None, I64(0, 5, 9), 0.6, None, 0,
                                  None, None, co, None) == B.MPM_OK
    assert list(co) == [0, 0, 0]
    # bad offsets, threshold, missing buffers
    bad = [(I64(1, 3, 6), I64(0, 1, 2), I64(0, 5, 9), 0.6), (I64(0, 3, 2), I64(0, 1, 2), I64(0, 5, 9), 0.6),
           (I64(0, 3, 6), I64(0, 2, 1), I64(0, 5, 9), 0.6), (I64(0, 3, 6), I64(0, 1, 2), I64(0, 5, 9), 1.5),
           (I64(0, 3, 6), I64(0, 1, 2), I64(0, 5, 9), float("nan")), (I64(0, 3, 6), I64(0, 1, 2), I64(0, 5, 9), 0.6)]
    for hv, ht, ro, thr in bad:
        assert lib.mpm_ipf_candidates(2, None, hv, None, ht, None, ro, thr, None, 0, None, None, co, None) == \
            B.MPM_EINVAL
    assert lib.mpm_ipf_candidates(2, None, I64(0, 3, 6), None, I64(0, 1, 2), None, I64(0, 5, 9), 0.6, None, 0,
                                  None, None, None, None) == B.MPM_EINVAL
