"""Python binding of libfastmpm.so (ctypes; argument marshalling only).

The functions keep the C names (``mpm_init``, ``mpm_substep``,
``mpm_step_n``, ``mpm_backward``, ...).  Device memory comes from PyTorch
CUDA (HIP) tensors and work is enqueued on the current torch stream.  Every
step of the simulation runs in the HIP library; if the library is missing
the binding raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfastmpm.so")

MPM_ABI_VERSION = 1
MPM_OK, MPM_EINVAL, MPM_ENOMEM, MPM_EDEVICE, MPM_ESTATE, MPM_EUNSTABLE, MPM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MPM_FLAG_DETERMINISTIC, MPM_FLAG_GRID_SPARSE, MPM_FLAG_GRID_DENSE = 1, 2, 4
_GRID_FLAGS = {"auto": 0, "sparse": MPM_FLAG_GRID_SPARSE, "dense": MPM_FLAG_GRID_DENSE}
EXPORTED = ("mpm_status_string", "mpm_last_error", "mpm_workspace_size", "mpm_init", "mpm_substep", "mpm_step_n", "mpm_load",
            "mpm_advance", "mpm_store", "mpm_export_frame", "mpm_tape_size",
            "mpm_backward", "mpm_grid_state", "mpm_export_covariance", "mpm_get_diagnostics",
            "mpm_set_tuning", "mpm_get_tuning", "mpm_autotune", "mpm_graph_begin", "mpm_graph_end",
            "mpm_graph_launch", "mpm_graph_destroy", "mpm_position_loss_grad", "mpm_bgdo_accumulate",
            "mpm_bgdo_apply", "mpm_ipf_workspace_size", "mpm_ipf_candidates", "mpm_mcis_workspace_size", "mpm_mcis_select", "mpm_mcis_select_static", "mpm_profile",
            "mpm_profile_read",
            "mpm_destroy")
PROFILE_CLASSES = ("fused_substep", "p2g_only", "g2p_only", "sort_permute", "grid_clear", "caller_io",
                   "adjoint_g2p", "adjoint_p2g")


class MPMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class mpm_config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("grid_res", ctypes.c_int32), ("bound", ctypes.c_int32),
                ("n_batch", ctypes.c_int32), ("dt", ctypes.c_float), ("gravity", ctypes.c_float * 3),
                ("sort_every", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class mpm_material(ctypes.Structure):
    _fields_ = [("elastic", ctypes.c_int32), ("plastic", ctypes.c_int32), ("yield_stress", ctypes.c_float),
                ("friction_deg", ctypes.c_float)]


class mpm_particles(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "v", "C", "F", "mass", "vol0", "log_E", "nu", "mat_id")]


class mpm_tuning(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("sort_every", ctypes.c_int32), ("tile_cap", ctypes.c_int32),
                ("workgroups", ctypes.c_int32), ("ms_per_substep", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class mpm_diag(ctypes.Structure):
    _fields_ = [("nonfinite", ctypes.c_int64), ("out_of_grid", ctypes.c_int64), ("tile_overflow", ctypes.c_int64),
                ("tile_escapes", ctypes.c_int64), ("substeps", ctypes.c_int64), ("cfl_violations", ctypes.c_int64),
                ("max_cfl", ctypes.c_double), ("max_wave_cfl", ctypes.c_double), ("order_fallbacks", ctypes.c_int64),
                ("det_rescales", ctypes.c_int64)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library (built by ``paper_2602_01723_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2602_01723_amd.build` "
                           "(there is no other implementation of the substep)")
    # torch's HIP runtime first: the library then binds to the same
    # libamdhip64 (one runtime per process).  Loaded the other way round,
    # torch would find the system runtime already in place and see no device.
    import torch
    if torch.cuda.is_available():
        torch.cuda.init()
    lib = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "mpm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "mpm_last_error": (ctypes.c_char_p, [vp]),
        "mpm_workspace_size": (ctypes.c_int, [ctypes.POINTER(mpm_config), i64, ctypes.POINTER(sz)]),
        "mpm_init": (ctypes.c_int, [ctypes.POINTER(mpm_config), ctypes.POINTER(mpm_material), i32, i64,
                                    ctypes.POINTER(ctypes.c_int64), vp, sz, ctypes.POINTER(vp)]),
        "mpm_substep": (ctypes.c_int, [vp, ctypes.POINTER(mpm_particles), vp]),
        "mpm_step_n": (ctypes.c_int, [vp, ctypes.POINTER(mpm_particles), i32, vp, i32, vp]),
        "mpm_load": (ctypes.c_int, [vp, ctypes.POINTER(mpm_particles), vp]),
        "mpm_advance": (ctypes.c_int, [vp, i32, vp]),
        "mpm_store": (ctypes.c_int, [vp, ctypes.POINTER(mpm_particles), vp]),
        "mpm_export_frame": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "mpm_tape_size": (ctypes.c_int, [vp, i32, i32, ctypes.POINTER(sz)]),
        "mpm_backward": (ctypes.c_int, [vp, ctypes.POINTER(mpm_particles), vp, i32] + [vp] * 10 + [vp]),
        "mpm_grid_state": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "mpm_export_covariance": (ctypes.c_int, [vp, vp, vp, vp, i64, vp]),
        "mpm_get_diagnostics": (ctypes.c_int, [vp, ctypes.POINTER(mpm_diag)]),
        "mpm_set_tuning": (ctypes.c_int, [vp, ctypes.POINTER(mpm_tuning)]),
        "mpm_get_tuning": (ctypes.c_int, [vp, ctypes.POINTER(mpm_tuning)]),
        "mpm_autotune": (ctypes.c_int, [vp, ctypes.POINTER(mpm_particles), i32, vp, ctypes.POINTER(mpm_tuning)]),
        "mpm_graph_begin": (ctypes.c_int, [vp, vp]),
        "mpm_graph_end": (ctypes.c_int, [vp, vp, ctypes.POINTER(vp)]),
        "mpm_position_loss_grad": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
        "mpm_graph_launch": (ctypes.c_int, [vp, vp]),
        "mpm_bgdo_accumulate": (ctypes.c_int, [vp, ctypes.POINTER(mpm_particles), vp, ctypes.c_float, vp, vp, vp, vp]),
        "mpm_bgdo_apply": (ctypes.c_int, [vp, vp, vp, i32, vp]),
        "mpm_ipf_workspace_size": (ctypes.c_int, [i32, i64, i64, i64, ctypes.POINTER(sz)]),
        "mpm_ipf_candidates": (ctypes.c_int, [i32, vp, ctypes.POINTER(i64), vp, ctypes.POINTER(i64), vp,
                                              ctypes.POINTER(i64), ctypes.c_double, vp, sz, vp, vp,
                                              ctypes.POINTER(i64), vp]),
        "mpm_mcis_workspace_size": (ctypes.c_int, [i32, i64, i64, ctypes.c_double, ctypes.c_double,
                                                   ctypes.POINTER(sz)]),
        "mpm_mcis_select": (ctypes.c_int, [i32, vp, ctypes.POINTER(i64), vp, ctypes.POINTER(i64), vp,
                                           ctypes.POINTER(i64), ctypes.c_double, ctypes.c_double, vp, sz, vp, vp,
                                           vp]),
        "mpm_mcis_select_static": (ctypes.c_int, [i32, vp, ctypes.POINTER(i64), vp, ctypes.POINTER(i64), vp,
                                                  ctypes.POINTER(i64), ctypes.c_double, ctypes.c_double, vp, vp, vp]),
        "mpm_graph_destroy": (ctypes.c_int, [vp]),
        "mpm_profile": (ctypes.c_int, [vp, i32]),
        "mpm_profile_read": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
        "mpm_destroy": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream(stream=None) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream) or None


class Context:
    """Owns an mpm_ctx and the device workspace it lives in (a torch
    tensor); destroyed on close() / garbage collection."""

    def __init__(self, handle, n_particles, n_batch, grid_res, workspace=None):
        self.handle = handle
        self.n_particles = n_particles
        self.n_batch = n_batch
        self.grid_res = grid_res
        self.workspace = workspace

    def close(self):
        if self.handle:
            load().mpm_destroy(self.handle)
            self.handle = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return load().mpm_last_error(self.handle).decode()


def _check(ctx: Optional[Context], rc: int, what: str):
    if rc != MPM_OK:
        lib = load()
        detail = ctx.last_error() if ctx is not None and ctx.handle else ""
        raise MPMError(rc, f"{what}: {lib.mpm_status_string(rc).decode()} ({detail})")


@dataclass
class Particles:
    """Device particle arrays in the library's SoA layout (float32 / int32)."""
    x: "torch.Tensor"       # [3, N]
    v: "torch.Tensor"       # [3, N]
    C: "torch.Tensor"       # [9, N]
    F: "torch.Tensor"       # [9, N]
    mass: "torch.Tensor"    # [N]
    vol0: "torch.Tensor"    # [N]
    log_E: "torch.Tensor"   # [N]
    nu: "torch.Tensor"      # [N]
    mat_id: "torch.Tensor"  # [N] int32

    @property
    def n(self) -> int:
        return int(self.mass.shape[0])

    def as_struct(self) -> mpm_particles:
        return mpm_particles(*[_ptr(getattr(self, k)) for k in ("x", "v", "C", "F", "mass", "vol0", "log_E",
                                                                "nu", "mat_id")])

    @classmethod
    def from_arrays(cls, x, v, C, F, mass, vol0, log_E, nu, mat_id, device="cuda"):
        import torch
        N = len(mass)

        def f32(a, shape):
            t = torch.as_tensor(np.ascontiguousarray(np.asarray(a, np.float32).reshape(N, shape).T)
                                if shape else np.asarray(a, np.float32))
            return t.contiguous().to(device)
        return cls(x=f32(x, 3), v=f32(v, 3), C=f32(C, 9), F=f32(F, 9), mass=f32(mass, 0), vol0=f32(vol0, 0),
                   log_E=f32(log_E, 0), nu=f32(nu, 0),
                   mat_id=torch.as_tensor(np.asarray(mat_id, np.int32)).contiguous().to(device))

    @classmethod
    def from_scene(cls, sc, device="cuda"):
        return cls.from_arrays(sc.x, sc.v, sc.C, sc.F, sc.mass, sc.vol0, sc.log_E, sc.nu, sc.mat_id, device)

    def state_numpy(self):
        """(x [N,3], v [N,3], C [N,3,3], F [N,3,3]) as float32 NumPy arrays."""
        N = self.n
        return (self.x.T.cpu().numpy().copy(), self.v.T.cpu().numpy().copy(),
                self.C.T.cpu().numpy().reshape(N, 3, 3).copy(), self.F.T.cpu().numpy().reshape(N, 3, 3).copy())

    def clone(self) -> "Particles":
        return Particles(**{k: getattr(self, k).clone() for k in self.__dataclass_fields__})


def make_config(grid_res, dt, n_batch=1, gravity=(0.0, -9.8, 0.0), bound=3, sort_every=0,
                deterministic=False, grid="auto") -> mpm_config:
    """grid: "auto", "sparse" or "dense" (block-sparse grid clearing, see
    MPM_FLAG_GRID_SPARSE in include/fastmpm.h)."""
    flags = (MPM_FLAG_DETERMINISTIC if deterministic else 0) | _GRID_FLAGS[grid]
    return mpm_config(MPM_ABI_VERSION, int(grid_res), int(bound), int(n_batch), float(dt),
                      (ctypes.c_float * 3)(*[float(g) for g in gravity]), int(sort_every), flags)


def mpm_workspace_size(cfg: mpm_config, n_particles: int) -> int:
    out = ctypes.c_size_t()
    _check(None, load().mpm_workspace_size(ctypes.byref(cfg), int(n_particles), ctypes.byref(out)),
           "mpm_workspace_size")
    return int(out.value)


def mpm_init(grid_res, dt, materials: Sequence[dict], n_particles, batch_offsets=None, gravity=(0.0, -9.8, 0.0),
             bound=3, sort_every=0, deterministic=False, grid="auto") -> Context:
    """Create a context; its device workspace is a torch uint8 tensor on the
    current device, held by the returned Context.  deterministic sets
    MPM_FLAG_DETERMINISTIC; grid chooses the grid clearing ("auto",
    "sparse", "dense")."""
    import torch
    lib = load()
    n_batch = 1 if batch_offsets is None else len(batch_offsets) - 1
    cfg = make_config(grid_res, dt, n_batch, gravity, bound, sort_every, deterministic, grid)
    mats = (mpm_material * len(materials))(*[mpm_material(int(m["elastic"]), int(m["plastic"]),
                                                          float(m.get("yield_stress", 0.0)),
                                                          float(m.get("friction_deg", 0.0))) for m in materials])
    offs = None
    if batch_offsets is not None:
        offs = (ctypes.c_int64 * len(batch_offsets))(*[int(b) for b in batch_offsets])
    nbytes = mpm_workspace_size(cfg, n_particles)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    rc = lib.mpm_init(ctypes.byref(cfg), mats, len(materials), int(n_particles), offs, _ptr(ws), nbytes,
                      ctypes.byref(h))
    _check(None, rc, "mpm_init")
    return Context(h, int(n_particles), n_batch, int(grid_res), ws)


def init_from_scene(sc, sort_every=0, deterministic=False, grid="auto") -> Context:
    return mpm_init(sc.grid_res, sc.dt, sc.materials, sc.n,
                    None if sc.n_batch == 1 else sc.batch_offsets, sc.gravity, sc.bound, sort_every, deterministic,
                    grid)


def mpm_substep(ctx: Context, p: Particles, stream=None):
    s = p.as_struct()
    _check(ctx, load().mpm_substep(ctx.handle, ctypes.byref(s), _stream(stream)), "mpm_substep")


def mpm_step_n(ctx: Context, p: Particles, n_steps: int, tape=None, checkpoint_every=0, stream=None):
    s = p.as_struct()
    rc = load().mpm_step_n(ctx.handle, ctypes.byref(s), int(n_steps), _ptr(tape), int(checkpoint_every),
                           _stream(stream))
    _check(ctx, rc, "mpm_step_n")


def mpm_load(ctx: Context, p: Particles, stream=None):
    s = p.as_struct()
    _check(ctx, load().mpm_load(ctx.handle, ctypes.byref(s), _stream(stream)), "mpm_load")


def mpm_advance(ctx: Context, n_steps: int, stream=None):
    _check(ctx, load().mpm_advance(ctx.handle, int(n_steps), _stream(stream)), "mpm_advance")


def mpm_store(ctx: Context, p: Particles, stream=None):
    s = p.as_struct()
    _check(ctx, load().mpm_store(ctx.handle, ctypes.byref(s), _stream(stream)), "mpm_store")


def mpm_export_frame(ctx: Context, x=None, cov0=None, cov=None, stream=None):
    rc = load().mpm_export_frame(ctx.handle, _ptr(x), _ptr(cov0), _ptr(cov), _stream(stream))
    _check(ctx, rc, "mpm_export_frame")


def mpm_tape_size(ctx: Context, n_steps: int, checkpoint_every: int) -> int:
    out = ctypes.c_size_t()
    _check(ctx, load().mpm_tape_size(ctx.handle, int(n_steps), int(checkpoint_every), ctypes.byref(out)),
           "mpm_tape_size")
    return int(out.value)


def mpm_backward(ctx: Context, p: Particles, tape, n_steps: int, g_x=None, g_v=None, g_C=None, g_F=None,
                 g_log_E=None, g_nu=None, g_x0=None, g_v0=None, g_C0=None, g_F0=None, stream=None):
    s = p.as_struct()
    rc = load().mpm_backward(ctx.handle, ctypes.byref(s), _ptr(tape), int(n_steps), _ptr(g_x), _ptr(g_v),
                             _ptr(g_C), _ptr(g_F), _ptr(g_log_E), _ptr(g_nu), _ptr(g_x0), _ptr(g_v0), _ptr(g_C0),
                             _ptr(g_F0), _stream(stream))
    _check(ctx, rc, "mpm_backward")


def mpm_grid_state(ctx: Context, m=None, mv=None, v=None, stream=None):
    rc = load().mpm_grid_state(ctx.handle, _ptr(m), _ptr(mv), _ptr(v), _stream(stream))
    _check(ctx, rc, "mpm_grid_state")


def grid_state(ctx: Context):
    """Convenience: (m [B, n^3], mv [B, n^3, 3], v [B, n^3, 3]) device tensors."""
    import torch
    nodes = ctx.n_batch * ctx.grid_res ** 3
    m = torch.empty(nodes, device="cuda")
    mv = torch.empty(nodes, 3, device="cuda")
    v = torch.empty(nodes, 3, device="cuda")
    mpm_grid_state(ctx, m, mv, v)
    return m, mv, v


def mpm_export_covariance(ctx: Context, F, cov0, cov, stream=None):
    n = int(F.shape[-1])
    rc = load().mpm_export_covariance(ctx.handle, _ptr(F), _ptr(cov0), _ptr(cov), n, _stream(stream))
    _check(ctx, rc, "mpm_export_covariance")


def mpm_get_diagnostics(ctx: Context) -> dict:
    d = mpm_diag()
    rc = load().mpm_get_diagnostics(ctx.handle, ctypes.byref(d))
    out = dict(nonfinite=d.nonfinite, out_of_grid=d.out_of_grid, tile_overflow=d.tile_overflow,
               tile_escapes=d.tile_escapes, substeps=d.substeps, cfl_violations=d.cfl_violations,
               max_cfl=d.max_cfl, max_wave_cfl=d.max_wave_cfl, order_fallbacks=d.order_fallbacks,
               det_rescales=d.det_rescales, status=rc)
    if rc not in (MPM_OK, MPM_EUNSTABLE):
        _check(ctx, rc, "mpm_get_diagnostics")
    return out


def mpm_set_tuning(ctx: Context, chunk=0, sort_every=0, tile_cap=0, workgroups=0):
    t = mpm_tuning(int(chunk), int(sort_every), int(tile_cap), int(workgroups), 0.0)
    _check(ctx, load().mpm_set_tuning(ctx.handle, ctypes.byref(t)), "mpm_set_tuning")


def mpm_get_tuning(ctx: Context) -> dict:
    t = mpm_tuning()
    _check(ctx, load().mpm_get_tuning(ctx.handle, ctypes.byref(t)), "mpm_get_tuning")
    return t.as_dict()


def mpm_autotune(ctx: Context, p: Particles, trial_steps: int = 8, stream=None) -> dict:
    """Run the library's autotuner on these particles (caller arrays untouched)."""
    s = p.as_struct()
    t = mpm_tuning()
    _check(ctx, load().mpm_autotune(ctx.handle, ctypes.byref(s), int(trial_steps), _stream(stream), ctypes.byref(t)),
           "mpm_autotune")
    return t.as_dict()


class Graph:
    """A captured evaluation (forward, optionally backward); see mpm_graph_capture."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep  # buffers and context the graph refers to

    def launch(self, stream=None):
        rc = load().mpm_graph_launch(self.handle, _stream(stream))
        if rc != MPM_OK:
            raise MPMError(rc, "mpm_graph_launch failed")

    def close(self):
        if self.handle:
            load().mpm_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mpm_graph_begin(ctx: Context, stream):
    """Start recording this context's calls on `stream` (a torch.cuda.Stream)."""
    _check(ctx, load().mpm_graph_begin(ctx.handle, _stream(stream)), "mpm_graph_begin")


def mpm_graph_end(ctx: Context, stream, keep=()) -> Graph:
    """Stop recording; `keep` lists the tensors the graph refers to (held alive)."""
    h = ctypes.c_void_p()
    _check(ctx, load().mpm_graph_end(ctx.handle, _stream(stream), ctypes.byref(h)), "mpm_graph_end")
    return Graph(h, (ctx,) + tuple(keep))


def mpm_position_loss_grad(ctx: Context, x, x_target, weight, g_x, stream=None):
    rc = load().mpm_position_loss_grad(ctx.handle, _ptr(x), _ptr(x_target), _ptr(weight), _ptr(g_x), _stream(stream))
    _check(ctx, rc, "mpm_position_loss_grad")


def mpm_bgdo_accumulate(ctx: Context, key: "Particles", F_next, delta_target, g_total, s_out=None, delta_out=None,
                        stream=None):
    st = key.as_struct()
    rc = load().mpm_bgdo_accumulate(ctx.handle, ctypes.byref(st), _ptr(F_next), float(delta_target),
                                    _ptr(g_total), _ptr(s_out), _ptr(delta_out), _stream(stream))
    _check(ctx, rc, "mpm_bgdo_accumulate")


def mpm_bgdo_apply(ctx: Context, log_E, g_total, n_keys, stream=None):
    rc = load().mpm_bgdo_apply(ctx.handle, _ptr(log_E), _ptr(g_total), int(n_keys), _stream(stream))
    _check(ctx, rc, "mpm_bgdo_apply")


def mpm_ipf_candidates(hull_vertices, hull_vertex_offsets, hull_triangles, hull_triangle_offsets, u, raw_offsets,
                       threshold=0.6, want_source=False, stream=None):
    """Candidate generation of the interior fill (see include/fastmpm.h).
    hull_vertices [3, V] float32, hull_triangles [3, T] int32 and u [3, R]
    float64 device tensors; offsets as integer sequences.  Returns (kept
    candidates [3, M_in] float32 device tensor, their offsets as a list of
    K+1 ints, and their raw indices [M_in] int64 or None)."""
    import torch
    lib = load()
    K = len(raw_offsets) - 1
    hvo = (ctypes.c_int64 * (K + 1))(*[int(v) for v in hull_vertex_offsets])
    hto = (ctypes.c_int64 * (K + 1))(*[int(v) for v in hull_triangle_offsets])
    ro = (ctypes.c_int64 * (K + 1))(*[int(v) for v in raw_offsets])
    R = int(ro[K])
    nbytes = ctypes.c_size_t()
    rc = lib.mpm_ipf_workspace_size(K, int(hvo[K]), int(hto[K]), R, ctypes.byref(nbytes))
    if rc:
        _check(None, rc, "mpm_ipf_workspace_size")
    dev = u.device if hasattr(u, "device") else "cuda"
    ws = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=dev)
    out = torch.empty(max(3 * R, 1), dtype=torch.float32, device=dev)
    src = torch.empty(max(R, 1), dtype=torch.int64, device=dev) if want_source else None
    co = (ctypes.c_int64 * (K + 1))()
    rc = lib.mpm_ipf_candidates(K, _ptr(hull_vertices) if int(hvo[K]) else None, hvo,
                                _ptr(hull_triangles) if int(hto[K]) else None, hto, _ptr(u) if R else None, ro,
                                float(threshold), _ptr(ws), int(nbytes.value), _ptr(out), _ptr(src), co,
                                _stream(stream))
    if rc:
        _check(None, rc, "mpm_ipf_candidates")
    offs = [int(v) for v in co]
    m = offs[K]
    return out[:3 * m].view(3, m), offs, (src[:m] if src is not None else None)


def mpm_mcis_select(surface, surface_offsets, candidates, candidate_offsets, u, n_select, sigma=0.02, eps=1e-6,
                    want_distance=False, stream=None):
    """MCIS interior filling (see include/fastmpm.h).  surface [3, S] and
    candidates [3, M] float32 device tensors, u [M] float64 device tensor,
    offsets and counts as integer sequences.  Returns (selected candidate
    indices, int64 device tensor instance by instance, and d [M] float64 or
    None)."""
    import torch
    lib = load()
    K = len(n_select)
    so = (ctypes.c_int64 * (K + 1))(*[int(v) for v in surface_offsets])
    co = (ctypes.c_int64 * (K + 1))(*[int(v) for v in candidate_offsets])
    ns = (ctypes.c_int64 * K)(*[int(v) for v in n_select])
    nbytes = ctypes.c_size_t()
    rc = lib.mpm_mcis_workspace_size(K, int(so[K]), int(co[K]), float(sigma), float(eps), ctypes.byref(nbytes))
    if rc:
        _check(None, rc, "mpm_mcis_workspace_size")
    dev = candidates.device if hasattr(candidates, "device") else "cuda"
    ws = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=dev)
    out = torch.empty(max(sum(int(v) for v in n_select), 1), dtype=torch.int64, device=dev)
    d = torch.empty(int(co[K]), dtype=torch.float64, device=dev) if want_distance else None
    rc = lib.mpm_mcis_select(K, _ptr(surface) if int(so[K]) else None, so, _ptr(candidates), co, _ptr(u), ns,
                             float(sigma), float(eps), _ptr(ws), int(nbytes.value), _ptr(out), _ptr(d),
                             _stream(stream))
    if rc:
        _check(None, rc, "mpm_mcis_select")
    return out[:sum(int(v) for v in n_select)], d


def mpm_mcis_select_static(surface, surface_offsets, candidates, candidate_offsets, u, n_select, out, sigma=0.02,
                           eps=1e-6, d=None, stream=None):
    """mpm_mcis_select on the library's fixed device scratch: no workspace is
    allocated; `out` (int64 device tensor of sum(n_select) entries) and the
    optional `d` (float64 device tensor of M entries) are the caller's."""
    lib = load()
    K = len(n_select)
    so = (ctypes.c_int64 * (K + 1))(*[int(v) for v in surface_offsets])
    co = (ctypes.c_int64 * (K + 1))(*[int(v) for v in candidate_offsets])
    ns = (ctypes.c_int64 * K)(*[int(v) for v in n_select])
    rc = lib.mpm_mcis_select_static(K, _ptr(surface) if int(so[K]) else None, so, _ptr(candidates), co, _ptr(u), ns,
                                    float(sigma), float(eps), _ptr(out), _ptr(d), _stream(stream))
    if rc:
        _check(None, rc, "mpm_mcis_select_static")


def mpm_profile(ctx: Context, enable: bool = True):
    _check(ctx, load().mpm_profile(ctx.handle, int(bool(enable))), "mpm_profile")


def mpm_profile_read(ctx: Context) -> dict:
    """{class: (total_ms, launches)} of the launches timed since the last read."""
    ms = (ctypes.c_double * 8)()
    cnt = (ctypes.c_int64 * 8)()
    _check(ctx, load().mpm_profile_read(ctx.handle, ms, cnt), "mpm_profile_read")
    return {name: (ms[k], cnt[k]) for k, name in enumerate(PROFILE_CLASSES)}


def mpm_destroy(ctx: Context):
    ctx.close()
