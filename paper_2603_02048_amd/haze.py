"""Thin Python binding of libhaze.so (include/haze.h).

Argument marshalling only: every step of the splat-and-trace path runs in the
library's gfx950 kernels.  PyTorch provides device memory (tensors) and the
current HIP stream.  Loading fails loudly when the library has not been built
(`python -m paper_2603_02048_amd.build`); there is no CPU fallback.

Function names follow the C ABI without the `hz_` prefix.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhaze.so")

OK, PENDING = 0, 1
E_INVALID, E_NOMEM, E_BUDGET, E_DEVICE, E_NOTFOUND, E_UNSUPPORTED = -1, -2, -3, -4, -5, -6
F32, F16, BF16 = 0, 1, 2
DTYPES = {"f32": F32, "f16": F16, "bf16": BF16}
RAY_OK, RAY_MAXSTEPS, RAY_NOHIT, RAY_NONFINITE, RAY_BAD_ID = 0, 1, 2, 3, 4


class HazeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class hz_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("m", C.c_void_p)]


class hz_grid(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("res", C.c_int32 * 3)]


class hz_splat_params(C.Structure):
    _fields_ = [("k_gd", C.c_float), ("h", C.c_float), ("dtype", C.c_int), ("store_scale", C.c_float)]


class hz_view(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("fwd", C.c_float * 3), ("up", C.c_float * 3), ("vfov", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32), ("plane_p", C.c_float * 3), ("plane_n", C.c_float * 3)]


class hz_step(C.Structure):
    _fields_ = [("uniform", C.c_int32), ("theta_max", C.c_float), ("ds_min", C.c_float), ("ds_max", C.c_float),
                ("eps", C.c_float), ("ds_uniform", C.c_float), ("max_steps", C.c_int32), ("tau_term", C.c_float)]


class hz_trace_out(C.Structure):
    _fields_ = [("disp", C.c_void_p), ("exit_pos", C.c_void_p), ("exit_dir", C.c_void_p), ("steps", C.c_void_p),
                ("status", C.c_void_p)]


MAX_QUADS = 8


class hz_quad(C.Structure):
    _fields_ = [("origin", C.c_float * 3), ("edge_u", C.c_float * 3), ("edge_v", C.c_float * 3)]


class hz_scene(C.Structure):
    _fields_ = [("nquads", C.c_int32), ("quads", C.POINTER(hz_quad))]


class hz_triangle(C.Structure):
    _fields_ = [("v0", C.c_float * 3), ("v1", C.c_float * 3), ("v2", C.c_float * 3), ("surface", C.c_int32)]


class hz_mesh_params(C.Structure):
    _fields_ = [("reach", C.c_float), ("cell", C.c_float), ("brute_force", C.c_int32)]


EXPORTS = ["hz_ctx_create", "hz_ctx_destroy", "hz_last_error", "hz_ctx_memory", "hz_ctx_tune", "hz_profile_enable",
           "hz_profile_select", "hz_profile_read", "hz_membench", "hz_membench_gather", "hz_splat_index_field",
           "hz_index_field_from_grid", "hz_field_read", "hz_field_info", "hz_field_release", "hz_trace_views",
           "hz_trace_views_noalloc", "hz_trace_scene", "hz_mesh_create", "hz_mesh_info", "hz_mesh_release",
           "hz_trace_mesh",
           "hz_server_start", "hz_submit", "hz_submit_scene", "hz_submit_mesh", "hz_poll", "hz_request_outputs",
           "hz_request_surface", "hz_request_timing", "hz_request_release", "hz_server_stop"]

_lib = None


def lib():
    """Load libhaze.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libhaze.so not built ({LIB_PATH}); run `python -m paper_2603_02048_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, S = C.c_void_p, C.c_int
        L.hz_ctx_create.argtypes, L.hz_ctx_create.restype = [C.c_int, C.c_uint64, C.POINTER(C.c_void_p)], S
        L.hz_ctx_destroy.argtypes, L.hz_ctx_destroy.restype = [P], None
        L.hz_last_error.argtypes, L.hz_last_error.restype = [], C.c_char_p
        L.hz_ctx_memory.argtypes, L.hz_ctx_memory.restype = [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)], S
        L.hz_ctx_tune.argtypes, L.hz_ctx_tune.restype = [P, C.c_char_p, C.c_int64], S
        L.hz_membench.argtypes = [P, C.c_uint64, C.c_int32, C.POINTER(C.c_double), P]
        L.hz_membench.restype = S
        L.hz_membench_gather.argtypes = [P, C.POINTER(hz_grid), C.c_int32, C.POINTER(hz_view), C.c_int32, C.c_float,
                                         C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64), P]
        L.hz_membench_gather.restype = S
        L.hz_profile_enable.argtypes, L.hz_profile_enable.restype = [P, C.c_int32], S
        L.hz_profile_select.argtypes, L.hz_profile_select.restype = [P, C.c_char_p], S
        L.hz_profile_read.argtypes = [P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
        L.hz_profile_read.restype = S
        L.hz_splat_index_field.argtypes = [P, C.POINTER(hz_particles), C.POINTER(hz_grid),
                                           C.POINTER(hz_splat_params), P, C.POINTER(C.c_void_p)]
        L.hz_splat_index_field.restype = S
        L.hz_index_field_from_grid.argtypes = [P, P, C.POINTER(hz_grid), C.c_int, C.c_float, P,
                                               C.POINTER(C.c_void_p)]
        L.hz_index_field_from_grid.restype = S
        L.hz_field_read.argtypes, L.hz_field_read.restype = [P, P, P, P, P, P, P], S
        L.hz_field_info.argtypes = [P, C.POINTER(hz_grid), C.POINTER(C.c_int), C.POINTER(C.c_float),
                                    C.POINTER(C.c_uint64)]
        L.hz_field_info.restype = S
        L.hz_field_release.argtypes, L.hz_field_release.restype = [P, P], S
        L.hz_trace_views.argtypes = [P, P, C.POINTER(hz_view), C.c_int32, C.POINTER(hz_step), P, C.c_int64,
                                     C.POINTER(hz_trace_out), P]
        L.hz_trace_views.restype = S
        L.hz_trace_views_noalloc.argtypes = L.hz_trace_views.argtypes
        L.hz_trace_views_noalloc.restype = S
        L.hz_trace_scene.argtypes = [P, P, C.POINTER(hz_view), C.c_int32, C.POINTER(hz_scene), C.POINTER(hz_step),
                                     P, C.c_int64, C.POINTER(hz_trace_out), P, P]
        L.hz_trace_scene.restype = S
        L.hz_mesh_create.argtypes = [P, C.POINTER(hz_triangle), C.c_int32, C.POINTER(hz_mesh_params), P,
                                     C.POINTER(C.c_void_p)]
        L.hz_mesh_create.restype = S
        L.hz_mesh_info.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_float),
                                   C.POINTER(C.c_int64), C.POINTER(C.c_uint64)]
        L.hz_mesh_info.restype = S
        L.hz_mesh_release.argtypes, L.hz_mesh_release.restype = [P, P], S
        L.hz_trace_mesh.argtypes = [P, P, C.POINTER(hz_view), C.c_int32, P, C.POINTER(hz_step), P, C.c_int64,
                                    C.POINTER(hz_trace_out), P, P, P]
        L.hz_trace_mesh.restype = S
        L.hz_server_start.argtypes, L.hz_server_start.restype = [P, C.c_int32, C.c_int64], S
        L.hz_submit.argtypes = [P, P, C.POINTER(hz_view), C.c_int32, C.POINTER(hz_step), C.POINTER(C.c_uint64)]
        L.hz_submit.restype = S
        L.hz_submit_scene.argtypes = [P, P, C.POINTER(hz_view), C.c_int32, C.POINTER(hz_scene), C.POINTER(hz_step),
                                      C.POINTER(C.c_uint64)]
        L.hz_submit_scene.restype = S
        L.hz_submit_mesh.argtypes = [P, P, C.POINTER(hz_view), C.c_int32, P, C.POINTER(hz_step),
                                     C.POINTER(C.c_uint64)]
        L.hz_submit_mesh.restype = S
        L.hz_request_surface.argtypes = [P, C.c_uint64, C.POINTER(C.c_void_p)]
        L.hz_request_surface.restype = S
        L.hz_poll.argtypes, L.hz_poll.restype = [P, C.c_uint64, C.POINTER(C.c_double)], S
        L.hz_request_outputs.argtypes = [P, C.c_uint64, C.POINTER(hz_trace_out), C.POINTER(C.c_int64)]
        L.hz_request_outputs.restype = S
        L.hz_request_timing.argtypes = [P, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.hz_request_timing.restype = S
        L.hz_request_release.argtypes, L.hz_request_release.restype = [P, C.c_uint64], S
        L.hz_server_stop.argtypes, L.hz_server_stop.restype = [P], S
        _lib = L
    return _lib


def last_error() -> str:
    return lib().hz_last_error().decode()


def _check(status: int, what: str) -> int:
    if status < 0:
        raise HazeError(status, f"{what}: {last_error()}")
    return status


def _stream(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def make_grid(grid) -> hz_grid:
    g = hz_grid()
    for a in range(3):
        g.lo[a] = float(grid.lo[a])
        g.hi[a] = float(grid.hi[a])
        g.res[a] = int(grid.res[a])
    return g


def make_view(v) -> hz_view:
    o = hz_view()
    for a in range(3):
        o.eye[a] = float(v.eye[a])
        o.fwd[a] = float(v.fwd[a])
        o.up[a] = float(v.up[a])
        o.plane_p[a] = float(v.plane_p[a])
        o.plane_n[a] = float(v.plane_n[a])
    o.vfov = float(v.vfov)
    o.width = int(v.width)
    o.height = int(v.height)
    return o


def make_views(views: Sequence) -> C.Array:
    arr = (hz_view * len(views))()
    for i, v in enumerate(views):
        arr[i] = make_view(v)
    return arr


def make_step(st) -> hz_step:
    return hz_step(int(st.uniform), float(st.theta_max), float(st.ds_min), float(st.ds_max), float(st.eps),
                   float(st.ds_uniform), int(min(st.max_steps, 2 ** 31 - 1)), float(st.tau_term))


@dataclass
class DeviceParticles:
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    m: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.x.numel())


def upload_particles(p: W.Particles, device="cuda") -> DeviceParticles:
    t = [torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device) for a in (p.x, p.y, p.z, p.m)]
    return DeviceParticles(*t)


class Field:
    """A device-resident (delta_n, grad n) field owned by a Context."""

    def __init__(self, ctx: "Context", handle: int, grid):
        self.ctx = ctx
        self.handle = handle
        self.grid = grid

    def info(self) -> dict:
        g = hz_grid()
        dt = C.c_int()
        sc = C.c_float()
        nb = C.c_uint64()
        _check(lib().hz_field_info(C.c_void_p(self.handle), C.byref(g), C.byref(dt), C.byref(sc), C.byref(nb)),
               "field_info")
        return dict(res=tuple(g.res), lo=tuple(g.lo), hi=tuple(g.hi), dtype=dt.value, store_scale=sc.value,
                    bytes=nb.value)

    def release(self):
        if self.handle:
            _check(lib().hz_field_release(C.c_void_p(self.ctx.handle), C.c_void_p(self.handle)), "field_release")
            self.handle = 0


class Mesh:
    """A device-resident triangle-mesh scene with its conservative shell."""

    def __init__(self, ctx: "Context", handle: int):
        self.ctx = ctx
        self.handle = handle

    def info(self) -> dict:
        n, res, cell, ent, nb = C.c_int32(), (C.c_int32 * 3)(), C.c_float(), C.c_int64(), C.c_uint64()
        _check(lib().hz_mesh_info(C.c_void_p(self.handle), C.byref(n), res, C.byref(cell), C.byref(ent),
                                  C.byref(nb)), "mesh_info")
        return dict(ntris=n.value, shell_res=tuple(res), shell_cell=cell.value, list_entries=ent.value,
                    bytes=nb.value)

    def release(self):
        if self.handle:
            _check(lib().hz_mesh_release(C.c_void_p(self.ctx.handle), C.c_void_p(self.handle)), "mesh_release")
            self.handle = 0


class Context:
    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = C.c_void_p()
        _check(lib().hz_ctx_create(int(device), int(budget_bytes), C.byref(h)), "ctx_create")
        self.handle = h.value
        self.device = device

    def close(self):
        if self.handle:
            lib().hz_ctx_destroy(C.c_void_p(self.handle))
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def memory(self) -> tuple:
        u, b = C.c_uint64(), C.c_uint64()
        _check(lib().hz_ctx_memory(C.c_void_p(self.handle), C.byref(u), C.byref(b)), "ctx_memory")
        return u.value, b.value

    def tune(self, key: str, value: int):
        _check(lib().hz_ctx_tune(C.c_void_p(self.handle), key.encode(), int(value)), "ctx_tune")

    def membench(self, nbytes: int, reps: int = 10, stream=None) -> float:
        """Achievable read GB/s of a buffer of `nbytes` (see hz_membench)."""
        g = C.c_double()
        _check(lib().hz_membench(C.c_void_p(self.handle), int(nbytes), int(reps), C.byref(g), _stream(stream)),
               "membench")
        return g.value

    def membench_gather(self, grid, voxel_bytes: int, views: Sequence, step_len: float, reps: int = 10,
                        stream=None) -> tuple:
        """Achievable GB/s of the marcher's 8-corner gathers along the views' own
        rays walked straight through the grid (see hz_membench_gather), and the
        samples per launch."""
        g = C.c_double()
        n = C.c_int64()
        _check(lib().hz_membench_gather(C.c_void_p(self.handle), C.byref(make_grid(grid)), int(voxel_bytes),
                                        make_views(views), len(views), float(step_len), int(reps), C.byref(g),
                                        C.byref(n), _stream(stream)), "membench_gather")
        return g.value, n.value

    def profile_enable(self, enable: bool = True):
        _check(lib().hz_profile_enable(C.c_void_p(self.handle), 1 if enable else 0), "profile_enable")

    def profile_select(self, groups=None):
        """Time only the named groups (a list or comma-separated string); None: all."""
        if groups is not None and not isinstance(groups, str):
            groups = ",".join(groups)
        _check(lib().hz_profile_select(C.c_void_p(self.handle), groups.encode() if groups else None),
               "profile_select")

    def profile_read(self, kernel: str, reset: bool = False) -> tuple:
        """(total milliseconds, launch count) of a kernel since the last reset."""
        ms, n = C.c_double(), C.c_int64()
        _check(lib().hz_profile_read(C.c_void_p(self.handle), kernel.encode(), C.byref(ms), C.byref(n),
                                     1 if reset else 0), "profile_read")
        return ms.value, n.value

    # -- index field ------------------------------------------------------
    def splat_index_field(self, particles: DeviceParticles, grid, k_gd: float, h: float, dtype: str = "f32",
                          store_scale: float = 1.0, stream=None) -> Field:
        P = hz_particles(particles.n, _ptr(particles.x), _ptr(particles.y), _ptr(particles.z), _ptr(particles.m))
        prm = hz_splat_params(float(k_gd), float(h), DTYPES[dtype], float(store_scale))
        out = C.c_void_p()
        g = make_grid(grid)
        _check(lib().hz_splat_index_field(C.c_void_p(self.handle), C.byref(P), C.byref(g), C.byref(prm),
                                          _stream(stream), C.byref(out)), "splat_index_field")
        return Field(self, out.value, grid)

    def index_field_from_grid(self, dn: torch.Tensor, grid, dtype: str = "f32", store_scale: float = 1.0,
                              stream=None) -> Field:
        assert dn.dtype == torch.float32 and dn.is_contiguous() and dn.is_cuda
        out = C.c_void_p()
        g = make_grid(grid)
        _check(lib().hz_index_field_from_grid(C.c_void_p(self.handle), _ptr(dn), C.byref(g), DTYPES[dtype],
                                              float(store_scale), _stream(stream), C.byref(out)),
               "index_field_from_grid")
        return Field(self, out.value, grid)

    def field_read(self, field: Field, stream=None) -> tuple:
        res = [int(r) for r in field.grid.res]
        shape = (res[2], res[1], res[0])
        arrs = [torch.empty(shape, dtype=torch.float32, device="cuda") for _ in range(4)]
        _check(lib().hz_field_read(C.c_void_p(self.handle), C.c_void_p(field.handle), *[_ptr(a) for a in arrs],
                                   _stream(stream)), "field_read")
        return tuple(arrs)

    # -- tracing ----------------------------------------------------------
    def trace_views(self, field: Field, views: Sequence, step, ray_ids: Optional[torch.Tensor] = None,
                    out: Optional[dict] = None, stream=None) -> dict:
        total = sum(int(v.width) * int(v.height) for v in views)
        n = total if ray_ids is None else int(ray_ids.numel())
        if out is None:
            out = alloc_outputs(n)
        o = hz_trace_out(_ptr(out.get("disp")), _ptr(out.get("exit_pos")), _ptr(out.get("exit_dir")),
                         _ptr(out.get("steps")), _ptr(out.get("status")))
        vs = make_views(views)
        st = make_step(step)
        if ray_ids is not None:
            assert ray_ids.dtype == torch.int64 and ray_ids.is_cuda and ray_ids.is_contiguous()
        _check(lib().hz_trace_views(C.c_void_p(self.handle), C.c_void_p(field.handle), vs, len(views),
                                    C.byref(st), _ptr(ray_ids), n, C.byref(o), _stream(stream)), "trace_views")
        return out

    def trace_views_noalloc(self, field: Field, views: Sequence, step, ray_ids: Optional[torch.Tensor] = None,
                            out: Optional[dict] = None, stream=None) -> dict:
        """trace_views with the launch scratch in the library's static device
        array (hz_trace_views_noalloc): the call allocates no device memory
        (`out` is allocated here when not given)."""
        total = sum(int(v.width) * int(v.height) for v in views)
        n = total if ray_ids is None else int(ray_ids.numel())
        if out is None:
            out = alloc_outputs(n)
        o = hz_trace_out(_ptr(out.get("disp")), _ptr(out.get("exit_pos")), _ptr(out.get("exit_dir")),
                         _ptr(out.get("steps")), _ptr(out.get("status")))
        if ray_ids is not None:
            assert ray_ids.dtype == torch.int64 and ray_ids.is_cuda and ray_ids.is_contiguous()
        _check(lib().hz_trace_views_noalloc(C.c_void_p(self.handle), C.c_void_p(field.handle), make_views(views),
                                            len(views), C.byref(make_step(step)), _ptr(ray_ids), n, C.byref(o),
                                            _stream(stream)), "trace_views_noalloc")
        return out

    def trace_scene(self, field: Field, views: Sequence, quads, step, ray_ids: Optional[torch.Tensor] = None,
                    out: Optional[dict] = None, stream=None) -> dict:
        """trace_views with scene boards: `quads` is (K, 3, 3) = K x (origin,
        edge_u, edge_v).  The outputs gain `surface` (uint8: 0 backdrop, k + 1
        board k, 255 none)."""
        total = sum(int(v.width) * int(v.height) for v in views)
        n = total if ray_ids is None else int(ray_ids.numel())
        if out is None:
            out = alloc_outputs(n)
        if "surface" not in out:
            out["surface"] = torch.empty(n, dtype=torch.uint8, device=out["status"].device)
        o = hz_trace_out(_ptr(out.get("disp")), _ptr(out.get("exit_pos")), _ptr(out.get("exit_dir")),
                         _ptr(out.get("steps")), _ptr(out.get("status")))
        sc, _keep = _make_scene(quads)
        if ray_ids is not None:
            assert ray_ids.dtype == torch.int64 and ray_ids.is_cuda and ray_ids.is_contiguous()
        _check(lib().hz_trace_scene(C.c_void_p(self.handle), C.c_void_p(field.handle), make_views(views),
                                    len(views), C.byref(sc), C.byref(make_step(step)), _ptr(ray_ids), n,
                                    C.byref(o), _ptr(out["surface"]), _stream(stream)), "trace_scene")
        return out

    def mesh_create(self, tris, surfaces, reach: float, cell: float = 0.0, brute_force: bool = False,
                    stream=None) -> Mesh:
        """A mesh scene from (T, 3, 3) triangle vertices and (T,) surface ids."""
        v = np.asarray(tris, np.float32).reshape(-1, 3, 3)
        sf = np.asarray(surfaces, np.int64).reshape(-1)
        arr = (hz_triangle * max(1, v.shape[0]))()
        for i in range(v.shape[0]):
            arr[i] = hz_triangle((C.c_float * 3)(*v[i, 0]), (C.c_float * 3)(*v[i, 1]), (C.c_float * 3)(*v[i, 2]),
                                 int(sf[i]))
        prm = hz_mesh_params(float(reach), float(cell), 1 if brute_force else 0)
        out = C.c_void_p()
        _check(lib().hz_mesh_create(C.c_void_p(self.handle), arr, v.shape[0], C.byref(prm), _stream(stream),
                                    C.byref(out)), "mesh_create")
        return Mesh(self, out.value)

    def trace_mesh(self, field: Field, views: Sequence, mesh: Mesh, step, ray_ids: Optional[torch.Tensor] = None,
                   out: Optional[dict] = None, count_tests: bool = False, stream=None) -> dict:
        """trace_views against a triangle mesh: outputs gain `surface` (uint8: 0
        backdrop, s + 1 surface s, 255 none) and, with count_tests, `tri_tests`
        (exact ray-triangle tests per ray)."""
        total = sum(int(v.width) * int(v.height) for v in views)
        n = total if ray_ids is None else int(ray_ids.numel())
        if out is None:
            out = alloc_outputs(n)
        dev = out["status"].device
        if "surface" not in out:
            out["surface"] = torch.empty(n, dtype=torch.uint8, device=dev)
        if count_tests and "tri_tests" not in out:
            out["tri_tests"] = torch.empty(n, dtype=torch.int32, device=dev)
        o = hz_trace_out(_ptr(out.get("disp")), _ptr(out.get("exit_pos")), _ptr(out.get("exit_dir")),
                         _ptr(out.get("steps")), _ptr(out.get("status")))
        if ray_ids is not None:
            assert ray_ids.dtype == torch.int64 and ray_ids.is_cuda and ray_ids.is_contiguous()
        _check(lib().hz_trace_mesh(C.c_void_p(self.handle), C.c_void_p(field.handle), make_views(views), len(views),
                                   C.c_void_p(mesh.handle), C.byref(make_step(step)), _ptr(ray_ids), n, C.byref(o),
                                   _ptr(out["surface"]), _ptr(out.get("tri_tests")), _stream(stream)), "trace_mesh")
        return out

    # -- serving ----------------------------------------------------------
    def server_start(self, slots: int = 4, max_batch_rays: int = 1 << 23):
        _check(lib().hz_server_start(C.c_void_p(self.handle), int(slots), int(max_batch_rays)), "server_start")

    def submit(self, field: Field, views: Sequence, step, quads=None, mesh: Optional[Mesh] = None) -> int:
        """Submit a request (with scene boards `quads`, (K, 3, 3), or a Mesh,
        if given).  Releasing the field or mesh fails while the request waits
        to be launched."""
        t = C.c_uint64()
        if mesh is not None:
            if quads is not None:
                raise ValueError("submit: boards and a mesh cannot be combined")
            _check(lib().hz_submit_mesh(C.c_void_p(self.handle), C.c_void_p(field.handle), make_views(views),
                                        len(views), C.c_void_p(mesh.handle), C.byref(make_step(step)), C.byref(t)),
                   "submit_mesh")
        elif quads is None:
            _check(lib().hz_submit(C.c_void_p(self.handle), C.c_void_p(field.handle), make_views(views), len(views),
                                   C.byref(make_step(step)), C.byref(t)), "submit")
        else:
            sc, _keep = _make_scene(quads)
            _check(lib().hz_submit_scene(C.c_void_p(self.handle), C.c_void_p(field.handle), make_views(views),
                                         len(views), C.byref(sc), C.byref(make_step(step)), C.byref(t)),
                   "submit_scene")
        return t.value

    def poll(self, ticket: int) -> Optional[float]:
        lat = C.c_double()
        s = _check(lib().hz_poll(C.c_void_p(self.handle), C.c_uint64(ticket), C.byref(lat)), "poll")
        return None if s == PENDING else lat.value

    def request_outputs(self, ticket: int, copy: bool = True) -> dict:
        """A completed request's outputs as torch tensors on the GPU (copies by
        default, complete on return; with copy=False, views valid until
        request_release, whose reads must have completed before it)."""
        o = hz_trace_out()
        n = C.c_int64()
        _check(lib().hz_request_outputs(C.c_void_p(self.handle), C.c_uint64(ticket), C.byref(o), C.byref(n)),
               "request_outputs")
        sp = C.c_void_p()
        _check(lib().hz_request_surface(C.c_void_p(self.handle), C.c_uint64(ticket), C.byref(sp)),
               "request_surface")
        return _wrap_device_outputs(o, n.value, copy, sp.value)

    def request_timing(self, ticket: int) -> tuple:
        """(device start ms, device end ms) of the launch that carried a
        completed request, from the server's start."""
        a, b = C.c_double(), C.c_double()
        _check(lib().hz_request_timing(C.c_void_p(self.handle), C.c_uint64(ticket), C.byref(a), C.byref(b)),
               "request_timing")
        return a.value, b.value

    def request_release(self, ticket: int):
        _check(lib().hz_request_release(C.c_void_p(self.handle), C.c_uint64(ticket)), "request_release")

    def server_stop(self):
        _check(lib().hz_server_stop(C.c_void_p(self.handle)), "server_stop")


def _make_scene(quads):
    """hz_scene of (K, 3, 3) boards; returns the struct and the array it points to."""
    q = np.asarray(quads, np.float32).reshape(-1, 3, 3)
    arr = (hz_quad * max(1, q.shape[0]))()
    for k in range(q.shape[0]):
        arr[k] = hz_quad((C.c_float * 3)(*q[k, 0]), (C.c_float * 3)(*q[k, 1]), (C.c_float * 3)(*q[k, 2]))
    return hz_scene(q.shape[0], arr), arr


def alloc_outputs(n: int, device="cuda") -> dict:
    return dict(disp=torch.empty((n, 2), dtype=torch.float32, device=device),
                exit_pos=torch.empty((n, 3), dtype=torch.float32, device=device),
                exit_dir=torch.empty((n, 3), dtype=torch.float32, device=device),
                steps=torch.empty(n, dtype=torch.int32, device=device),
                status=torch.empty(n, dtype=torch.uint8, device=device))


class _DeviceArray:
    """Zero-copy view of library-owned device memory (CUDA array interface)."""

    def __init__(self, ptr: int, shape: tuple, typestr: str):
        self.__cuda_array_interface__ = {"data": (int(ptr), False), "shape": shape, "typestr": typestr,
                                         "version": 2, "strides": None}


def _wrap_device_outputs(o: hz_trace_out, n: int, copy: bool = True, surface: Optional[int] = None) -> dict:
    """Torch tensors over a request's library-owned outputs (cloned by default,
    since the library reuses them after request_release)."""
    spec = [("disp", o.disp, (n, 2), "<f4"), ("exit_pos", o.exit_pos, (n, 3), "<f4"),
            ("exit_dir", o.exit_dir, (n, 3), "<f4"), ("steps", o.steps, (n,), "<i4"), ("status", o.status, (n,), "|u1")]
    if surface:
        spec.append(("surface", surface, (n,), "|u1"))
    out = {}
    for name, ptr, shape, ts in spec:
        t = torch.as_tensor(_DeviceArray(ptr, shape, ts), device="cuda")
        out[name] = t.clone() if copy else t
    if copy:
        # the library reuses the memory once the request is released
        torch.cuda.current_stream().synchronize()
    return out
