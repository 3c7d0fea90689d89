"""FP64 CPU oracle of the splat-and-trace path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It loads `libhaze_oracle.so`, compiled from the plain C
in this directory (`haze_oracle.c`), which shares no code with the HIP path.

Every function takes the seeded inputs drawn by
`paper_2603_02048_amd.workloads` (float32 particle and camera values are
widened to float64 here) and returns float64 numpy arrays.  Arrays on the grid
are indexed [z][y][x].

What each function follows in the paper:
  splat          Sec. 3.3.1 and Eq. 12 (kernel splat at voxel centres, Gladstone-Dale)
  gradient       Sec. 3.3.1 and Eq. 13 (finite differences on the grid)
  sample         Sec. 3.3.1 (trilinear n and grad n along the ray)
  trace_views    Sec. 3.3.2-3.3.3, Eqs. 16-18, Fig. 1 caption (straight outside),
                 Sec. 3.3.2 last paragraph (image purely from bending)
  trace_scene    the same with planar scene surfaces anywhere along the ray
                 (the slanted and two-board scenes of Sec. 4.2)
  reference_views  the continuous ODE of Eq. 15 through the same medium
                 (step halving + Richardson extrapolation)
  trace_rays_rk4 classical RK4 on Eq. 15, a cross-check of the reference
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "haze_oracle.c")
_LIB = os.path.join(_HERE, "libhaze_oracle.so")

MEDIUM_GRID, MEDIUM_CONST, MEDIUM_LINEAR, MEDIUM_NSQ_LINEAR, MEDIUM_GAUSS = 0, 1, 2, 3, 4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("res", C.c_int32 * 3)]


class _Medium(C.Structure):
    _fields_ = [("kind", C.c_int32), ("grid", _Grid), ("dn", C.c_void_p), ("gx", C.c_void_p),
                ("gy", C.c_void_p), ("gz", C.c_void_p), ("p", C.c_double * 8)]


class _View(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("fwd", C.c_double * 3), ("up", C.c_double * 3), ("vfov", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32), ("plane_p", C.c_double * 3),
                ("plane_n", C.c_double * 3)]


class _Step(C.Structure):
    _fields_ = [("uniform", C.c_int32), ("theta_max", C.c_double), ("ds_min", C.c_double),
                ("ds_max", C.c_double), ("eps", C.c_double), ("ds_uniform", C.c_double),
                ("max_steps", C.c_int64), ("tau_term", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.ho_kernel.restype = C.c_double
        L.ho_kernel.argtypes = [C.c_double, C.c_double]
        L.ho_splat_brute.restype = None
        L.ho_splat_brute.argtypes = [C.c_int64, P, P, P, P, C.POINTER(_Grid), C.c_double, C.c_double, P]
        L.ho_splat_cells.restype = C.c_int
        L.ho_splat_cells.argtypes = [C.c_int64, P, P, P, P, C.POINTER(_Grid), C.c_double, C.c_double, P]
        L.ho_gradient.restype = None
        L.ho_gradient.argtypes = [P, C.POINTER(_Grid), P, P, P]
        L.ho_sample.restype = None
        L.ho_sample.argtypes = [C.POINTER(_Medium), P, P, P]
        L.ho_step_length.restype = C.c_double
        L.ho_step_length.argtypes = [C.POINTER(_Step), C.c_double, P, P]
        L.ho_advance.restype = C.c_double
        L.ho_advance.argtypes = [C.POINTER(_Medium), C.POINTER(_Step), C.c_double, P, P]
        L.ho_curvature.restype = C.c_double
        L.ho_curvature.argtypes = [C.c_double, P, P]
        L.ho_trace_views.restype = C.c_int
        L.ho_trace_views.argtypes = [C.POINTER(_Medium), C.POINTER(_View), C.c_int32, C.POINTER(_Step), P,
                                     C.c_int64, P, P, P, P, P]
        L.ho_trace_scene.restype = C.c_int
        L.ho_trace_scene.argtypes = [C.POINTER(_Medium), C.POINTER(_View), C.c_int32, P, C.c_int32,
                                     C.POINTER(_Step), P, C.c_int64, P, P, P, P, P, P]
        L.ho_trace_mesh.restype = C.c_int
        L.ho_trace_mesh.argtypes = [C.POINTER(_Medium), C.POINTER(_View), C.c_int32, P, C.c_int32,
                                    C.POINTER(_Step), P, C.c_int64, P, P, P, P, P, P]
        L.ho_trace_rays.restype = C.c_int
        L.ho_trace_rays.argtypes = [C.POINTER(_Medium), C.POINTER(_Step), P, P, C.c_int64, P, P, P, P]
        L.ho_trace_rays_rk4.restype = C.c_int
        L.ho_trace_rays_rk4.argtypes = [C.POINTER(_Medium), C.c_double, C.c_int64, C.c_double, P, P, C.c_int64,
                                        P, P, P, P]
        L.ho_pixel_rays.restype = C.c_int
        L.ho_pixel_rays.argtypes = [C.POINTER(_View), P, C.c_int64, P]
        L.ho_backdrop.restype = C.c_int
        L.ho_backdrop.argtypes = [C.POINTER(_View), P, P, P, C.c_int64, P, P]
        L.ho_reference_views.restype = C.c_int
        L.ho_reference_views.argtypes = [C.POINTER(_Medium), C.POINTER(_View), C.c_int32, C.POINTER(_Step),
                                         C.c_double, C.c_int32, C.c_double, C.c_double, P, C.c_int64, P, P, P,
                                         P, P]
        L.ho_num_threads.restype = C.c_int
        L.ho_num_threads.argtypes = []
        L.ho_set_num_threads.restype = None
        L.ho_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _grid(grid) -> _Grid:
    g = _Grid()
    for a in range(3):
        g.lo[a] = float(grid.lo[a])
        g.hi[a] = float(grid.hi[a])
        g.res[a] = int(grid.res[a])
    return g


def _view(v) -> _View:
    o = _View()
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


def _step(st) -> _Step:
    return _Step(int(st.uniform), float(st.theta_max), float(st.ds_min), float(st.ds_max), float(st.eps),
                 float(st.ds_uniform), int(st.max_steps), float(st.tau_term))


def num_threads() -> int:
    return int(lib().ho_num_threads())


def set_num_threads(n: int):
    lib().ho_set_num_threads(int(n))


def kernel(r, h: float) -> np.ndarray:
    r = np.atleast_1d(np.asarray(r, np.float64))
    return np.array([lib().ho_kernel(float(v), float(h)) for v in r.ravel()]).reshape(r.shape)


def splat(particles, grid, k_gd: float, h: float, method: str = "auto") -> np.ndarray:
    """delta_n at voxel centres, [z][y][x] float64."""
    res = [int(r) for r in grid.res]
    out = np.zeros((res[2], res[1], res[0]), np.float64)
    xs = [np.ascontiguousarray(a, np.float32) for a in (particles.x, particles.y, particles.z, particles.m)]
    n = int(xs[0].shape[0])
    g = _grid(grid)
    if method == "auto":
        method = "brute" if n * out.size <= 2e8 else "cells"
    if method == "brute":
        lib().ho_splat_brute(n, *[_ptr(a) for a in xs], C.byref(g), float(k_gd), float(h), _ptr(out))
    elif method == "cells":
        rc = lib().ho_splat_cells(n, *[_ptr(a) for a in xs], C.byref(g), float(k_gd), float(h), _ptr(out))
        if rc != 0:
            raise MemoryError("oracle cell list allocation failed")
    else:
        raise ValueError(method)
    return out


def gradient(dn: np.ndarray, grid) -> tuple:
    dn = np.ascontiguousarray(dn, np.float64)
    gx, gy, gz = (np.empty_like(dn) for _ in range(3))
    lib().ho_gradient(_ptr(dn), C.byref(_grid(grid)), _ptr(gx), _ptr(gy), _ptr(gz))
    return gx, gy, gz


class Medium:
    """A refractive medium: a gridded field, or an analytic one for closed-form pins."""

    def __init__(self, kind: int, grid, params: Sequence[float] = (), arrays=None):
        self.kind = kind
        self.grid = grid
        self._keep = None
        m = _Medium()
        m.kind = kind
        m.grid = _grid(grid)
        for i, p in enumerate(params):
            m.p[i] = float(p)
        if arrays is not None:
            self._keep = [np.ascontiguousarray(a, np.float64) for a in arrays]
            m.dn, m.gx, m.gy, m.gz = [a.ctypes.data for a in self._keep]
        self._m = m

    @property
    def arrays(self):
        """(dn, gx, gy, gz) of a gridded medium, [z][y][x] float64."""
        return tuple(self._keep) if self._keep is not None else None

    @classmethod
    def from_grid(cls, grid, dn, gx=None, gy=None, gz=None):
        if gx is None:
            gx, gy, gz = gradient(dn, grid)
        return cls(MEDIUM_GRID, grid, arrays=(dn, gx, gy, gz))

    @property
    def ref(self):
        return C.byref(self._m)


def field(particles, grid, k_gd: float, h: float, method: str = "auto") -> Medium:
    """Splat + gradient: the gridded medium the tracer samples."""
    dn = splat(particles, grid, k_gd, h, method)
    return Medium.from_grid(grid, dn)


def sample(medium: Medium, points: np.ndarray) -> tuple:
    pts = np.ascontiguousarray(np.atleast_2d(points), np.float64)
    n = np.empty(pts.shape[0])
    g = np.empty((pts.shape[0], 3))
    L = lib()
    for i in range(pts.shape[0]):
        nn = np.empty(1)
        gg = np.empty(3)
        L.ho_sample(medium.ref, _ptr(pts[i]), _ptr(nn), _ptr(gg))
        n[i] = nn[0]
        g[i] = gg
    return n, g


def step_length(step, n: float, w, g) -> float:
    w = np.ascontiguousarray(w, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    return float(lib().ho_step_length(C.byref(_step(step)), float(n), _ptr(w), _ptr(g)))


def advance(medium: "Medium", step, c, w, te: float = float("inf")) -> tuple:
    """One update of Eq. 16 from position c, direction w; returns (c', w', n_k)."""
    c = np.array(c, np.float64)
    w = np.array(w, np.float64)
    n = lib().ho_advance(medium.ref, C.byref(_step(step)), float(te), _ptr(c), _ptr(w))
    return c, w, float(n)


def curvature(n: float, w, g) -> float:
    w = np.ascontiguousarray(w, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    return float(lib().ho_curvature(float(n), _ptr(w), _ptr(g)))


def _views(views):
    arr = (_View * len(views))()
    for i, v in enumerate(views):
        arr[i] = _view(v)
    return arr


def trace_views(medium: Medium, views, step, ray_ids: Optional[np.ndarray] = None) -> dict:
    """Per-ray exit position/direction, step count, status and displacement (px)."""
    total = sum(int(v.width) * int(v.height) for v in views)
    ids = None if ray_ids is None else np.ascontiguousarray(ray_ids, np.int64)
    n = total if ids is None else int(ids.shape[0])
    out = dict(disp=np.empty((n, 2)), exit_pos=np.empty((n, 3)), exit_dir=np.empty((n, 3)),
               steps=np.empty(n, np.int64), status=np.empty(n, np.uint8))
    rc = lib().ho_trace_views(medium.ref, _views(views), len(views), C.byref(_step(step)),
                              None if ids is None else _ptr(ids), n, _ptr(out["disp"]), _ptr(out["exit_pos"]),
                              _ptr(out["exit_dir"]), _ptr(out["steps"]), _ptr(out["status"]))
    if rc != 0:
        raise ValueError(f"oracle trace failed ({rc}): ray id out of range")
    return out


def trace_scene(medium: Medium, views, quads, step, ray_ids: Optional[np.ndarray] = None) -> dict:
    """trace_views with scene quads: `quads` is (K, 3, 3) = K x (origin, edge_u,
    edge_v), each the parallelogram origin + u edge_u + v edge_v, 0 <= u, v <= 1.
    Adds `surface` per ray: 0 backdrop plane, k + 1 quad k, 255 none."""
    q = np.ascontiguousarray(np.asarray(quads, np.float64).reshape(-1, 3, 3))
    total = sum(int(v.width) * int(v.height) for v in views)
    ids = None if ray_ids is None else np.ascontiguousarray(ray_ids, np.int64)
    n = total if ids is None else int(ids.shape[0])
    out = dict(disp=np.empty((n, 2)), exit_pos=np.empty((n, 3)), exit_dir=np.empty((n, 3)),
               steps=np.empty(n, np.int64), status=np.empty(n, np.uint8), surface=np.empty(n, np.uint8))
    rc = lib().ho_trace_scene(medium.ref, _views(views), len(views), _ptr(q) if q.shape[0] else None, q.shape[0],
                              C.byref(_step(step)), None if ids is None else _ptr(ids), n, _ptr(out["disp"]),
                              _ptr(out["exit_pos"]), _ptr(out["exit_dir"]), _ptr(out["steps"]),
                              _ptr(out["status"]), _ptr(out["surface"]))
    if rc != 0:
        raise ValueError(f"oracle trace failed ({rc}): ray id out of range")
    return out


class _Tri(C.Structure):
    _fields_ = [("v0", C.c_double * 3), ("e1", C.c_double * 3), ("e2", C.c_double * 3), ("surf", C.c_int32)]


def trace_mesh(medium: Medium, views, tris, surfaces, step, ray_ids: Optional[np.ndarray] = None) -> dict:
    """trace_views with a triangle-mesh scene, every chord and straight segment
    tested against every triangle: `tris` is (T, 3, 3) vertices (v0, v1, v2)
    per triangle, `surfaces` (T,) the surface each belongs to.  Adds `surface`
    per ray: 0 backdrop plane, s + 1 a triangle of surface s, 255 none."""
    v = np.asarray(tris, np.float64).reshape(-1, 3, 3)
    sf = np.asarray(surfaces, np.int64).reshape(-1)
    assert sf.shape[0] == v.shape[0]
    arr = (_Tri * max(1, v.shape[0]))()
    for i in range(v.shape[0]):
        t = arr[i]
        for a in range(3):
            t.v0[a] = float(v[i, 0, a])
            t.e1[a] = float(v[i, 1, a] - v[i, 0, a])
            t.e2[a] = float(v[i, 2, a] - v[i, 0, a])
        t.surf = int(sf[i])
    total = sum(int(vw.width) * int(vw.height) for vw in views)
    ids = None if ray_ids is None else np.ascontiguousarray(ray_ids, np.int64)
    n = total if ids is None else int(ids.shape[0])
    out = dict(disp=np.empty((n, 2)), exit_pos=np.empty((n, 3)), exit_dir=np.empty((n, 3)),
               steps=np.empty(n, np.int64), status=np.empty(n, np.uint8), surface=np.empty(n, np.uint8))
    rc = lib().ho_trace_mesh(medium.ref, _views(views), len(views), C.cast(arr, C.c_void_p) if v.shape[0] else None,
                             v.shape[0], C.byref(_step(step)), None if ids is None else _ptr(ids), n,
                             _ptr(out["disp"]), _ptr(out["exit_pos"]), _ptr(out["exit_dir"]), _ptr(out["steps"]),
                             _ptr(out["status"]), _ptr(out["surface"]))
    if rc != 0:
        raise ValueError(f"oracle trace failed ({rc}): ray id out of range")
    return out


def trace_rays(medium: Medium, step, origins: np.ndarray, dirs: np.ndarray) -> dict:
    o = np.ascontiguousarray(np.atleast_2d(origins), np.float64)
    d = np.ascontiguousarray(np.atleast_2d(dirs), np.float64)
    n = o.shape[0]
    out = dict(exit_pos=np.empty((n, 3)), exit_dir=np.empty((n, 3)), steps=np.empty(n, np.int64),
               status=np.empty(n, np.uint8))
    lib().ho_trace_rays(medium.ref, C.byref(_step(step)), _ptr(o), _ptr(d), n, _ptr(out["exit_pos"]),
                        _ptr(out["exit_dir"]), _ptr(out["steps"]), _ptr(out["status"]))
    return out


def trace_rays_rk4(medium: Medium, ds: float, origins: np.ndarray, dirs: np.ndarray, tau: float = 0.0,
                   max_steps: int = 1 << 40) -> dict:
    o = np.ascontiguousarray(np.atleast_2d(origins), np.float64)
    d = np.ascontiguousarray(np.atleast_2d(dirs), np.float64)
    n = o.shape[0]
    out = dict(exit_pos=np.empty((n, 3)), exit_dir=np.empty((n, 3)), steps=np.empty(n, np.int64),
               status=np.empty(n, np.uint8))
    lib().ho_trace_rays_rk4(medium.ref, float(ds), int(max_steps), float(tau), _ptr(o), _ptr(d), n,
                            _ptr(out["exit_pos"]), _ptr(out["exit_dir"]), _ptr(out["steps"]), _ptr(out["status"]))
    return out


def pixel_rays(view, pixels: np.ndarray) -> np.ndarray:
    pix = np.ascontiguousarray(np.atleast_2d(pixels), np.int64)
    d = np.empty((pix.shape[0], 3))
    lib().ho_pixel_rays(C.byref(_view(view)), _ptr(pix), pix.shape[0], _ptr(d))
    return d


def backdrop(view, pixels: np.ndarray, x: np.ndarray, w: np.ndarray) -> tuple:
    pix = np.ascontiguousarray(np.atleast_2d(pixels), np.int64)
    xx = np.ascontiguousarray(np.atleast_2d(x), np.float64)
    ww = np.ascontiguousarray(np.atleast_2d(w), np.float64)
    n = pix.shape[0]
    disp = np.empty((n, 2))
    st = np.empty(n, np.uint8)
    lib().ho_backdrop(C.byref(_view(view)), _ptr(pix), _ptr(xx), _ptr(ww), n, _ptr(disp), _ptr(st))
    return disp, st


def reference_views(medium: Medium, views, step, ray_ids: Optional[np.ndarray] = None, ds0: Optional[float] = None,
                    max_levels: int = 14, tol_px: float = 1e-4, tol_dir: float = 1e-8) -> dict:
    """Converged solution of the continuous ray ODE through `medium` (fixed-step
    halving from ds0, default 1/8 voxel, then Richardson extrapolation)."""
    total = sum(int(v.width) * int(v.height) for v in views)
    ids = None if ray_ids is None else np.ascontiguousarray(ray_ids, np.int64)
    n = total if ids is None else int(ids.shape[0])
    if ds0 is None:
        ds0 = medium.grid.voxel / 8.0
    # the continuous path leaves exactly through the face: terminate only
    # within a negligible distance of it (the discrete replica keeps tau_term)
    step = _step(step)
    step.tau_term = 1e-9 * ds0
    out = dict(disp=np.empty((n, 2)), exit_pos=np.empty((n, 3)), exit_dir=np.empty((n, 3)),
               levels=np.empty(n, np.int32), converged=np.empty(n, np.uint8))
    rc = lib().ho_reference_views(medium.ref, _views(views), len(views), C.byref(step), float(ds0),
                                  int(max_levels), float(tol_px), float(tol_dir),
                                  None if ids is None else _ptr(ids), n, _ptr(out["disp"]), _ptr(out["exit_pos"]),
                                  _ptr(out["exit_dir"]), _ptr(out["levels"]), _ptr(out["converged"]))
    if rc != 0:
        raise ValueError(f"oracle reference failed ({rc})")
    return out
