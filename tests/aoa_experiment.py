"""Depth-law experiment set-up shared by the CPU and GPU tests (Sec. 4.2, Eq. 19).

Cameras sit just in front of the y = 0 face of a box of homogeneous synthetic
turbulence, all looking +y with a narrow field of view; scene boards inside
the volume are perpendicular to y (or slanted).  For each ray the arrival
angle of the board point it sees is the displacement converted to an angle
(the pinhole projection's derivative at that pixel), and the plane-wave tilt
is the change of direction between the pixel ray and the ray where it meets
the board.
"""
import math

import numpy as np

from paper_2603_02048_amd import workloads as W

STANDOFF = 0.01


def random_eye_views(grid, n_eyes: int, width: int, vfov_deg: float, seed: int, margin: float = 0.06,
                     offsets=None, fpx_scale: float = 0.0):
    """n_eyes pinhole cameras at seeded uniform positions over the y = lo face
    (`margin` from its edges), each width x width pixels.  With `offsets`
    (pixel units, (a, b) pairs) every site gets one camera per offset, moved
    by (a, b) * fpx_scale metres along (x, z): an aperture sampled at the
    board distance's pixel footprint."""
    rng = np.random.default_rng(seed)
    lo, hi = np.asarray(grid.lo, np.float64), np.asarray(grid.hi, np.float64)
    xs = rng.uniform(lo[0] + margin, hi[0] - margin, n_eyes)
    zs = rng.uniform(lo[2] + margin, hi[2] - margin, n_eyes)
    offs = [(0, 0)] if offsets is None else list(offsets)
    views = []
    for ex, ez in zip(xs, zs):
        for a, b in offs:
            eye = (ex + a * fpx_scale, lo[1] - STANDOFF, ez + b * fpx_scale)
            views.append(W.View(eye=W._f32(eye), fwd=W._f32([0, 1, 0]), up=W._f32([0, 0, 1]),
                                vfov=float(np.float32(math.radians(vfov_deg))), width=width, height=width,
                                plane_p=W._f32([ex, hi[1] + 1.0, ez]), plane_n=W._f32([0, -1, 0])))
    return views


def focal_px(width: int, vfov_deg: float) -> float:
    return 0.5 * width / math.tan(math.radians(vfov_deg) / 2)


def pixel_offsets(width: int):
    p = np.tile(np.arange(width), width)
    q = np.repeat(np.arange(width), width)
    return p + 0.5 - width / 2, q + 0.5 - width / 2


def board_at(depth: float, x_range=(-1.0, 3.0), z_range=(-1.0, 3.0)):
    return ((x_range[0], depth, z_range[0]), (x_range[1] - x_range[0], 0, 0), (0, 0, z_range[1] - z_range[0]))


def angles(out: dict, views, width: int, vfov_deg: float, pixel_dirs: np.ndarray) -> dict:
    """Per ray: arrival-angle errors (x: image right = +x, z: image up = +z) of
    the board point seen, and the plane-wave tilt (exit minus pixel direction),
    arrays [view][pixel]."""
    f = focal_px(width, vfov_deg)
    sx, sy = pixel_offsets(width)
    nv = len(views)
    disp = np.asarray(out["disp"], np.float64).reshape(nv, width * width, 2)
    ax = disp[..., 0] * f / (f * f + sx * sx)
    az = -disp[..., 1] * f / (f * f + sy * sy)
    dw = np.asarray(out["exit_dir"], np.float64).reshape(nv, width * width, 3) - pixel_dirs[None]
    return dict(point_x=ax, point_z=az, plane_x=dw[..., 0], plane_z=dw[..., 2])


def disk_offsets(diameter: float, footprint: float, target: int = 29):
    """Integer pixel offsets (a, b) on a square lattice inside a disk of the
    given diameter (metres) at `footprint` metres per pixel, about `target`
    of them."""
    r = 0.5 * diameter / footprint
    step = max(1, int(round(r * math.sqrt(math.pi / target))))
    n = int(r // step)
    return [(i * step, j * step) for i in range(-n, n + 1) for j in range(-n, n + 1)
            if (i * step) ** 2 + (j * step) ** 2 <= r * r]


def aperture_average(values: np.ndarray, offsets, width: int, shift: bool) -> np.ndarray:
    """Average over the aperture cameras of one site ([site][offset][pixel]
    array).  shift=True: the rays from every aperture point to the same board
    point (pixel (p - a, q + b) of offset (a, b)); False: parallel rays (same
    pixel).  Only pixels whose partners exist in every camera are kept."""
    m = max(max(abs(a), abs(b)) for a, b in offsets)
    v = values.reshape(values.shape[0], len(offsets), width, width)    # [site][k][q][p]
    acc = np.zeros((values.shape[0], width - 2 * m, width - 2 * m))
    for k, (a, b) in enumerate(offsets):
        if shift:
            acc += v[:, k, m + b:width - m + b, m - a:width - m - a]
        else:
            acc += v[:, k, m:width - m, m:width - m]
    return acc / len(offsets)
