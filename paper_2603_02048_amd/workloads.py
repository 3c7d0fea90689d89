"""Seeded synthetic inputs for the splat-and-trace path.

This module only *draws* inputs: particle positions and masses shaped like
heat plumes, pinhole camera poses with a backdrop plane, step-control
settings and random ray subsets.  It holds none of the method's arithmetic
(no smoothing kernel, no refractive index, no gradient, no ray integration),
so the FP64 oracle and the HIP path can both consume its bytes without
sharing any of the computation they are compared on.

Particle state follows the paper's per-particle record (Sec. 3.1, Eq. 1);
only mass and position are consumed downstream.  The thermofluid solver that
would produce them (Sec. 3.1-3.2) is replaced by a closed-form temperature
law: T = 300 K + sum_p dT_p exp(-r_p^2 / (2 sigma_p^2)), r_p the horizontal
distance to plume p's vertical axis, density rho = 1.2 * 300 / T kg/m^3 and
mass m = rho * V_box / N, so that m / rho is each particle's volume.

Random numbers come from numpy's PCG64 (`numpy.random.default_rng(seed)`),
drawn in a fixed order: positions, then plume parameters; ray subsets use
`default_rng(seed + 1)`.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

# Gladstone-Dale constant of air used by every workload (Sec. 3.3.1, Eq. 12);
# the paper does not print its value, 2.26e-4 m^3/kg is the textbook one.
K_GD_AIR = 2.26e-4
# Smoothing length of the cubic-spline splat (support 2h).
H_SPLAT = 0.04
# Step statuses reported per ray.
STATUS_OK, STATUS_MAXSTEPS, STATUS_NOHIT, STATUS_NONFINITE = 0, 1, 2, 3


@dataclass
class Grid:
    """Regular voxel grid; voxel centres at lo + (i + 1/2) * (hi - lo) / res."""
    lo: np.ndarray          # (3,) float64, metres
    hi: np.ndarray          # (3,) float64
    res: np.ndarray         # (3,) int32, (Rx, Ry, Rz)

    @property
    def spacing(self) -> np.ndarray:
        return (self.hi - self.lo) / self.res

    @property
    def voxel(self) -> float:
        """Length unit of step control and tolerances: the smallest spacing."""
        return float(np.min(self.spacing))

    @property
    def nvox(self) -> int:
        return int(np.prod(self.res))


@dataclass
class Particles:
    x: np.ndarray           # (N,) float32
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray           # (N,) float32, kg

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class View:
    """Pinhole camera plus the backdrop plane its rays land on (float32)."""
    eye: np.ndarray         # (3,) float32
    fwd: np.ndarray         # (3,) float32, unit
    up: np.ndarray          # (3,) float32
    vfov: float             # radians (stored as float32 value)
    width: int
    height: int
    plane_p: np.ndarray     # (3,) float32, a point of the backdrop plane
    plane_n: np.ndarray     # (3,) float32, unit normal facing the camera

    @property
    def nrays(self) -> int:
        return self.width * self.height


@dataclass
class Step:
    """Step control (Sec. 3.3.3, Eq. 18; fixed-step variant Sec. 4.1). Lengths in metres."""
    uniform: int
    theta_max: float
    ds_min: float
    ds_max: float
    eps: float
    ds_uniform: float
    max_steps: int
    tau_term: float


@dataclass
class Workload:
    name: str
    particles: Particles
    grid: Grid
    k_gd: float
    h: float
    views: List[View]
    step_adaptive: Step
    step_uniform: Step
    subset: Optional[np.ndarray] = None     # int64 global ray ids (sorted)
    meta: dict = field(default_factory=dict)

    @property
    def nrays(self) -> int:
        return sum(v.nrays for v in self.views)

    def with_k_gd(self, factor: float) -> "Workload":
        """Stress variant: same particles, Gladstone-Dale constant scaled."""
        return dataclasses.replace(self, name=f"{self.name}_kgd_x{factor:g}",
                                   k_gd=self.k_gd * factor)


def _f32(v) -> np.ndarray:
    return np.asarray(v, dtype=np.float64).astype(np.float32)


def plume_particles(rng: np.random.Generator, n: int, lo, hi, plumes) -> Particles:
    """i.i.d. uniform positions in the box; masses from the plume temperature law.

    `plumes` is a sequence of (cx, cy, dT, sigma): vertical axes through (cx, cy).
    """
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    pos = lo + rng.random((n, 3)) * (hi - lo)
    return _particles_from_positions(pos, lo, hi, plumes)


def _axis_exit(eye, fwd, lo, hi) -> np.ndarray:
    """Point where the line eye + t*fwd leaves the box (scene set-up only)."""
    t_out = math.inf
    for a in range(3):
        if fwd[a] > 0:
            t_out = min(t_out, (hi[a] - eye[a]) / fwd[a])
        elif fwd[a] < 0:
            t_out = min(t_out, (lo[a] - eye[a]) / fwd[a])
    return eye + t_out * fwd


def ring_view(lo, hi, azimuth: float, radius: float, width: int, height: int,
              vfov_deg: float = 40.0, backdrop_beyond: float = 2.0,
              elevation: float = 0.0) -> View:
    """Camera on a horizontal ring around the box's vertical axis, looking at the box centre.

    Azimuth 0 puts the camera on the -y side looking +y; up is +z.  The
    backdrop plane is perpendicular to the optical axis, `backdrop_beyond`
    metres past the point where that axis leaves the box, normal facing the
    camera.
    """
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    c = 0.5 * (lo + hi)
    eye = c + np.array([radius * math.sin(azimuth), -radius * math.cos(azimuth), elevation])
    fwd = c - eye
    fwd /= np.linalg.norm(fwd)
    exit_pt = _axis_exit(eye, fwd, lo, hi)
    plane_p = exit_pt + backdrop_beyond * fwd
    return View(eye=_f32(eye), fwd=_f32(fwd), up=_f32([0.0, 0.0, 1.0]),
                vfov=float(np.float32(math.radians(vfov_deg))), width=int(width), height=int(height),
                plane_p=_f32(plane_p), plane_n=_f32(-fwd))


def quads(items) -> np.ndarray:
    """Scene boards as a (K, 3, 3) float32 array of (origin, edge_u, edge_v):
    each is the parallelogram origin + u edge_u + v edge_v, 0 <= u, v <= 1."""
    a = np.asarray(items, np.float64).reshape(-1, 3, 3)
    return a.astype(np.float32)


def make_steps(grid: Grid, theta_max: float = 0.003, h_max_vox: float = 1.0,
               h_min_vox: float = 1.0 / 64.0, uniform_vox: float = 0.25,
               eps: float = 1e-12, max_steps: int = 1 << 20) -> tuple:
    """Adaptive (Eq. 18) and fixed-step settings in metres from voxel units."""
    vox = grid.voxel
    common = dict(theta_max=float(np.float32(theta_max)), ds_min=float(np.float32(h_min_vox * vox)),
                  ds_max=float(np.float32(h_max_vox * vox)), eps=float(np.float32(eps)),
                  ds_uniform=float(np.float32(uniform_vox * vox)), max_steps=int(max_steps),
                  tau_term=float(np.float32(1e-4 * vox)))
    return Step(uniform=0, **common), Step(uniform=1, **common)


def draw_subset(total: int, size: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed + 1)
    size = min(size, total)
    return np.sort(rng.choice(total, size=size, replace=False)).astype(np.int64)


def make_grid(lo, hi, res) -> Grid:
    return Grid(lo=np.asarray(lo, np.float64), hi=np.asarray(hi, np.float64),
                res=np.asarray(res, np.int32))


def make_config(index: int, seed: int = 0, subset_size: Optional[int] = None) -> Workload:
    """The five workload configurations (1-based index).

    1: 16,384 particles in [0,1]^3, one plume, 64^3 grid, one 128x128 view.
    2: 262,144 particles in [0,1]x[0,1]x[0,2], main plume + 3 random plumes,
       128^3 grid, one 1280x720 view, 4,096-ray subset.
    3: configuration 2's field seen by 8 views on a 3 m ring (45 deg apart).
    4: 1,048,576 particles in [0,2]^3, 16 random plumes, 256^3, 4 views 1920x1080.
    5: configuration 4's particle set (the serving sequence advects it).
    """
    rng = np.random.default_rng(seed)
    if index == 1:
        lo, hi, res, n = (0, 0, 0), (1, 1, 1), (64, 64, 64), 16384
        plumes = [(0.5, 0.5, 60.0, 0.1)]
        parts = plume_particles(rng, n, lo, hi, plumes)
        views = [ring_view(lo, hi, 0.0, 3.0, 128, 128)]
        sub = subset_size
    elif index in (2, 3):
        lo, hi, res, n = (0, 0, 0), (1, 1, 2), (128, 128, 128), 262144
        # positions first, then plume parameters (fixed draw order)
        pos = lo + rng.random((n, 3)) * (np.asarray(hi, float) - np.asarray(lo, float))
        extra = [(rng.uniform(0, 1), rng.uniform(0, 1), rng.uniform(20, 80), 0.1) for _ in range(3)]
        plumes = [(0.5, 0.5, 60.0, 0.1)] + extra
        parts = _particles_from_positions(pos, lo, hi, plumes)
        if index == 2:
            views = [ring_view(lo, hi, 0.0, 3.0, 1280, 720)]
        else:
            views = [ring_view(lo, hi, math.radians(45.0 * k), 3.0, 1280, 720) for k in range(8)]
        sub = 4096 if subset_size is None else subset_size
    elif index in (4, 5):
        lo, hi, res, n = (0, 0, 0), (2, 2, 2), (256, 256, 256), 1048576
        pos = lo + rng.random((n, 3)) * (np.asarray(hi, float) - np.asarray(lo, float))
        plumes = [(rng.uniform(0, 2), rng.uniform(0, 2), rng.uniform(10, 100), rng.uniform(0.05, 0.3))
                  for _ in range(16)]
        parts = _particles_from_positions(pos, lo, hi, plumes)
        views = [ring_view(lo, hi, math.radians(90.0 * k), 3.0, 1920, 1080) for k in range(4)]
        sub = 16384 if subset_size is None else subset_size
    else:
        raise ValueError(f"unknown configuration {index}")
    grid = make_grid(lo, hi, res)
    st_a, st_u = make_steps(grid)
    wl = Workload(name=f"config{index}", particles=parts, grid=grid, k_gd=K_GD_AIR, h=H_SPLAT,
                  views=views, step_adaptive=st_a, step_uniform=st_u,
                  meta=dict(seed=seed, plumes=plumes))
    if sub is not None:
        wl.subset = draw_subset(wl.nrays, sub, seed)
    return wl


def _particles_from_positions(pos: np.ndarray, lo, hi, plumes) -> Particles:
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    n = pos.shape[0]
    pos32 = pos.astype(np.float32)
    p = pos32.astype(np.float64)
    temp = np.full(n, 300.0)
    for cx, cy, dt, sig in plumes:
        r2 = (p[:, 0] - cx) ** 2 + (p[:, 1] - cy) ** 2
        temp += dt * np.exp(-r2 / (2.0 * sig * sig))
    rho = 1.2 * 300.0 / temp
    m = (rho * float(np.prod(hi - lo)) / n).astype(np.float32)
    return Particles(x=np.ascontiguousarray(pos32[:, 0]), y=np.ascontiguousarray(pos32[:, 1]),
                     z=np.ascontiguousarray(pos32[:, 2]), m=m)


def make_small(seed: int = 0, n: int = 3000, lo=(0.0, 0.0, 0.0), hi=(0.5, 0.4, 0.3),
               res=(21, 17, 13), h: float = 0.03, width: int = 37, height: int = 23,
               nviews: int = 2, k_gd: float = K_GD_AIR, radius: float = 1.2,
               vfov_deg: float = 40.0) -> Workload:
    """A ragged small case: odd grid sizes, odd image sizes, views on a ring."""
    rng = np.random.default_rng(seed)
    pos = np.asarray(lo) + rng.random((n, 3)) * (np.asarray(hi) - np.asarray(lo))
    c = 0.5 * (np.asarray(lo) + np.asarray(hi))
    plumes = [(c[0], c[1], 60.0, 0.05), (rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]),
                                         rng.uniform(20, 80), 0.04)]
    parts = _particles_from_positions(pos, lo, hi, plumes)
    grid = make_grid(lo, hi, res)
    views = [ring_view(lo, hi, math.radians(360.0 / max(nviews, 1) * k + 10.0), radius, width, height,
                       vfov_deg=vfov_deg, backdrop_beyond=0.7, elevation=0.05 * k)
             for k in range(nviews)]
    st_a, st_u = make_steps(grid)
    return Workload(name="small", particles=parts, grid=grid, k_gd=k_gd, h=h, views=views,
                    step_adaptive=st_a, step_uniform=st_u, meta=dict(seed=seed, plumes=plumes))


def voxel_centres(grid: Grid) -> tuple:
    """Voxel-centre coordinate vectors (x, y, z), float64 (scene set-up helper)."""
    sp = grid.spacing
    return tuple(grid.lo[a] + (np.arange(grid.res[a]) + 0.5) * sp[a] for a in range(3))


def analytic_grid_linear(grid: Grid, a0: float, b: Sequence[float]) -> np.ndarray:
    """delta-n sampled at voxel centres from a0 + b . x (array [z][y][x], float64)."""
    cx, cy, cz = voxel_centres(grid)
    return (a0 + b[0] * cx[None, None, :] + b[1] * cy[None, :, None] + b[2] * cz[:, None, None])


def analytic_grid_gauss(grid: Grid, amp: float, centre: Sequence[float], sigma: float) -> np.ndarray:
    """delta-n sampled at voxel centres from amp * exp(-|x - c|^2 / (2 sigma^2))."""
    cx, cy, cz = voxel_centres(grid)
    r2 = ((cx[None, None, :] - centre[0]) ** 2 + (cy[None, :, None] - centre[1]) ** 2
          + (cz[:, None, None] - centre[2]) ** 2)
    return amp * np.exp(-r2 / (2.0 * sigma * sigma))


# ---------------------------------------------------------------------------
# serving workload: an advected frame sequence and Poisson request arrivals
# ---------------------------------------------------------------------------

def turbulence_field(grid: Grid, rms: float, outer: float, inner: float, seed: int = 0) -> np.ndarray:
    """Statistically homogeneous, isotropic delta-n on the grid (array [z][y][x],
    float64): a Gaussian random field with the von Karman spectrum
        Phi(k) ~ (k^2 + (2 pi / outer)^2)^(-11/6) exp(-k^2 / (5.92 / inner)^2),
    periodic over the box, scaled to the given RMS.  Input for the depth law
    of the angle-of-arrival variance (Sec. 4.2, Eq. 19), which assumes
    constant turbulence strength along the path."""
    res = [int(r) for r in grid.res]
    sp = grid.spacing
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((res[2], res[1], res[0]))
    kz = 2 * np.pi * np.fft.fftfreq(res[2], sp[2])
    ky = 2 * np.pi * np.fft.fftfreq(res[1], sp[1])
    kx = 2 * np.pi * np.fft.rfftfreq(res[0], sp[0])
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    k0, km = 2 * np.pi / outer, 5.92 / inner
    amp = np.sqrt((k2 + k0 * k0) ** (-11.0 / 6.0) * np.exp(-k2 / (km * km)))
    f = np.fft.irfftn(np.fft.rfftn(white) * amp, s=white.shape, axes=(0, 1, 2))
    f -= f.mean()
    return f * (rms / f.std())


def depth_views(lo, hi, n_side: int, width: int, height: int, vfov_deg: float, standoff: float = 0.01,
                backdrop_beyond: float = 1.0) -> list:
    """A square grid of n_side x n_side cameras just in front of the box's
    y = lo face, all looking +y (up +z), spread over the face; the backdrop is
    a plane of constant y beyond the box."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    views = []
    for j in range(n_side):
        for i in range(n_side):
            ex = lo[0] + (i + 0.5) / n_side * (hi[0] - lo[0])
            ez = lo[2] + (j + 0.5) / n_side * (hi[2] - lo[2])
            eye = np.array([ex, lo[1] - standoff, ez])
            views.append(View(eye=_f32(eye), fwd=_f32([0.0, 1.0, 0.0]), up=_f32([0.0, 0.0, 1.0]),
                              vfov=float(np.float32(math.radians(vfov_deg))), width=int(width),
                              height=int(height), plane_p=_f32([ex, hi[1] + backdrop_beyond, ez]),
                              plane_n=_f32([0.0, -1.0, 0.0])))
    return views


class CurlNoise:
    """Seeded divergence-free velocity v(x) = curl A(x), A = sum_m a_m sin(k_m . x + phi_m).

    curl(a sin(k.x + phi)) = cos(k.x + phi) (k x a), so
    v(x) = sum_m cos(k_m . x + phi_m) (k_m x a_m), scaled to the requested RMS speed.
    """

    def __init__(self, rng: np.random.Generator, nmodes: int = 16, wavelength=(0.25, 1.0), rms: float = 0.2):
        lam = rng.uniform(wavelength[0], wavelength[1], nmodes)
        dirs = rng.standard_normal((nmodes, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        self.k = dirs * (2.0 * math.pi / lam)[:, None]
        self.a = rng.standard_normal((nmodes, 3))
        self.phi = rng.uniform(0.0, 2.0 * math.pi, nmodes)
        self.ka = np.cross(self.k, self.a)
        # mean of cos^2 is 1/2 over random positions: scale the modes to the RMS speed
        ms = 0.5 * float(np.sum(self.ka ** 2))
        self.ka *= rms / math.sqrt(ms)

    def velocity(self, x: np.ndarray) -> np.ndarray:
        ph = x @ self.k.T + self.phi          # (N, M)
        return np.cos(ph) @ self.ka           # (N, 3)


def advect_frames(particles: Particles, lo, hi, nframes: int = 60, dt: float = 1.0 / 30.0, rms: float = 0.2,
                  seed: int = 0, device=None):
    """Yield `nframes` particle sets: positions advected by seeded curl noise with
    midpoint steps, wrapped periodically into the box; masses travel with the
    particles.  With `device` (a torch device) the arithmetic runs in torch
    float64 there and frames are yielded as numpy float32 as well."""
    rng = np.random.default_rng(seed + 2)
    field = CurlNoise(rng, rms=rms)
    lo64 = np.asarray(lo, np.float64)
    hi64 = np.asarray(hi, np.float64)
    x0 = np.stack([particles.x, particles.y, particles.z], 1).astype(np.float64)
    if device is None:
        xp_cos, x, lo_, ext = np.cos, x0, lo64, hi64 - lo64
        k, phi, ka = field.k, field.phi, field.ka
        to_np = lambda a: a
        mod = np.mod
    else:
        import torch
        t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device)
        xp_cos, x, lo_, ext = torch.cos, t(x0), t(lo64), t(hi64 - lo64)
        k, phi, ka = t(field.k), t(field.phi), t(field.ka)
        to_np = lambda a: a.cpu().numpy()
        mod = torch.remainder
    vel = lambda y: xp_cos(y @ k.T + phi) @ ka
    for f in range(nframes):
        if f > 0:
            mid = x + 0.5 * dt * vel(x)
            x = x + dt * vel(mid)
            x = lo_ + mod(x - lo_, ext)
        x32 = to_np(x).astype(np.float32)
        yield Particles(x=np.ascontiguousarray(x32[:, 0]), y=np.ascontiguousarray(x32[:, 1]),
                        z=np.ascontiguousarray(x32[:, 2]), m=particles.m)


@dataclass
class Request:
    t_arrive: float          # seconds from the start of the run
    frame: int
    views: List[View]


def serving_requests(lo, hi, duration_s: float, rate_hz: float = 200.0, nframes: int = 60, seed: int = 0,
                     resolutions=((640, 360), (1280, 720), (1920, 1080)), radius=(2.5, 5.0),
                     max_views: int = 5) -> List[Request]:
    """Poisson arrivals; each request: a random frame, 1..max_views cameras evenly
    spaced on a ring of random radius and phase, one random resolution."""
    rng = np.random.default_rng(seed + 3)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        frame = int(rng.integers(0, nframes))
        nv = int(rng.integers(1, max_views + 1))
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        rad = float(rng.uniform(radius[0], radius[1]))
        ph = float(rng.uniform(0.0, 2.0 * math.pi))
        views = [ring_view(lo, hi, ph + 2.0 * math.pi * k / nv, rad, w, h) for k in range(nv)]
        out.append(Request(t_arrive=t, frame=frame, views=views))
    return out


def tessellate_quads(quads, n: int = 4):
    """Scene boards as triangle meshes: each parallelogram (origin, edge_u,
    edge_v) cut into n x n cells of two triangles, all of the board's surface
    id (its index).  Returns (T, 3, 3) float64 vertices and (T,) surface ids."""
    tris, surf = [], []
    for k, (o, eu, ev) in enumerate(np.asarray(quads, np.float64)):
        def p(i, j):
            return o + (i / n) * eu + (j / n) * ev
        for i in range(n):
            for j in range(n):
                a, b, c, d = p(i, j), p(i + 1, j), p(i + 1, j + 1), p(i, j + 1)
                tris += [(a, b, c), (a, c, d)]
                surf += [k, k]
    return np.asarray(tris, np.float64), np.asarray(surf, np.int64)


def icosphere(centre, radius: float, subdiv: int = 2):
    """Triangles of a sphere: an icosahedron whose faces are split in four
    `subdiv` times, vertices pushed onto the sphere.  (T, 3, 3) float64."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
         (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    tris = [tuple(np.asarray(v[i], float) / np.linalg.norm(v[i]) for i in face) for face in f]
    for _ in range(subdiv):
        nxt = []
        for a, b, c in tris:
            ab, bc, ca = [(x + y) / np.linalg.norm(x + y) for x, y in ((a, b), (b, c), (c, a))]
            nxt += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        tris = nxt
    return np.asarray(centre, np.float64) + radius * np.asarray(tris, np.float64)
