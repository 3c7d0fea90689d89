"""Angle-of-arrival statistics of the traced field -- TEST INFRASTRUCTURE ONLY.

The paper (Sec. 4.2, Eq. 19) checks its simulator against the depth law of
the angle-of-arrival variance: for turbulence of constant strength along the
path, the variance of the apparent direction of a scene point at distance L
grows linearly with L,

    <alpha^2> = K^2 int_0^L (z / L)^{5/3} dz = (3/8) K^2 L,

where K^2 L is the variance of a plane wave's tilt over the same path and
aperture, and z is measured from the scene point.  The exponent 5/3 is the
lever arm squared, (z/L)^2, times the aperture filter of a Kolmogorov
spectrum, (z/L)^{-1/3}: at distance z from the point the rays that reach an
aperture of diameter D span only D z / L.

This module states that law for a gridded field and an arbitrary aperture, in
the first-order (weak deflection) and Markov (path much longer than the
correlation length) approximations:

    plane wave:  <a^2> = L sum_k S(k) |A(k)|^2
    point at L:  <a^2> = L int_0^1 u^2 sum_k S(k) |A(u k)|^2 du

with u = z / L, S(k) the transverse spectrum of the depth-averaged gradient
component (the Markov slice k_depth = 0), and A(k) the mean of exp(i k . e)
over the aperture points e.  With a single aperture point (a pinhole camera,
as the paper's renderer and this tracer use) A = 1 and the ratio of the two
is 1/3 for any spectrum; if sum_k S |A(s k)|^2 falls as s^{-1/3} (Kolmogorov,
inner scale << D << outer scale) the ratio is 3/8, Eq. 19's constant.

S(k) includes what the tracer's sampling does to the spectrum: the gradient is
the finite difference of Eq. 13 on the grid, and a ray at a random transverse
position sees its bilinear interpolation, whose mean power per mode is
prod_a (2 + cos(k_a h_a)) / 3 (the mean over t in [0, 1] of the squared linear
interpolation weights of a mode).
"""
from __future__ import annotations

import numpy as np

from . import gradient


def _u_rule(n: int):
    """Nodes u and weights for int_0^1 h(u) du with h ~ u^2 times a power of u
    down to u^{-1/3}: Gauss-Legendre in v = u^{1/3} (du = 3 v^2 dv), exact for
    h = u^2."""
    x, w = np.polynomial.legendre.leggauss(n)
    v = 0.5 * (x + 1.0)
    return v ** 3, 0.5 * w * 3.0 * v * v


def weighting_ratio(F, n: int = 64) -> float:
    """int_0^1 u^2 F(u) du / F(1): the point-source to plane-wave variance
    ratio when the aperture-filtered tilt power at scale u D is F(u).
    F = 1 gives 1/3, F = u^{-1/3} gives Eq. 19's 3/8."""
    u, wt = _u_rule(n)
    return float(np.sum(wt * u * u * np.array([F(x) for x in u])) / F(1.0))


def tilt_spectrum(dn: np.ndarray, grid, component: int, depth_axis: int = 1):
    """Transverse spectrum S(k) of the depth-averaged gradient component
    `component` (0: x, 2: z) of the gridded field, for rays along the y axis.
    Returns (kx, kz, S) with S summing to the plane-wave tilt variance per
    metre of path, T = sum S."""
    if depth_axis != 1:
        raise ValueError("rays along y only")
    g = gradient(dn, grid)[component]                  # [z][y][x]
    gbar = g.mean(axis=1)                              # [z][x], the k_y = 0 slice
    sp = grid.spacing
    depth = float(grid.hi[1] - grid.lo[1])
    F = np.fft.fft2(gbar - gbar.mean())
    P = np.abs(F) ** 2 / float(gbar.size) ** 2
    kz = 2 * np.pi * np.fft.fftfreq(gbar.shape[0], sp[2])
    kx = 2 * np.pi * np.fft.fftfreq(gbar.shape[1], sp[0])
    interp = ((2 + np.cos(kz * sp[2])) / 3)[:, None] * ((2 + np.cos(kx * sp[0])) / 3)[None, :]
    return kx[None, :], kz[:, None], depth * P * interp


def line_weights(grid, L: float, standoff: float, kind: str, sub: int = 64, ds: float = 0.0) -> np.ndarray:
    """Weights c_j with int_{lo_y}^{L} w(y) g~(y) dy = sum_j c_j g_j, where g~
    is the tracer's linear interpolation along y of the samples g_j at the
    voxel centres (cell index clamped to [0, R - 2], so the outer half voxels
    extrapolate, Sec. 3.3.1) and w is the lever weight of the arrival angle:
        kind 'plane': w = 1
        kind 'point': w = 1 - (y - lo_y + standoff) / (L - lo_y + standoff)
    (eye `standoff` before the y = lo_y face, scene point at depth L).

    ds = 0: the continuous ray equation; midpoint rule on `sub` points per
    voxel, exact for this piecewise quadratic integrand up to O(sub^-2) at
    the cell breaks.  ds > 0: the explicit update of Eq. 16 with fixed steps
    ds from the face: the turn ds g(y_k) taken at y_k = lo_y + k ds (every k
    with y_k < L; the board is met on the chord of the last one) acts with
    the lever from y_k itself, since the position update uses the new
    direction."""
    h = float(grid.spacing[1])
    y0 = float(grid.lo[1])
    R = int(grid.res[1])
    if ds > 0.0:
        y = y0 + np.arange(int(np.ceil((L - y0) / ds))) * ds
        y = y[y < L]
        dy = ds
    else:
        m = max(1, int(np.ceil((L - y0) / h * sub)))
        dy = (L - y0) / m
        y = y0 + (np.arange(m) + 0.5) * dy
    if kind == "plane":
        w = np.ones(y.shape)
    elif kind == "point":
        w = 1.0 - (y - y0 + standoff) / (L - y0 + standoff)
    else:
        raise ValueError(kind)
    u = (y - y0) / h - 0.5
    i = np.clip(np.floor(u), 0, R - 2).astype(np.int64)
    t = u - i
    c = np.zeros(R)
    np.add.at(c, i, w * (1.0 - t) * dy)
    np.add.at(c, i + 1, w * t * dy)
    return c


def line_variances(dn: np.ndarray, grid, component: int, depths, standoff: float, ds: float = 0.0) -> dict:
    """First-order variances, over rays parallel to y at uniformly random
    transverse positions, of the pinhole arrival angle of a scene point at
    depth L ('point') and of the plane-wave tilt over the same path
    ('plane'), for the gridded gradient component of this field as the tracer
    samples it (linear along y with the clamped ends, bilinear across).  No
    Markov approximation: the path weights act on the samples directly, so
    finite path lengths are exact to first order in the deflection.  ds > 0:
    the discrete scheme with fixed steps ds (see line_weights).  Returns
    arrays over `depths`."""
    g = gradient(dn, grid)[component]                         # [z][y][x]
    sp = grid.spacing
    Gh = np.fft.fft2(g, axes=(0, 2)) / float(g.shape[0] * g.shape[2])   # per y layer, coefficients of exp(i k.r)
    Gh[0, :, 0] = 0.0                                         # the transverse mean does not vary between rays
    kz = 2 * np.pi * np.fft.fftfreq(g.shape[0], sp[2])
    kx = 2 * np.pi * np.fft.fftfreq(g.shape[2], sp[0])
    interp = ((2 + np.cos(kz * sp[2])) / 3)[:, None] * ((2 + np.cos(kx * sp[0])) / 3)[None, :]
    out = dict(point=[], plane=[])
    for L in depths:
        for key in out:
            c = line_weights(grid, L, standoff, key, ds=ds)
            line = np.tensordot(Gh, c, axes=([1], [0]))           # [kz][kx]
            out[key].append(float(np.sum(interp * np.abs(line) ** 2)))
    return {k: np.array(v) for k, v in out.items()}


def aperture_power(kx, kz, offsets: np.ndarray, u: float = 1.0) -> np.ndarray:
    """|mean_e exp(i u k . e)|^2 over aperture offsets e = (x, z) in metres."""
    off = np.asarray(offsets, np.float64).reshape(-1, 2)
    ph = np.zeros(np.broadcast(kx, kz).shape, np.complex128)
    for ex, ez in off:
        ph += np.exp(1j * u * (kx * ex + kz * ez))
    return np.abs(ph / off.shape[0]) ** 2


def predicted_variances(spectrum, offsets, L: float, n: int = 48) -> dict:
    """Plane-wave and point-source (scene point at distance L) variances of
    the aperture-averaged arrival angle, one transverse component (Markov
    approximation)."""
    kx, kz, S = spectrum
    plane = L * float(np.sum(S * aperture_power(kx, kz, offsets, 1.0)))
    u, wt = _u_rule(n)
    pts = np.array([np.sum(S * aperture_power(kx, kz, offsets, x)) for x in u])
    point = L * float(np.sum(wt * u * u * pts))
    return dict(plane=plane, point=point, ratio=point / plane, T=float(np.sum(S)))
