"""Pins of the angle-of-arrival depth law (Sec. 4.2, Eq. 19) used to check the
tracer on homogeneous synthetic turbulence (CPU only).

  * the weighting integral: int_0^1 u^2 F(u) du / F(1) is 1/3 for a pinhole
    (F = 1) and Eq. 19's 3/8 for a Kolmogorov aperture filter F = u^{-1/3};
  * a single aperture point gives the point-to-plane ratio 1/3 for any spectrum;
  * the bilinear-sampling transfer prod (2 + cos k h) / 3 against a Monte
    Carlo average of interpolated values;
  * the path weights of the tracer's sampling along y are exact for linear
    profiles, and the finite-path variances approach the Markov tilt rate
    over a long path;
  * predictions for the discrete scheme (fixed steps) converge to the
    continuum at first order, and the continuum variance is linear in depth
    with slope T/3;
  * the oracle's own tracer (pinned elsewhere by closed forms) reproduces the
    predicted variances of the discrete scheme and their growth with depth.
"""
import numpy as np
import pytest

from oracle import aoa
from paper_2603_02048_amd import workloads as W
from tests import aoa_experiment as X


def test_weighting_ratio_closed_forms():
    assert abs(aoa.weighting_ratio(lambda u: 1.0) - 1.0 / 3.0) < 1e-6
    assert abs(aoa.weighting_ratio(lambda u: u ** (-1.0 / 3.0)) - 3.0 / 8.0) < 1e-6     # Eq. 19
    for a in (0.5, 1.0, 2.0):
        assert abs(aoa.weighting_ratio(lambda u: u ** (-a)) - 1.0 / (3.0 - a)) < 1e-5


@pytest.fixture(scope="module")
def small_field():
    grid = W.make_grid((0, 0, 0), (1, 1, 1), (64, 64, 64))
    dn = W.turbulence_field(grid, rms=1e-5, outer=0.15, inner=3 * grid.voxel, seed=0)
    return grid, dn


def test_pinhole_ratio_is_one_third(small_field):
    grid, dn = small_field
    spec = aoa.tilt_spectrum(dn, grid, 0)
    r = aoa.predicted_variances(spec, [(0.0, 0.0)], 0.8)
    assert abs(r["ratio"] - 1.0 / 3.0) < 1e-4
    assert abs(r["plane"] - 0.8 * r["T"]) < 1e-12 * r["T"]
    # a finite aperture lowers both variances
    q = aoa.predicted_variances(spec, [(-0.02, 0.0), (0.02, 0.0), (0.0, -0.02), (0.0, 0.02)], 0.8)
    assert q["plane"] < r["plane"] and q["point"] < r["point"]


def test_bilinear_transfer_monte_carlo():
    rng = np.random.default_rng(3)
    nz, nx, hz, hx = 40, 48, 0.02, 0.015
    f = rng.standard_normal((nz, nx))
    f = np.fft.ifft2(np.fft.fft2(f) * np.exp(-0.05 * np.add.outer(np.fft.fftfreq(nz) ** 2 * nz ** 2,
                                                                    np.fft.fftfreq(nx) ** 2 * nx ** 2))).real
    f -= f.mean()
    # mean square of the periodic bilinear interpolant at uniform random points
    n = 2_000_000
    x = rng.uniform(0, nx, n)
    z = rng.uniform(0, nz, n)
    i, k = np.floor(x).astype(int), np.floor(z).astype(int)
    tx, tz = x - i, z - k
    i1, k1 = (i + 1) % nx, (k + 1) % nz
    v = ((1 - tz) * ((1 - tx) * f[k, i] + tx * f[k, i1]) + tz * ((1 - tx) * f[k1, i] + tx * f[k1, i1]))
    mc = np.mean(v * v)
    P = np.abs(np.fft.fft2(f)) ** 2 / f.size ** 2
    kz = 2 * np.pi * np.fft.fftfreq(nz, hz)
    kx = 2 * np.pi * np.fft.fftfreq(nx, hx)
    pred = np.sum(P * ((2 + np.cos(kz * hz)) / 3)[:, None] * ((2 + np.cos(kx * hx)) / 3)[None, :])
    assert abs(mc / pred - 1) < 0.01, (mc, pred)
    assert abs(np.mean(f * f) / pred - 1) > 0.02      # the transfer matters for this field


def test_line_weights_exact_for_linear_profiles():
    # the tracer's linear interpolation (with the clamped, extrapolating ends)
    # is exact for a field linear in y, so the weights integrate 1 and y exactly
    grid = W.make_grid((0, 0.1, 0), (1, 0.9, 1), (8, 23, 8))
    yc = grid.lo[1] + (np.arange(23) + 0.5) * grid.spacing[1]
    for L in (0.1 + 0.013, 0.4, 0.9):
        for kind, wfun in (("plane", lambda y: np.ones_like(y)),
                           ("point", lambda y: 1 - (y - 0.1 + 0.02) / (L - 0.1 + 0.02))):
            c = aoa.line_weights(grid, L, 0.02, kind, sub=256)
            yy = np.linspace(0.1, L, 200001)
            for prof in (np.ones_like, lambda y: y - 0.3):
                exact = np.trapezoid(wfun(yy) * prof(yy), yy)
                assert abs(np.dot(c, prof(yc)) - exact) < 1e-7, (L, kind)


def test_line_variances_markov_limit(small_field):
    # over the full depth of a long periodic box the plane-wave variance
    # approaches the Markov tilt rate times the length
    grid, dn = small_field
    for comp in (0, 2):
        T = float(np.sum(aoa.tilt_spectrum(dn, grid, comp)[2]))
        lv = aoa.line_variances(dn, grid, comp, [1.0], standoff=0.0)
        assert abs(lv["plane"][0] / T - 1) < 0.05, lv["plane"][0] / T
        assert 0.25 < lv["point"][0] / lv["plane"][0] < 0.4


def test_discrete_scheme_weights_converge(small_field):
    # the explicit update's first-order error: predictions for fixed steps ds
    # approach the continuous ray equation linearly in ds
    grid, dn = small_field
    h = grid.spacing[1]
    cont = aoa.line_variances(dn, grid, 0, [0.3, 0.8], 0.01)
    errs = []
    for ds in (h, h / 2, h / 4):
        d = aoa.line_variances(dn, grid, 0, [0.3, 0.8], 0.01, ds=ds)
        errs.append(d["point"] / cont["point"] - 1)
    errs = np.array(errs)
    assert np.all(errs[0] > 0)                    # the new-direction position update over-counts the lever
    ratios = errs[:-1] / errs[1:]
    assert np.all((ratios > 1.6) & (ratios < 2.5)), ratios


def test_continuum_depth_law(small_field):
    # the law itself: the point-source variance grows linearly with depth with
    # one third of the plane-wave tilt rate (pinhole weighting of Eq. 19)
    grid, dn = small_field
    depths = np.array([0.4, 0.55, 0.7, 0.85, 0.99])
    for comp in (0, 2):
        T = float(np.sum(aoa.tilt_spectrum(dn, grid, comp)[2]))
        lv = aoa.line_variances(dn, grid, comp, depths, 0.0)
        slope, icpt = np.polyfit(depths, lv["point"], 1)
        assert abs(slope / (T / 3) - 1) < 0.1, (slope, T / 3)
        assert abs(icpt) < 0.1 * slope
        assert np.max(np.abs(np.polyval((slope, icpt), depths) / lv["point"] - 1)) < 0.03


def test_oracle_tracer_follows_depth_law(oracle_lib, small_field):
    grid, dn = small_field
    md = oracle_lib.Medium.from_grid(grid, dn)
    width, vfov = 8, 4.0
    views = X.random_eye_views(grid, 2048, width, vfov, seed=1)
    pix = np.stack([np.tile(np.arange(width), width), np.repeat(np.arange(width), width)], 1)
    dirs = oracle_lib.pixel_rays(views[0], pix)
    depths = [0.3, 0.6, 0.95]
    st = W.make_steps(grid)[0]           # adaptive; saturates at h_max = 1 voxel on this weak field
    meas = {k: [] for k in ("point_x", "point_z", "plane_x", "plane_z")}
    for L in depths:
        r = oracle_lib.trace_scene(md, views, W.quads([X.board_at(L)]), st)
        assert np.all(r["surface"] == 1)
        a = X.angles(r, views, width, vfov, dirs)
        for k in meas:
            meas[k].append(np.var(a[k]))
    for comp, ax in ((0, "x"), (2, "z")):
        lv = aoa.line_variances(dn, grid, comp, depths, X.STANDOFF, ds=st.ds_max)
        for kind in ("point", "plane"):
            ratio = np.array(meas[f"{kind}_{ax}"]) / lv[kind]
            assert np.all(np.abs(ratio - 1) < 0.1), (kind, ax, ratio)
        # linear in depth
        slope, icpt = np.polyfit(depths, meas[f"point_{ax}"], 1)
        pslope, _ = np.polyfit(depths, lv["point"], 1)
        assert abs(slope / pslope - 1) < 0.1, (slope, pslope)
        assert abs(icpt) < 0.15 * slope
