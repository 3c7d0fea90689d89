"""Depth law of the angle-of-arrival variance on the GPU tracer (Sec. 4.2, Eq. 19).

Workload: statistically homogeneous synthetic turbulence (von Karman
spectrum, outer scale 0.1 m, inner scale 3 voxels, RMS delta-n 1e-5) on a
128^3 grid over 1 m^3; 4096 narrow pinhole cameras at seeded positions just in
front of the y = 0 face, looking +y; scene boards inside the volume.  The
variances of the arrival angles measured through hz_trace_scene are compared
with the first-order predictions of `oracle.aoa` for the same field:

  * boards at four depths: every variance matches the prediction for the
    traced scheme, and the variance grows linearly with depth with one third
    of the plane-wave tilt rate (pinhole form of Eq. 19);
  * the paper's two settings, two boards at different depths and one slanted
    board, give the variances their hit depths predict;
  * cameras with an aperture (averaging the arrival angle over aperture
    points) reproduce the aperture-filtered weighting whose Kolmogorov limit is
    Eq. 19's 3/8;
  * per-ray parity with the oracle on a subset.
"""
import time

import numpy as np
import pytest
import torch

import oracle
from oracle import aoa
from paper_2603_02048_amd import workloads as W
from tests import aoa_experiment as X
from tests.parity import assert_rays_match, to_np

pytestmark = pytest.mark.gpu

RES = 128
WIDTH, VFOV = 8, 4.0


@pytest.fixture(scope="module")
def haze():
    from paper_2603_02048_amd import haze as h
    h.lib()
    return h


@pytest.fixture(scope="module")
def setup(haze):
    grid = W.make_grid((0, 0, 0), (1, 1, 1), (RES, RES, RES))
    dn = W.turbulence_field(grid, rms=1e-5, outer=0.1, inner=3 * grid.voxel, seed=0)
    ctx = haze.Context(0)
    field = ctx.index_field_from_grid(torch.from_numpy(dn.astype(np.float32)).cuda(), grid)
    dn32 = dn.astype(np.float32).astype(np.float64)
    yield dict(grid=grid, dn=dn32, ctx=ctx, field=field)
    field.release()
    ctx.close()


def _dirs(views, width):
    pix = np.stack([np.tile(np.arange(width), width), np.repeat(np.arange(width), width)], 1)
    return oracle.pixel_rays(views[0], pix)


def _trace(S, views, quads, st):
    t0 = time.perf_counter()
    out = S["ctx"].trace_scene(S["field"], views, quads, st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return to_np(out), dt


def test_depth_law_boards(setup):
    S = setup
    grid, dn = S["grid"], S["dn"]
    views = X.random_eye_views(grid, 4096, WIDTH, VFOV, seed=1)
    dirs = _dirs(views, WIDTH)
    depths = [0.25, 0.5, 0.75, 0.98]
    st_a, st_u = W.make_steps(grid)
    st_f = W.make_steps(grid, uniform_vox=0.125)[1]
    for st, ds, label in ((st_a, st_a.ds_max, "adaptive (1 voxel)"), (st_f, st_f.ds_uniform, "uniform 1/8 voxel")):
        meas = {k: [] for k in ("point_x", "point_z", "plane_x", "plane_z")}
        for L in depths:
            out, dt = _trace(S, views, W.quads([X.board_at(L)]), st)
            assert np.all(out["surface"] == 1) and np.all(out["status"] == 0)
            a = X.angles(out, views, WIDTH, VFOV, dirs)
            for k in meas:
                meas[k].append(float(np.var(a[k])))
            print(f"aoa {label} L={L}: {out['steps'].sum() / dt / 1e9:.2f} G ray-steps/s incl. sync", flush=True)
        for comp, ax in ((0, "x"), (2, "z")):
            lv = aoa.line_variances(dn, grid, comp, depths, X.STANDOFF, ds=ds)
            for kind in ("point", "plane"):
                ratio = np.array(meas[f"{kind}_{ax}"]) / lv[kind]
                print(f"aoa {label} {kind}_{ax}: measured/predicted {np.round(ratio, 3).tolist()}", flush=True)
                assert np.all(np.abs(ratio - 1) < 0.1), (label, kind, ax, ratio)
            if ds < grid.voxel / 4:
                # continuum law: linear in depth, slope T/3, through the origin
                T = float(np.sum(aoa.tilt_spectrum(dn, grid, comp)[2]))
                slope, icpt = np.polyfit(depths, meas[f"point_{ax}"], 1)
                print(f"aoa point_{ax}: slope {slope:.4e} vs T/3 {T / 3:.4e}, intercept {icpt:.2e}; "
                      f"point/plane at L=0.98 {meas[f'point_{ax}'][-1] / meas[f'plane_{ax}'][-1]:.3f}", flush=True)
                assert abs(slope / (T / 3) - 1) < 0.12
                assert abs(icpt) < 0.1 * slope
                assert abs(meas[f"point_{ax}"][-1] / meas[f"plane_{ax}"][-1] * 3 - 1) < 0.12


def test_depth_law_two_boards_and_slanted_board(setup):
    S = setup
    grid, dn = S["grid"], S["dn"]
    views = X.random_eye_views(grid, 4096, WIDTH, VFOV, seed=2)
    dirs = _dirs(views, WIDTH)
    st = W.make_steps(grid)[0]
    ds = st.ds_max
    L1, L2 = 0.45, 0.95
    # near board over the lower half of the face, far board behind everything
    two = W.quads([X.board_at(L1, z_range=(-1.0, 0.5)), X.board_at(L2)])
    out, _ = _trace(S, views, two, st)
    a = X.angles(out, views, WIDTH, VFOV, dirs)
    surf = out["surface"].reshape(len(views), -1)
    for comp, ax in ((0, "x"), (2, "z")):
        lv = aoa.line_variances(dn, grid, comp, [L1, L2], X.STANDOFF, ds=ds)
        v1 = np.var(a[f"point_{ax}"][surf == 1])
        v2 = np.var(a[f"point_{ax}"][surf == 2])
        print(f"aoa two boards {ax}: near {v1 / lv['point'][0]:.3f}, far {v2 / lv['point'][1]:.3f} of predicted; "
              f"far/near {v2 / v1:.3f} (predicted {lv['point'][1] / lv['point'][0]:.3f})", flush=True)
        assert (surf == 1).sum() > 50_000 and (surf == 2).sum() > 50_000
        assert abs(v1 / lv["point"][0] - 1) < 0.12 and abs(v2 / lv["point"][1] - 1) < 0.12
        assert abs((v2 / v1) / (lv["point"][1] / lv["point"][0]) - 1) < 0.15
    # slanted board: depth rises from 0.2 m at x = 0 to 0.95 m at x = 1, so
    # each depth bin sees only a band of x, a slab of one realization; three
    # field realizations are pooled
    slant = W.quads([((-1.0, 0.2 - 0.75, -1.0), (3.0, 2.25, 0.0), (0.0, 0.0, 3.0))])
    grid_d = np.linspace(0.15, 1.0, 35)
    edges = np.linspace(0.25, 0.9, 6)
    acc = {ax: [[] for _ in range(5)] for ax in ("x", "z")}
    for real in range(3):
        if real == 0:
            f, dn_r = S["field"], dn
        else:
            dn_r = W.turbulence_field(grid, rms=1e-5, outer=0.1, inner=3 * grid.voxel, seed=real)
            dn_r = dn_r.astype(np.float32).astype(np.float64)
            f = S["ctx"].index_field_from_grid(torch.from_numpy(dn_r.astype(np.float32)).cuda(), grid)
        vs = views if real == 0 else X.random_eye_views(grid, 4096, WIDTH, VFOV, seed=2 + real)
        out = to_np(S["ctx"].trace_scene(f, vs, slant, st))
        torch.cuda.synchronize()
        assert np.all(out["surface"] == 1)
        a = X.angles(out, vs, WIDTH, VFOV, dirs)
        depth = out["exit_pos"][:, 1].astype(np.float64)
        for comp, ax in ((0, "x"), (2, "z")):
            pred_ray = np.interp(depth, grid_d, aoa.line_variances(dn_r, grid, comp, grid_d, X.STANDOFF, ds=ds)["point"])
            vals_all = a[f"point_{ax}"].ravel()
            for b, (lo_, hi_) in enumerate(zip(edges[:-1], edges[1:])):
                m = (depth >= lo_) & (depth < hi_)
                acc[ax][b].append((vals_all[m], pred_ray[m], depth[m]))
        if real > 0:
            f.release()
    for ax in ("x", "z"):
        meas, pred, mid = [], [], []
        for b in range(5):
            vals = np.concatenate([p[0] for p in acc[ax][b]])
            meas.append(np.mean(vals * vals) - np.mean(vals) ** 2)
            pred.append(np.mean(np.concatenate([p[1] for p in acc[ax][b]])))
            mid.append(np.mean(np.concatenate([p[2] for p in acc[ax][b]])))
        ratio = np.array(meas) / np.array(pred)
        slope, icpt = np.polyfit(mid, meas, 1)
        pslope, _ = np.polyfit(mid, pred, 1)
        print(f"aoa slanted {ax}: bins at {np.round(mid, 3).tolist()} measured/predicted {np.round(ratio, 3).tolist()}; "
              f"slope {slope:.3e} vs {pslope:.3e}", flush=True)
        assert np.all(np.abs(ratio - 1) < 0.15), ratio
        assert abs(slope / pslope - 1) < 0.15
    # a subset of the rays against the oracle, ray by ray
    md = oracle.Medium.from_grid(grid, dn)
    sub = views[:48]
    g, _ = _trace(S, sub, slant, st)
    ref = oracle.trace_scene(md, sub, slant, st)
    assert np.array_equal(g["surface"], ref["surface"])
    assert_rays_match({k: v for k, v in g.items() if k != "surface"},
                      {k: v for k, v in ref.items() if k != "surface"}, grid.voxel, "aoa slanted subset")


def test_aperture_weighting(setup):
    S = setup
    grid, dn = S["grid"], S["dn"]
    width, vfov = 48, 6.0
    f = X.focal_px(width, vfov)
    L = 0.98
    Lp = L + X.STANDOFF
    st = W.make_steps(grid, uniform_vox=0.125)[1]
    board = W.quads([X.board_at(L)])
    spec = aoa.tilt_spectrum(dn, grid, 0)
    results = {}
    for D in (0.0, 0.02, 0.04):
        offs = X.disk_offsets(D, Lp / f) if D > 0 else [(0, 0)]
        point, plane = [], []
        n_sites = 4096 // len(offs)
        for seed in range(4):
            views = X.random_eye_views(grid, n_sites, width, vfov, seed=10 + seed, margin=0.1, offsets=offs,
                                       fpx_scale=Lp / f)
            out, _ = _trace(S, views, board, st)
            a = X.angles(out, views, width, vfov, _dirs(views, width))
            point.append(X.aperture_average(a["point_x"].reshape(n_sites, len(offs), -1), offs, width, True))
            plane.append(X.aperture_average(a["plane_x"].reshape(n_sites, len(offs), -1), offs, width, False))
        vp, vw = np.var(np.concatenate(point)), np.var(np.concatenate(plane))
        off_m = np.array(offs, np.float64) * Lp / f
        pr = aoa.predicted_variances(spec, off_m, L)
        results[D] = (vp / vw, pr["ratio"])
        print(f"aoa aperture D={D}: {len(offs)} points, point/plane {vp / vw:.3f} (predicted {pr['ratio']:.3f}); "
              f"plane {vw / pr['plane']:.3f}, point {vp / pr['point']:.3f} of predicted", flush=True)
        assert abs((vp / vw) / pr["ratio"] - 1) < 0.12
    # the aperture raises the ratio above the pinhole's 1/3, as predicted
    assert results[0.0][1] < results[0.02][1] < results[0.04][1]
    assert results[0.0][0] < results[0.02][0] < results[0.04][0]
