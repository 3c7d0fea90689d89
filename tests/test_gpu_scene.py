"""GPU parity of scene boards (hz_trace_scene) against the FP64 oracle.

The image point of a ray is where it meets the scene (Sec. 3.3.2, last
paragraph); the depth experiments of Sec. 4.2 use boards at two depths or one
slanted board.  Boards are met before the volume, on a step's chord inside it,
or by the straight exit ray.  Which board a ray meets is decided by floating
point near a board's edge; there the oracle is run with every board shrunk
and grown by a small margin, and a ray whose answer differs between the two
is compared only for validity (its surface must be one of the two answers).
Every other ray must match surface, status and the plain tolerances.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_02048_amd import workloads as W
from tests.parity import TOL_DIR, TOL_PX, TOL_POS_VOX, assert_rays_match, ray_errors, summary, to_np

pytestmark = pytest.mark.gpu

MARGIN_VOX = 2e-3


@pytest.fixture(scope="module")
def haze():
    from paper_2603_02048_amd import haze as h
    h.lib()
    return h


@pytest.fixture(scope="module")
def ctx(haze):
    c = haze.Context(0)
    yield c
    c.close()


def _inflate(quads, delta):
    q = np.asarray(quads, np.float64).copy()
    for k in range(q.shape[0]):
        eu, ev = q[k, 1], q[k, 2]
        uh, vh = eu / np.linalg.norm(eu), ev / np.linalg.norm(ev)
        q[k, 0] = q[k, 0] - delta * (uh + vh)
        q[k, 1] = eu + 2 * delta * uh
        q[k, 2] = ev + 2 * delta * vh
    return q


def _boards(lo, hi, which="all"):
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    ext = hi - lo
    inner = [
        # slanted board across the left part of the volume
        (lo + ext * (0.10, 0.25, 0.05), ext * (0.45, 0.50, 0.0), ext * (0.0, 0.0, 0.85)),
        # upright board behind it, right part
        (lo + ext * (0.55, 0.70, 0.10), ext * (0.40, 0.0, 0.0), ext * (0.0, 0.10, 0.80)),
    ]
    outer = [
        # in front of the volume, upper right of the view
        (lo + ext * (0.60, -0.75, 0.55), ext * (0.50, 0.0, 0.0), ext * (0.0, 0.0, 0.60)),
        # beyond the volume, before the backdrop, lower half
        (lo + ext * (-0.30, 1.40, -0.30), ext * (1.60, 0.0, 0.0), ext * (0.0, 0.20, 0.75)),
    ]
    items = {"all": inner + outer, "inner": inner, "outer": outer}[which]
    return W.quads(items)


def _views(lo, hi, n=2, width=37, height=23):
    return [W.ring_view(lo, hi, 0.15 * k - 0.05, 1.1, width, height, backdrop_beyond=0.7, elevation=0.03 * k)
            for k in range(n)]


def _compare(out, md, views, quads, st, voxel, label, ray_ids=None, tol_scale=1.0):
    g = to_np(out)
    ref = oracle.trace_scene(md, views, quads, st, ray_ids=ray_ids)
    lo_ = oracle.trace_scene(md, views, _inflate(quads, -MARGIN_VOX * voxel), st, ray_ids=ray_ids)
    hi_ = oracle.trace_scene(md, views, _inflate(quads, MARGIN_VOX * voxel), st, ray_ids=ray_ids)
    amb = (lo_["surface"] != hi_["surface"]) | (lo_["surface"] != ref["surface"])
    ok_amb = (g["surface"] == lo_["surface"]) | (g["surface"] == hi_["surface"]) | (g["surface"] == ref["surface"])
    print(f"{label}: {amb.sum()} of {amb.size} rays within {MARGIN_VOX} voxel of a board edge; surfaces seen "
          f"{np.bincount(ref['surface'], minlength=256)[[0, 1, 2, 3, 4, 255]].tolist()}", flush=True)
    assert amb.mean() < 0.03, label
    assert ok_amb[amb].all(), label
    keep = ~amb
    assert np.array_equal(g["surface"][keep], ref["surface"][keep]), label
    gk = {k: v[keep] for k, v in g.items() if k != "surface"}
    rk = {k: v[keep] for k, v in ref.items() if k != "surface"}
    if tol_scale == 1.0:
        assert_rays_match(gk, rk, voxel, label)
    else:
        err = ray_errors(gk, rk, voxel)
        msg = f"{label}: {summary(err)}"
        print(msg, flush=True)
        assert err["status_equal"] and err["steps_diff"].max() <= 1, msg
        assert err["pos"].max() <= tol_scale * TOL_POS_VOX and err["dir"].max() <= tol_scale * TOL_DIR, msg
        assert err["px"].max() <= tol_scale * TOL_PX, msg
    return g, ref


@pytest.mark.parametrize("kgd", [1.0, 200.0])
@pytest.mark.parametrize("mode", ["adaptive", "uniform"])
def test_scene_parity_small(ctx, haze, kgd, mode):
    wl = W.make_small(seed=11, width=37, height=23, nviews=1).with_k_gd(kgd)
    print(f"case scene small kgd x{kgd} {mode}", flush=True)
    parts = haze.upload_particles(wl.particles)
    field = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
    md = oracle.field(wl.particles, wl.grid, wl.k_gd, wl.h)
    views = _views(wl.grid.lo, wl.grid.hi)
    quads = _boards(wl.grid.lo, wl.grid.hi)
    st = wl.step_adaptive if mode == "adaptive" else wl.step_uniform
    out = ctx.trace_scene(field, views, quads, st)
    torch.cuda.synchronize()
    g, ref = _compare(out, md, views, quads, st, wl.grid.voxel, f"scene kgd x{kgd} {mode}")
    for k in (0, 1, 2, 3, 4):   # backdrop and every board are seen
        assert (ref["surface"] == k).sum() > 20, k
    inner_hit = (ref["surface"] == 1) | (ref["surface"] == 2)
    assert (g["steps"][inner_hit] > 0).all()
    assert (g["steps"][ref["surface"] == 3] == 0).all()
    field.release()


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_scene_reduced_precision_fields(ctx, haze, dtype):
    # the board tests of every march variant also run on 8-byte F16/BF16 voxels
    wl = W.make_small(seed=15, width=37, height=23, nviews=1)
    print(f"case scene dtype={dtype}", flush=True)
    parts = haze.upload_particles(wl.particles)
    field = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h, dtype=dtype, store_scale=1e4)
    md = oracle.field(wl.particles, wl.grid, wl.k_gd, wl.h)
    views = _views(wl.grid.lo, wl.grid.hi)
    for which in ("all", "outer"):
        quads = _boards(wl.grid.lo, wl.grid.hi, which)
        for st in (wl.step_adaptive, wl.step_uniform):
            out = ctx.trace_scene(field, views, quads, st)
            _compare(out, md, views, quads, st, wl.grid.voxel, f"scene {dtype} {which} uniform={st.uniform}",
                     tol_scale=5.0 if dtype == "bf16" else 1.0)
    field.release()


def test_scene_outer_boards_only_and_subset(ctx, haze):
    wl = W.make_small(seed=12, width=40, height=24, nviews=1).with_k_gd(150.0)
    parts = haze.upload_particles(wl.particles)
    field = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
    md = oracle.field(wl.particles, wl.grid, wl.k_gd, wl.h)
    views = _views(wl.grid.lo, wl.grid.hi, n=2, width=40, height=24)
    for which in ("outer", "all"):
        quads = _boards(wl.grid.lo, wl.grid.hi, which)
        full = ctx.trace_scene(field, views, quads, wl.step_adaptive)
        _compare(full, md, views, quads, wl.step_adaptive, wl.grid.voxel, f"scene {which}")
        total = sum(v.nrays for v in views)
        ids = np.array([0, 17, total - 1, 5, 5, total // 2, 1234, 999, 63, 64], np.int64)
        part = ctx.trace_scene(field, views, quads, wl.step_adaptive, ray_ids=torch.from_numpy(ids).cuda())
        F, P = to_np(full), to_np(part)
        for k in P:   # a ray's result does not depend on the rest of the launch
            assert np.array_equal(P[k].view(np.uint8), F[k][ids].view(np.uint8)), (which, k)
    field.release()


def test_scene_without_boards_is_trace_views(ctx, haze):
    wl = W.make_small(seed=13, width=29, height=19, nviews=2).with_k_gd(100.0)
    parts = haze.upload_particles(wl.particles)
    field = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
    a = to_np(ctx.trace_views(field, wl.views, wl.step_adaptive))
    b = to_np(ctx.trace_scene(field, wl.views, np.zeros((0, 3, 3), np.float32), wl.step_adaptive))
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k
    assert np.all(b["surface"] == np.where(b["status"] == 0, 0, 255))
    field.release()


def test_scene_two_boards_in_one_step(ctx, haze):
    # boards 2 mm apart inside a zero field, 0.25-voxel steps of ~6 mm: both
    # are crossed within one chord; the nearer wins in either list order
    grid = W.make_grid((0.0, 0.0, 0.0), (0.8, 0.8, 0.8), (32, 32, 32))
    f = ctx.index_field_from_grid(torch.zeros((32, 32, 32), dtype=torch.float32, device="cuda"), grid)
    md = oracle.Medium.from_grid(grid, np.zeros((32, 32, 32)))
    view = W.ring_view(grid.lo, grid.hi, 0.0, 1.5, 31, 27, vfov_deg=20.0, backdrop_beyond=0.5)
    near = ((0.2, 0.400, 0.2), (0.4, 0.0, 0.0), (0.0, 0.0, 0.4))
    far = ((0.2, 0.402, 0.2), (0.4, 0.0, 0.0), (0.0, 0.0, 0.4))
    st = W.make_steps(grid)[1]
    for order, want in (((near, far), 1), ((far, near), 2)):
        quads = W.quads(order)
        out = ctx.trace_scene(f, [view], quads, st)
        g, ref = _compare(out, md, [view], quads, st, grid.voxel, f"two boards {want}")
        hit = (ref["surface"] == 1) | (ref["surface"] == 2)
        assert hit.sum() > 50 and np.all(ref["surface"][hit] == want)
        np.testing.assert_allclose(g["exit_pos"][hit][:, 1], 0.400, atol=1e-6)
        assert np.abs(g["disp"][hit]).max() < 1e-3
    f.release()


def test_scene_errors(ctx, haze):
    wl = W.make_small(seed=14, width=8, height=8, nviews=1)
    parts = haze.upload_particles(wl.particles)
    field = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
    lo, hi = np.asarray(wl.grid.lo), np.asarray(wl.grid.hi)
    ok = _boards(lo, hi, "outer")[0]
    with pytest.raises(haze.HazeError) as e:
        ctx.trace_scene(field, wl.views, np.stack([ok] * 9), wl.step_adaptive)
    assert e.value.status == haze.E_INVALID
    flat = ok.copy()
    flat[2] = 2.0 * flat[1]          # parallel edges
    with pytest.raises(haze.HazeError) as e:
        ctx.trace_scene(field, wl.views, flat[None], wl.step_adaptive)
    assert e.value.status == haze.E_INVALID
    c = 0.5 * (lo + hi)
    inside = [(c + (0, 0.01 * k, 0), (0.05, 0, 0), (0, 0, 0.05)) for k in range(5)]
    with pytest.raises(haze.HazeError) as e:
        ctx.trace_scene(field, wl.views, W.quads(inside), wl.step_adaptive)
    assert e.value.status == haze.E_UNSUPPORTED
    # four boards inside is fine
    out = to_np(ctx.trace_scene(field, wl.views, W.quads(inside[:4]), wl.step_adaptive))
    assert out["status"].max() <= 2
    field.release()
