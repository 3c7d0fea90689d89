"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Splat (Sec. 3.3.1, Eqs. 12-13) and trace (Sec. 3.3.2-3.3.3, Eqs. 16-18) on
seeded inputs: small ragged cases (odd grid and image sizes, several views,
partial 8x8 tiles), stress fields (K_GD x 200) where bending is large enough
for the tolerances to bite, adaptive and fixed steps, analytic grids, and
edge cases.  Every launch goes through libhaze.so.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_02048_amd import workloads as W
from tests.parity import (assert_field_match, assert_rays_match, assert_rays_match_conditioned,
                          oracle_sensitivity, to_np)

pytestmark = pytest.mark.gpu


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


def _field_np(ctx, field):
    arrs = ctx.field_read(field)
    torch.cuda.synchronize()
    return [a.cpu().numpy() for a in arrs]


def _splat_both(ctx, haze, wl, dtype="f32", scale=1.0):
    print(f"case {wl.name}: n={wl.particles.n} res={tuple(wl.grid.res)} h={wl.h} dtype={dtype}", flush=True)
    parts = haze.upload_particles(wl.particles)
    field = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h, dtype=dtype, store_scale=scale)
    md = oracle.field(wl.particles, wl.grid, wl.k_gd, wl.h)
    return field, md


# splat kernels: (splat.method, splat.brick_z); the gather brick depth is
# chosen per grid by default and forced here so both depths are checked
SPLAT_METHODS = {"gather": (1, 4), "gather8": (1, 8), "scatter": (2, 0)}


def _use(ctx, method):
    m, bz = SPLAT_METHODS[method]
    ctx.tune("splat.method", m)
    ctx.tune("splat.brick_z", bz)


def _default(ctx):
    ctx.tune("splat.method", 0)
    ctx.tune("splat.brick_z", 0)


@pytest.mark.parametrize("method", ["gather", "gather8", "scatter"])
@pytest.mark.parametrize("seed,res,h", [(0, (21, 17, 13), 0.03), (1, (8, 9, 30), 0.05), (2, (2, 3, 2), 0.2),
                                        (3, (40, 33, 19), 0.02),
                                        # z reach (cell + 4h) shorter than a brick: cell rows whose reach
                                        # cuts the brick at both ends (full loop) or misses it
                                        (4, (24, 20, 10), 0.012),
                                        # z spacing 4-5x the x-y spacing: the support spans about one plane
                                        # either side, and the default brick depth is 4
                                        (5, (40, 40, 6), 0.03)])
def test_splat_parity_small(ctx, haze, seed, res, h, method):
    _use(ctx, method)
    try:
        wl = W.make_small(seed=seed, res=res, h=h, n=6000)
        if method == "scatter" and seed == 4:
            # the scatter tile grown by 2h spans more cell rows than it can
            # list at this h: refused, as documented
            with pytest.raises(haze.HazeError) as e:
                ctx.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
            assert e.value.status == haze.E_UNSUPPORTED
            return
        field, md = _splat_both(ctx, haze, wl)
        dn, gx, gy, gz = _field_np(ctx, field)
        ref = md.arrays
        assert_field_match(dn, (gx, gy, gz), ref[0], ref[1:], wl.grid.spacing,
                           f"splat {method} seed={seed} res={res}")
        field.release()
    finally:
        _default(ctx)


@pytest.mark.parametrize("method", ["gather", "gather8", "scatter"])
def test_splat_is_bitwise_repeatable(ctx, haze, method):
    _use(ctx, method)
    try:
        wl = W.make_small(seed=3, n=5000)
        parts = haze.upload_particles(wl.particles)
        f1 = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
        f2 = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
        a, b = _field_np(ctx, f1), _field_np(ctx, f2)
        for x, y in zip(a, b):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
        f1.release()
        f2.release()
    finally:
        _default(ctx)


def test_splat_brick_order_keeps_the_field(ctx, haze):
    """The gather hands out its bricks heaviest first, by each brick's
    candidate count in the previous gather over the same bricks.  The field is
    bitwise the same in plain order, on a context's first gather (no counts
    yet), on the gathers after it, and after the grid changes (the counts of
    other bricks are not used); the order is a permutation, so no brick is
    lost or repeated."""
    print("case splat brick order: config 1, then a small grid, orders off/on", flush=True)
    wls = [W.make_config(1), W.make_small(seed=8, n=6000, res=(40, 24, 16))]
    parts = [haze.upload_particles(w.particles) for w in wls]

    def field(k):
        f = ctx.splat_index_field(parts[k], wls[k].grid, wls[k].k_gd, wls[k].h)
        out = _field_np(ctx, f)
        f.release()
        return out

    try:
        fresh = haze.Context(0)   # first gather of a context: no counts
        try:
            f = fresh.splat_index_field(parts[0], wls[0].grid, wls[0].k_gd, wls[0].h)
            first = _field_np(fresh, f)
            f.release()
        finally:
            fresh.close()
        ctx.tune("splat.order", 0)
        plain = [field(0), field(1)]
        ctx.tune("splat.order", 1)
        runs = [(0, field(0)), (0, field(0)), (1, field(1)), (1, field(1)), (0, field(0))]
        for k, got in [(0, first)] + runs:
            for x, y in zip(plain[k], got):
                assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), k
    finally:
        ctx.tune("splat.order", 1)


@pytest.mark.parametrize("method", ["gather", "gather8", "scatter"])
def test_splat_skips_nonfinite_masses(ctx, haze, method):
    """Particles whose mass is NaN or infinite add nothing: the field with a
    few of them interleaved is bitwise the field without them (the others keep
    their relative order, so every voxel's sum runs in the same order)."""
    _use(ctx, method)
    try:
        wl = W.make_small(seed=5, n=4000)
        p = wl.particles
        rng = np.random.default_rng(5)
        k = 7
        at = np.sort(rng.choice(p.n + k, size=k, replace=False))
        keep = np.setdiff1d(np.arange(p.n + k), at)
        lo, hi = np.asarray(wl.grid.lo), np.asarray(wl.grid.hi)
        def merged(a, extra):
            out = np.empty(p.n + k, np.float32)
            out[keep] = a
            out[at] = extra
            return out
        pos = lo + (hi - lo) * rng.random((k, 3))
        bad_m = np.array([np.nan, np.inf, -np.inf, np.nan, np.inf, -np.nan, np.inf], np.float32)
        both = W.Particles(merged(p.x, pos[:, 0]), merged(p.y, pos[:, 1]), merged(p.z, pos[:, 2]), merged(p.m, bad_m))
        print(f"case non-finite masses {method}: {k} of {p.n + k} particles", flush=True)
        f1 = ctx.splat_index_field(haze.upload_particles(p), wl.grid, wl.k_gd, wl.h)
        f2 = ctx.splat_index_field(haze.upload_particles(both), wl.grid, wl.k_gd, wl.h)
        a, b = _field_np(ctx, f1), _field_np(ctx, f2)
        assert np.isfinite(b[0]).all()
        for x, y in zip(a, b):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
        f1.release()
        f2.release()
    finally:
        _default(ctx)


def test_splat_methods_on_config2(ctx, haze):
    # both splat kernels at the benchmark's size, against the oracle
    wl = W.make_config(2)
    md = oracle.field(wl.particles, wl.grid, wl.k_gd, wl.h)
    ref = md.arrays
    parts = haze.upload_particles(wl.particles)
    for method in SPLAT_METHODS:
        _use(ctx, method)
        f = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
        dn, gx, gy, gz = _field_np(ctx, f)
        assert_field_match(dn, (gx, gy, gz), ref[0], ref[1:], wl.grid.spacing, f"config2 splat {method}")
        f.release()
    _default(ctx)


def test_splat_particles_outside_grid(ctx, haze):
    # particles beyond the grid box still contribute within 2h; far ones never
    rng = np.random.default_rng(7)
    n = 4000
    pos = rng.uniform(-0.3, 0.8, (n, 3))
    p = W.Particles(*(pos[:, a].astype(np.float32) for a in range(3)), m=rng.uniform(0.5, 1.5, n).astype(np.float32))
    grid = W.make_grid((0.0, 0.1, 0.2), (0.5, 0.45, 0.4), (19, 11, 9))
    wl = W.Workload("outside", p, grid, 2.26e-4, 0.04, [], None, None)
    field, md = _splat_both(ctx, haze, wl)
    dn, gx, gy, gz = _field_np(ctx, field)
    ref = md.arrays
    assert_field_match(dn, (gx, gy, gz), ref[0], ref[1:], grid.spacing, "outside")
    field.release()


def test_splat_cell_scan_paths(ctx, haze):
    # The cell histogram is scanned in one launch up to 1024 tiles of 2048
    # cells and in three passes beyond; the histogram and the one-pass scan's
    # counter carry state from call to call.  Alternate the two paths (a
    # support far below the voxel size gives ~9e6 cells), with the scatter
    # splat in between, in one context.
    small = W.make_small(seed=4, n=6000)
    fine = W.make_small(seed=5, n=20000, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), res=(64, 64, 64), h=0.005)
    refs = {}
    for wl, method in ((small, "gather"), (fine, "gather"), (small, "gather"), (small, "scatter"),
                       (small, "gather"), (fine, "gather"), (fine, "gather")):
        _use(ctx, method)
        try:
            if wl.name + str(wl.h) not in refs:
                refs[wl.name + str(wl.h)] = oracle.field(wl.particles, wl.grid, wl.k_gd, wl.h).arrays
            ref = refs[wl.name + str(wl.h)]
            print(f"case scan paths: h={wl.h} res={tuple(wl.grid.res)} {method}", flush=True)
            parts = haze.upload_particles(wl.particles)
            f = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
            dn, gx, gy, gz = _field_np(ctx, f)
            assert np.count_nonzero(ref[0]) > 1000
            assert_field_match(dn, (gx, gy, gz), ref[0], ref[1:], wl.grid.spacing, f"scan paths h={wl.h} {method}")
            f.release()
        finally:
            _default(ctx)


@pytest.mark.parametrize("kgd", [1.0, 200.0])
@pytest.mark.parametrize("mode", ["adaptive", "uniform", "adaptive_fine"])
def test_trace_parity_small(ctx, haze, kgd, mode):
    wl = W.make_small(seed=0, width=37, height=23, nviews=3).with_k_gd(kgd)
    field, md = _splat_both(ctx, haze, wl)
    if mode == "adaptive":
        st = wl.step_adaptive
    elif mode == "uniform":
        st = wl.step_uniform
    else:   # small theta so the curvature rule engages between the clamps
        st, _ = W.make_steps(wl.grid, theta_max=1e-5 if kgd > 1 else 1e-7)
    out = ctx.trace_views(field, wl.views, st)
    torch.cuda.synchronize()
    ref = oracle.trace_views(md, wl.views, st)
    assert_rays_match(out, ref, wl.grid.voxel, f"small kgd x{kgd} {mode}")
    g = to_np(out)
    assert (g["steps"] > 0).sum() > 100
    if mode == "adaptive_fine" and kgd > 1:
        # the step rule really varies the step: not all rays take the same number of steps per length
        assert np.unique(g["steps"]).size > 20
    field.release()


def test_trace_subset_and_repeatability(ctx, haze):
    wl = W.make_small(seed=4, width=40, height=24, nviews=2).with_k_gd(100.0)
    field, md = _splat_both(ctx, haze, wl)
    total = wl.nrays
    ids = np.array([0, 5, total - 1, 7, 7, 123, total // 2, 999], np.int64)
    t_ids = torch.from_numpy(ids).cuda()
    a = ctx.trace_views(field, wl.views, wl.step_adaptive, ray_ids=t_ids)
    b = ctx.trace_views(field, wl.views, wl.step_adaptive, ray_ids=t_ids)
    full = ctx.trace_views(field, wl.views, wl.step_adaptive)
    torch.cuda.synchronize()
    A, B, F = to_np(a), to_np(b), to_np(full)
    for k in A:
        assert np.array_equal(A[k].view(np.uint8), B[k].view(np.uint8)), k
        # a ray's result does not depend on which other rays share the launch
        assert np.array_equal(A[k].view(np.uint8), F[k][ids].view(np.uint8)), k
    ref = oracle.trace_views(md, wl.views, wl.step_adaptive, ray_ids=ids)
    assert_rays_match(a, ref, wl.grid.voxel, "subset")
    field.release()


def test_trace_repeated_calls_reset_the_queue(ctx, haze):
    # few march waves (one workgroup per CU) and many rays, so most rays come
    # from the dynamic batches: every call must start from a fresh queue
    wl = W.make_small(seed=8, width=256, height=192, nviews=8, radius=0.9).with_k_gd(50.0)
    parts = haze.upload_particles(wl.particles)
    field = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
    ctx.tune("march.blocks_per_cu", 1)
    try:
        a1 = to_np(ctx.trace_views(field, wl.views, wl.step_adaptive))
        u1 = to_np(ctx.trace_views(field, wl.views, wl.step_uniform))
        a2 = to_np(ctx.trace_views(field, wl.views, wl.step_adaptive))
        u2 = to_np(ctx.trace_views(field, wl.views, wl.step_uniform))
    finally:
        ctx.tune("march.blocks_per_cu", 0)
    hits = int((a1["steps"] > 0).sum())
    print(f"repeated calls: {hits} rays in the volume", flush=True)
    assert hits > 4 * 256 * 64        # well past the static batches of 1024 waves
    for x, y in ((a1, a2), (u1, u2)):
        for k in x:
            assert np.array_equal(x[k].view(np.uint8), y[k].view(np.uint8)), k
    # and the same as a default launch shape
    a3 = to_np(ctx.trace_views(field, wl.views, wl.step_adaptive))
    for k in a1:
        assert np.array_equal(a1[k].view(np.uint8), a3[k].view(np.uint8)), k
    field.release()


def test_trace_nonfinite_field(ctx, haze):
    # a NaN voxel: rays whose samples touch it (directly or through the
    # gradient's differences) end with status NONFINITE and NaN displacement,
    # as in the oracle; every other ray is unaffected
    grid = W.make_grid((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (24, 24, 24))
    dn = W.analytic_grid_gauss(grid, 2e-3, (0.5, 0.5, 0.5), 0.2)
    dn[12, 11, 10] = np.nan
    f = ctx.index_field_from_grid(torch.from_numpy(dn.astype(np.float32)).cuda(), grid)
    md = oracle.Medium.from_grid(grid, dn.astype(np.float32).astype(np.float64))
    views = [W.ring_view(grid.lo, grid.hi, 0.0, 2.0, 48, 48, vfov_deg=35.0)]
    for st in W.make_steps(grid):
        out = to_np(ctx.trace_views(f, views, st))
        ref = oracle.trace_views(md, views, st)
        bad = ref["status"] == W.STATUS_NONFINITE
        assert bad.sum() > 5 and (~bad).sum() > 1000
        assert np.array_equal(out["status"], ref["status"])
        assert np.isnan(out["disp"][bad]).all()
        good = {k: v[~bad] for k, v in out.items()}
        assert_rays_match(good, {k: v[~bad] for k, v in ref.items()}, grid.voxel, f"nonfinite uniform={st.uniform}")
    f.release()


def test_trace_bad_ray_ids_flagged(ctx, haze):
    wl = W.make_small(seed=5, width=9, height=8, nviews=1)
    field, _ = _splat_both(ctx, haze, wl)
    ids = torch.tensor([3, -1, 72, 10_000, 71], dtype=torch.int64, device="cuda")
    out = to_np(ctx.trace_views(field, wl.views, wl.step_adaptive, ray_ids=ids))
    assert list(out["status"]) == [0, 4, 4, 4, 0]
    assert np.isnan(out["disp"][1:4]).all()
    field.release()


def test_trace_edge_cases(ctx, haze):
    wl = W.make_small(seed=6, width=1, height=1, nviews=1).with_k_gd(50.0)
    field, md = _splat_both(ctx, haze, wl)
    # 1x1 image looking at the box centre
    out = ctx.trace_views(field, wl.views, wl.step_uniform)
    ref = oracle.trace_views(md, wl.views, wl.step_uniform)
    assert_rays_match(out, ref, wl.grid.voxel, "1x1")
    # views that miss the volume entirely (looking away): zero steps, zero displacement
    v = wl.views[0]
    away = W.View(eye=v.eye, fwd=-v.fwd, up=v.up, vfov=v.vfov, width=13, height=11,
                  plane_p=(v.eye - 2.0 * v.fwd).astype(np.float32), plane_n=v.fwd)
    out = to_np(ctx.trace_views(field, [away], wl.step_adaptive))
    assert (out["steps"] == 0).all() and (out["status"] == 0).all()
    assert np.abs(out["disp"]).max() < 1e-3
    ref = oracle.trace_views(md, [away], wl.step_adaptive)
    assert_rays_match(out, ref, wl.grid.voxel, "away")
    # max_steps cap
    st = W.make_steps(wl.grid)[1]
    st.max_steps = 3
    wl2 = W.make_small(seed=6, width=11, height=7, nviews=1)
    out = to_np(ctx.trace_views(field, wl2.views, st))
    ref = oracle.trace_views(md, wl2.views, st)
    assert (out["status"] == 1).sum() > 0
    assert_rays_match(out, ref, wl.grid.voxel, "max_steps")
    field.release()


def test_tune_keys_checked(ctx, haze):
    for key, bad in (("march.refill_min", 0), ("march.refill_min", 65), ("march.blocks_per_cu", -1),
                     ("march.blocks_per_cu", 65), ("splat.method", 3), ("splat.brick_z", 5), ("splat.brick_z", 16),
                     ("splat.order", 2), ("splat.order", -1), ("no.such.key", 1)):
        with pytest.raises(haze.HazeError) as e:
            ctx.tune(key, bad)
        assert e.value.status == haze.E_INVALID, (key, bad)
    for key, good in (("march.refill_min", 32), ("march.blocks_per_cu", 0), ("splat.method", 0),
                      ("splat.brick_z", 8), ("splat.brick_z", 0), ("splat.order", 0), ("splat.order", 1)):
        ctx.tune(key, good)


def test_grid_limits_rejected(ctx, haze):
    # each axis holds 2 to 65535 voxels; nothing is launched for a bad grid
    wl = W.make_small(seed=6, n=500)
    parts = haze.upload_particles(wl.particles)
    for res in ((1, 8, 8), (8, 65536, 2), (65536, 2, 2)):
        bad = W.make_grid(wl.grid.lo, wl.grid.hi, res)
        with pytest.raises(haze.HazeError) as e:
            ctx.splat_index_field(parts, bad, wl.k_gd, wl.h)
        assert e.value.status == haze.E_INVALID and "65535" in str(e.value)


def test_grid_axis_at_limit(ctx, haze):
    # 65535 voxels along one axis (the largest accepted), a few along the
    # others; the long axis spans 0.5 m, so that float32 coordinates of voxel
    # centres and particles (~ulp 6e-8 m) stay far below the 8 mm support
    rng = np.random.default_rng(11)
    n = 3000
    lo, hi = (0.0, 0.0, 0.0), (0.5, 0.01, 0.012)
    pos = np.asarray(lo) + rng.random((n, 3)) * (np.asarray(hi) - np.asarray(lo))
    p = W.Particles(*(pos[:, a].astype(np.float32) for a in range(3)), m=rng.uniform(0.5, 1.5, n).astype(np.float32))
    for res in ((65535, 2, 3), (3, 2, 65535)):
        lo_r = lo if res[0] > 3 else (0.0, 0.0, 0.0)
        hi_r = hi if res[0] > 3 else (0.012, 0.01, 0.5)
        pts = p if res[0] > 3 else W.Particles(p.z.copy(), p.y, p.x.copy(), m=p.m)
        grid = W.make_grid(lo_r, hi_r, res)
        wl = W.Workload("axis-limit", pts, grid, 2.26e-4, 0.004, [], None, None)
        field, md = _splat_both(ctx, haze, wl)
        dn, gx, gy, gz = _field_np(ctx, field)
        ref = md.arrays
        assert np.count_nonzero(ref[0]) > 1000
        assert_field_match(dn, (gx, gy, gz), ref[0], ref[1:], grid.spacing, f"axis limit res={res}")
        field.release()


def test_field_from_grid_round_trip(ctx, haze):
    # the packed field keeps its own voxel order; the [z][y][x] export must
    # give back the [z][y][x] input bit for bit (F32), and the gradient the
    # central / one-sided differences of it, voxel by voxel, on a ragged grid
    grid = W.make_grid((0.0, 0.0, 0.0), (1.0, 0.8, 1.3), (7, 5, 11))
    print("case field round trip: 7 x 5 x 11 grid, random delta-n", flush=True)
    rng = np.random.default_rng(3)
    dn = rng.standard_normal((11, 5, 7)).astype(np.float32) * np.float32(1e-4)
    f = ctx.index_field_from_grid(torch.from_numpy(dn).cuda(), grid)
    d, gx, gy, gz = _field_np(ctx, f)
    assert np.array_equal(d.view(np.uint32), dn.view(np.uint32))
    ref = np.gradient(dn.astype(np.float64), *[float(s) for s in grid.spacing[::-1]], edge_order=1)
    for g, r, name in ((gz, ref[0], "z"), (gy, ref[1], "y"), (gx, ref[2], "x")):
        assert np.abs(g - r).max() <= 1e-5 * np.abs(r).max(), name
    f.release()


def test_field_from_grid_linear_and_catenary(ctx, haze):
    # a linear delta-n grid: the GPU gradient is exact up to rounding and the
    # rays follow the oracle's (grid-exact) catenary replica
    grid = W.make_grid((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (33, 29, 31))
    G = (0.02, 0.0, -0.01)
    dn = W.analytic_grid_linear(grid, 1e-3, G)
    f = ctx.index_field_from_grid(torch.from_numpy(dn.astype(np.float32)).cuda(), grid)
    d, gx, gy, gz = _field_np(ctx, f)
    for g, b in zip((gx, gy, gz), G):
        assert np.abs(g - b).max() < 2e-5 * max(abs(b), 1e-3) + 1e-9
    md = oracle.Medium.from_grid(grid, dn.astype(np.float32).astype(np.float64))
    views = [W.ring_view(grid.lo, grid.hi, az, 2.5, 31, 17) for az in (0.0, 0.7)]
    st_a, st_u = W.make_steps(grid, theta_max=1e-4)
    for st in (st_a, st_u):
        out = ctx.trace_views(f, views, st)
        ref = oracle.trace_views(md, views, st)
        assert_rays_match(out, ref, grid.voxel, f"linear uniform={st.uniform}")
    f.release()


def test_config1_full_parity(ctx, haze):
    wl = W.make_config(1)
    field, md = _splat_both(ctx, haze, wl)
    dn, gx, gy, gz = _field_np(ctx, field)
    ref = md.arrays
    assert_field_match(dn, (gx, gy, gz), ref[0], ref[1:], wl.grid.spacing, "config1")
    for st in (wl.step_adaptive, wl.step_uniform):
        out = ctx.trace_views(field, wl.views, st)
        r = oracle.trace_views(md, wl.views, st)
        assert_rays_match(out, r, wl.grid.voxel, f"config1 uniform={st.uniform}")
    field.release()
    # stress variant (the paper's theta_max binds): a few rays are ill-conditioned
    wl = wl.with_k_gd(250.0)
    field, md = _splat_both(ctx, haze, wl)
    for st in (wl.step_adaptive, wl.step_uniform):
        out = ctx.trace_views(field, wl.views, st)
        r = oracle.trace_views(md, wl.views, st)
        sens = oracle_sensitivity(oracle, wl.grid, md.arrays[0], wl.views, st)
        assert_rays_match_conditioned(out, r, sens, wl.grid.voxel, f"config1 kgd x250 uniform={st.uniform}")
    field.release()


def test_config2_subset_parity(ctx, haze):
    wl = W.make_config(2)
    field, md = _splat_both(ctx, haze, wl)
    dn, gx, gy, gz = _field_np(ctx, field)
    ref = md.arrays
    assert_field_match(dn, (gx, gy, gz), ref[0], ref[1:], wl.grid.spacing, "config2")
    ids = torch.from_numpy(wl.subset).cuda()
    for st in (wl.step_adaptive, wl.step_uniform):
        # full launch as the benchmark runs it; compare the subset rays
        full = to_np(ctx.trace_views(field, wl.views, st))
        r = oracle.trace_views(md, wl.views, st, ray_ids=wl.subset)
        sub = {k: v[wl.subset] for k, v in full.items()}
        assert_rays_match(sub, r, wl.grid.voxel, f"config2 uniform={st.uniform}")
        part = ctx.trace_views(field, wl.views, st, ray_ids=ids)
        for k, v in to_np(part).items():
            assert np.array_equal(v.view(np.uint8), sub[k].view(np.uint8)), k
    field.release()
