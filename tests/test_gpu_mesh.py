"""GPU parity of triangle-mesh scenes (hz_trace_mesh) against the FP64 oracle,
and the conservative shell of Sec. 4.1.

The oracle tests every triangle on every chord and straight segment; the GPU
tests only the triangles the shell lists for the cells it passes, and none
where the shell's distance bound exceeds the step.  Which surface a ray meets
is decided in floating point near a surface's rim: there the oracle is also
run with the geometry shrunk and grown by a small margin, and a ray whose
answer differs between those runs is checked only for validity.  Every other
ray must match surface and status, and the tolerances as on the other stress
fields: the plain ones, or 3x the oracle's own spread under perturbations of
the FP32 path's rounding size where that is larger, with at least 99.5% of
the rays within the plain ones.  The shell must not
change any result: a brute-force mesh (no shell) gives the same bits, with
many more exact tests per ray.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_02048_amd import workloads as W
from tests.parity import assert_rays_match_conditioned, oracle_sensitivity, to_np
from tests.test_gpu_scene import _boards, _inflate, _views

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


def _compare(g, md, views, geo, st, voxel, label):
    """geo: (tris, surf) and the shrunk and grown variants [(tris, surf)] * 3.
    The fields here are stress fields (K_GD x 200), so rays are held to the
    plain tolerances or, where the oracle's own answer moves more under
    perturbations of the FP32 path's rounding size, to 3x that spread."""
    (tr, sf), (tlo, slo), (thi, shi) = geo
    ref = oracle.trace_mesh(md, views, tr, sf, st)
    sens = oracle_sensitivity(oracle, md.grid, md.arrays[0], views, st,
                              tracer=lambda m, v, s, ray_ids: oracle.trace_mesh(m, v, tr, sf, s, ray_ids=ray_ids))
    lo_ = oracle.trace_mesh(md, views, tlo, slo, st)
    hi_ = oracle.trace_mesh(md, views, thi, shi, st)
    amb = (lo_["surface"] != hi_["surface"]) | (lo_["surface"] != ref["surface"])
    ok_amb = (g["surface"] == lo_["surface"]) | (g["surface"] == hi_["surface"]) | (g["surface"] == ref["surface"])
    print(f"{label}: {amb.sum()} of {amb.size} rays near a rim; surfaces seen "
          f"{np.bincount(ref['surface'], minlength=256)[[0, 1, 2, 3, 4, 255]].tolist()}", flush=True)
    assert amb.mean() < 0.03, label
    assert ok_amb[amb].all(), label
    keep = ~amb
    assert np.array_equal(g["surface"][keep], ref["surface"][keep]), label
    assert_rays_match_conditioned({k: v[keep] for k, v in g.items() if k not in ("surface", "tri_tests")},
                                  {k: v[keep] for k, v in ref.items() if k != "surface"},
                                  {k: v[keep] for k, v in sens.items()}, voxel, label)
    return ref


def _board_geometry(grid, n=4):
    quads = _boards(grid.lo, grid.hi)
    m = MARGIN_VOX * grid.voxel
    return [W.tessellate_quads(q, n) for q in (quads, _inflate(quads, -m), _inflate(quads, m))]


@pytest.mark.parametrize("mode", ["adaptive", "uniform"])
def test_mesh_boards_parity(ctx, haze, mode):
    wl = W.make_small(seed=11, width=37, height=23, nviews=1).with_k_gd(200.0)
    print(f"case mesh boards kgd x200 {mode}", flush=True)
    field = ctx.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
    md = oracle.field(wl.particles, wl.grid, wl.k_gd, wl.h)
    views = _views(wl.grid.lo, wl.grid.hi)
    geo = _board_geometry(wl.grid)
    st = wl.step_adaptive if mode == "adaptive" else wl.step_uniform
    mesh = ctx.mesh_create(*geo[0], reach=wl.step_adaptive.ds_max)
    out = to_np(ctx.trace_mesh(field, views, mesh, st, count_tests=True))
    ref = _compare(out, md, views, geo, st, wl.grid.voxel, f"mesh boards {mode}")
    for k in (0, 1, 2, 3, 4):
        assert (ref["surface"] == k).sum() > 20, k
    inner = (ref["surface"] == 1) | (ref["surface"] == 2)
    assert (out["steps"][inner] > 0).all()
    mesh.release()
    field.release()


def test_mesh_shell_changes_no_result(ctx, haze):
    wl = W.make_small(seed=12, width=48, height=36, nviews=2).with_k_gd(200.0)
    print("case mesh shell vs brute force: 4 boards of 32 triangles + a sphere of 320", flush=True)
    field = ctx.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
    views = _views(wl.grid.lo, wl.grid.hi, n=2, width=48, height=36)
    tb, sb = W.tessellate_quads(_boards(wl.grid.lo, wl.grid.hi), 4)
    c = 0.5 * (wl.grid.lo + wl.grid.hi) + np.array([0.05, 0.02, 0.0])
    ts = W.icosphere(c, 0.09, 2)
    tris = np.concatenate([tb, ts])
    surf = np.concatenate([sb, np.full(len(ts), 9)])
    reach = wl.step_adaptive.ds_max
    shell = ctx.mesh_create(tris, surf, reach=reach)
    brute = ctx.mesh_create(tris, surf, reach=reach, brute_force=True)
    info = shell.info()
    for st in (wl.step_adaptive, wl.step_uniform):
        a = to_np(ctx.trace_mesh(field, views, shell, st, count_tests=True))
        b = to_np(ctx.trace_mesh(field, views, brute, st, count_tests=True))
        for k in a:
            if k != "tri_tests":
                assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k
        ins = a["steps"] > 0
        print(f"uniform={st.uniform}: {len(tris)} triangles, shell {info['shell_res']} cells of "
              f"{info['shell_cell'] * 1e3:.1f} mm, {info['list_entries']} list entries; exact tests per ray "
              f"with the shell {a['tri_tests'].mean():.1f} (rays in the volume {a['tri_tests'][ins].mean():.1f}), "
              f"without {b['tri_tests'].mean():.1f} ({b['tri_tests'][ins].mean():.1f}); surfaces "
              f"{np.bincount(a['surface'], minlength=256)[[0, 1, 2, 3, 4, 10, 255]].tolist()}", flush=True)
        assert (a["surface"] == 10).sum() > 50            # the sphere is seen
        assert a["tri_tests"].sum() * 5 < b["tri_tests"].sum()
    # a subset of ray ids: the same bits as the full launch
    ids = torch.arange(5, sum(v.nrays for v in views), 7, dtype=torch.int64, device="cuda")
    full = to_np(ctx.trace_mesh(field, views, shell, wl.step_adaptive))
    part = to_np(ctx.trace_mesh(field, views, shell, wl.step_adaptive, ray_ids=ids))
    sel = ids.cpu().numpy()
    for k in part:
        assert np.array_equal(part[k].view(np.uint8), full[k][sel].view(np.uint8)), k
    shell.release()
    brute.release()
    field.release()


def test_mesh_sphere_inside_volume(ctx, haze):
    wl = W.make_small(seed=13, width=64, height=48, nviews=1).with_k_gd(200.0)
    print("case mesh sphere of 320 triangles inside the volume", flush=True)
    field = ctx.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
    md = oracle.field(wl.particles, wl.grid, wl.k_gd, wl.h)
    views = _views(wl.grid.lo, wl.grid.hi, n=1, width=64, height=48)
    c = 0.5 * (wl.grid.lo + wl.grid.hi)
    r = 0.11
    m = MARGIN_VOX * wl.grid.voxel
    geo = [(W.icosphere(c, rr, 2), np.full(320, 4)) for rr in (r, r - m, r + m)]
    mesh = ctx.mesh_create(*geo[0], reach=wl.step_adaptive.ds_max)
    for st in (wl.step_adaptive, wl.step_uniform):
        out = to_np(ctx.trace_mesh(field, views, mesh, st))
        ref = _compare(out, md, views, geo, st, wl.grid.voxel, f"mesh sphere uniform={st.uniform}")
        hit = ref["surface"] == 5
        assert hit.sum() > 100 and (out["steps"][hit] > 0).all()
    mesh.release()
    field.release()


def test_mesh_arguments_checked(ctx, haze):
    wl = W.make_small(seed=14, width=8, height=8, nviews=1)
    field = ctx.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
    tris, surf = W.tessellate_quads(_boards(wl.grid.lo, wl.grid.hi), 2)
    with pytest.raises(haze.HazeError) as e:
        ctx.mesh_create(tris, surf, reach=0.0)
    assert e.value.status == haze.E_INVALID
    bad = tris.copy()
    bad[3, 2] = bad[3, 0]                               # a degenerate triangle
    with pytest.raises(haze.HazeError) as e:
        ctx.mesh_create(bad, surf, reach=0.01)
    assert e.value.status == haze.E_INVALID and "degenerate" in str(e.value)
    with pytest.raises(haze.HazeError) as e:
        ctx.mesh_create(tris, np.full(len(tris), 254), reach=0.01)
    assert e.value.status == haze.E_INVALID
    short = ctx.mesh_create(tris, surf, reach=0.5 * wl.step_adaptive.ds_max)
    with pytest.raises(haze.HazeError) as e:           # the adaptive step can exceed the shell's reach
        ctx.trace_mesh(field, wl.views, short, wl.step_adaptive)
    assert e.value.status == haze.E_INVALID and "shell serves" in str(e.value)
    ctx.trace_mesh(field, wl.views, short, wl.step_uniform)   # 0.25 voxel steps fit
    torch.cuda.synchronize()
    short.release()
    field.release()
