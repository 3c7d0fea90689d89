"""Pins of the oracle's triangle-mesh scenes (CPU only).

Sec. 4.1 speeds up the scene intersection of the refracted ray with a
conservative shell around the geometry, doing exact ray-triangle tests only
inside it.  The shell changes which exact tests are done, never their result,
so the oracle tests every triangle on every chord and straight segment (brute
force).  Pins:

  * a mesh made of two triangles per board reproduces the board (parallelogram)
    results of trace_scene, whose pins are in test_oracle_scene.py: same
    surfaces, hit points, exit directions, steps and displacements, in a
    constant, a linear (catenary) and a gridded medium;
  * n constant, two triangles of different surfaces at different depths: the
    surface each straight pixel ray meets follows from the triangles' closed
    inequalities (x >= a, z >= a, x + z <= b, ...) evaluated at the ray's
    crossing of each plane, so a wrong in-triangle condition, vertex order or
    surface id fails;
  * n constant, an axis-aligned cube of 12 triangles inside the volume: the hit
    point is the slab-test entry point of the cube and the surface its face;
  * n linear (grid-exact catenary): the hit point on a slanted two-triangle
    board converges at first order to the closed-form catenary's crossing of
    the board's plane.
"""
import math

import numpy as np
from scipy.optimize import brentq

from paper_2603_02048_amd import workloads as W
from tests.test_oracle_scene import BOX, _catenary_path, _scene_quads, _step, _view


def _split(quads, diagonal=0):
    """Two triangles per parallelogram (o, ea, eb), both of the quad's surface:
    (o, o + ea, o + eb) and (o + ea + eb, o + eb, o + ea) (diagonal 0), or the
    other diagonal (diagonal 1)."""
    tris, surf = [], []
    for k, (o, ea, eb) in enumerate(np.asarray(quads, np.float64)):
        a, b, c, d = o, o + ea, o + ea + eb, o + eb
        if diagonal == 0:
            tris += [(a, b, d), (c, d, b)]
        else:
            tris += [(a, b, c), (a, c, d)]
        surf += [k, k]
    return np.asarray(tris), np.asarray(surf)


def _assert_same(a, b, tol=1e-9):
    assert np.array_equal(a["surface"], b["surface"])
    assert np.array_equal(a["status"], b["status"])
    assert np.array_equal(a["steps"], b["steps"])
    for k in ("exit_pos", "exit_dir", "disp"):
        np.testing.assert_allclose(np.nan_to_num(a[k], nan=-7.0), np.nan_to_num(b[k], nan=-7.0), atol=tol, rtol=0)


def test_two_triangle_boards_reproduce_quads(oracle_lib):
    view = _view(64, 48)
    quads = _scene_quads()
    media = [oracle_lib.Medium(oracle_lib.MEDIUM_CONST, BOX, [3e-4]),
             oracle_lib.Medium(oracle_lib.MEDIUM_LINEAR, BOX, [1e-2, 0.02, -0.01, -0.03])]
    wl = W.make_small(seed=2, n=3000, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), res=(17, 19, 15), h=0.06)
    dn = oracle_lib.splat(wl.particles, wl.grid, wl.k_gd * 300.0, wl.h)
    media.append(oracle_lib.Medium.from_grid(wl.grid, dn))
    for md in media:
        grid_box = md.grid if hasattr(md, "grid") else BOX
        a, _ = W.make_steps(BOX, theta_max=1e-3)
        st = _step(0.011)
        for stp in (st, a):
            ref = oracle_lib.trace_scene(md, [view], quads, stp)
            for diag in (0, 1):
                tris, surf = _split(quads, diag)
                got = oracle_lib.trace_mesh(md, [view], tris, surf, stp)
                _assert_same(got, ref)
            for s in range(4):
                assert (ref["surface"] == s).sum() > 50, s


def test_triangles_of_two_surfaces(oracle_lib):
    # camera looking +y at two triangles in planes y = 0.5 (surface 3) and
    # y = 0.55 (surface 7), seen through a constant medium
    view = W.View(eye=W._f32([0.5, -1.0, 0.5]), fwd=W._f32([0, 1, 0]), up=W._f32([0, 0, 1]),
                  vfov=float(np.float32(math.radians(48))), width=48, height=40,
                  plane_p=W._f32([0.5, 3.0, 0.5]), plane_n=W._f32([0, -1, 0]))
    tris = np.array([[(0.2, 0.5, 0.2), (0.8, 0.5, 0.2), (0.2, 0.5, 0.8)],      # x, z >= 0.2, x + z <= 1.0
                     [(0.85, 0.55, 0.85), (0.85, 0.55, 0.15), (0.15, 0.55, 0.85)]])   # x, z <= 0.85, x + z >= 1.0
    surf = np.array([3, 7])
    md = oracle_lib.Medium(oracle_lib.MEDIUM_CONST, BOX, [2e-4])
    r = oracle_lib.trace_mesh(md, [view], tris, surf, _step(0.023))
    pix = np.array([(p, q) for q in range(view.height) for p in range(view.width)], np.int64)
    d = oracle_lib.pixel_rays(view, pix)
    eye = np.asarray(view.eye, np.float64)
    want = np.zeros(len(pix), np.int64)
    hit = np.full((len(pix), 3), np.nan)
    margin = np.zeros(len(pix))
    for y, test, sid in ((0.55, lambda x, z: (x <= 0.85) & (z <= 0.85) & (x + z >= 1.0), 8),
                         (0.50, lambda x, z: (x >= 0.2) & (z >= 0.2) & (x + z <= 1.0), 4)):
        t = (y - eye[1]) / d[:, 1]
        h = eye + t[:, None] * d
        inside = test(h[:, 0], h[:, 2])
        want[inside] = sid          # the nearer plane (y = 0.5) is assigned last and wins
        hit[inside] = h[inside]
    # rays within 1e-9 of a triangle edge are not compared
    for tri in tris:
        for i in range(3):
            p0, p1 = tri[i], tri[(i + 1) % 3]
            t = (p0[1] - eye[1]) / d[:, 1]
            h = eye + t[:, None] * d
            e = p1 - p0
            s = np.clip(((h - p0) @ e) / (e @ e), 0.0, 1.0)
            dist = np.linalg.norm(h - (p0 + s[:, None] * e), axis=1)
            margin = np.maximum(margin, (dist < 1e-9).astype(float))
    ok = margin == 0
    assert (want == 4).sum() > 100 and (want == 8).sum() > 100 and (want == 0).sum() > 100
    assert np.array_equal(r["surface"][ok].astype(np.int64), want[ok])
    m = ok & (want > 0)
    np.testing.assert_allclose(r["exit_pos"][m], hit[m], atol=1e-12)
    np.testing.assert_allclose(r["disp"][ok], 0.0, atol=1e-9)


def _cube(lo, hi):
    """12 triangles of the box [lo, hi]; surface 2a (lower face) / 2a + 1
    (upper face) on axis a."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    tris, surf = [], []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for side, val in ((0, lo[a]), (1, hi[a])):
            def pt(u, v):
                p = np.zeros(3)
                p[a], p[b], p[c] = val, u, v
                return p
            q = [pt(lo[b], lo[c]), pt(hi[b], lo[c]), pt(hi[b], hi[c]), pt(lo[b], hi[c])]
            tris += [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
            surf += [2 * a + side] * 2
    return np.asarray(tris), np.asarray(surf)


def test_cube_inside_volume_is_its_slab_entry(oracle_lib):
    # seen from above one corner, so that three faces face the camera
    view = W.ring_view(BOX.lo, BOX.hi, 0.7, 1.5, 96, 72, vfov_deg=44.0, backdrop_beyond=1.5, elevation=0.9)
    lo, hi = np.array([0.32, 0.36, 0.30]), np.array([0.61, 0.63, 0.58])
    tris, surf = _cube(lo, hi)
    md = oracle_lib.Medium(oracle_lib.MEDIUM_CONST, BOX, [1e-4])
    r = oracle_lib.trace_mesh(md, [view], tris, surf, _step(0.017))
    pix = np.array([(p, q) for q in range(view.height) for p in range(view.width)], np.int64)
    d = oracle_lib.pixel_rays(view, pix)
    eye = np.asarray(view.eye, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1, t2 = (lo - eye) / d, (hi - eye) / d
    tmin, tmax = np.minimum(t1, t2), np.maximum(t1, t2)
    ta, tb = tmin.max(axis=1), tmax.min(axis=1)
    hit = (ta <= tb) & (tb > 0)
    axis = tmin.argmax(axis=1)
    upper = d[np.arange(len(d)), axis] < 0            # entering through the upper face of that axis
    want = np.where(hit, 2 * axis + upper + 1, 0)
    # not compared: rays whose entry is within 1e-9 of a cube edge (two axes tie)
    srt = np.sort(tmin, axis=1)
    clear = ~hit | (srt[:, 2] - srt[:, 1] > 1e-9)
    assert hit.sum() > 200 and clear.sum() > 0.95 * len(pix)
    assert np.array_equal(r["surface"][clear].astype(np.int64), want[clear])
    m = clear & hit
    np.testing.assert_allclose(r["exit_pos"][m], eye + ta[m, None] * d[m], atol=1e-12)
    assert len(set(want[m].tolist())) >= 3            # several faces are seen


def test_slanted_two_triangle_board_in_catenary_medium(oracle_lib):
    G = np.array([0.0, 0.0, -0.03])
    a0 = 0.01
    md = oracle_lib.Medium(oracle_lib.MEDIUM_LINEAR, BOX, [a0, *G])
    view = W.View(eye=W._f32([0.45, -0.6, 0.40]),
                  fwd=W._f32(np.array([0.04, 1.0, 0.07]) / np.linalg.norm([0.04, 1.0, 0.07])),
                  up=W._f32([0, 0, 1]), vfov=float(np.float32(math.radians(1.0))), width=1, height=1,
                  plane_p=W._f32([0.5, 4.0, 0.5]), plane_n=W._f32([0, -1, 0]))
    board = W.quads([((0.1, 0.45, 0.0), (0.8, 0.35, 0.0), (0.0, 0.0, 1.0))])
    tris, surf = _split(board, 1)
    o, ea, eb = np.asarray(board[0], np.float64)
    nrm = np.cross(ea, eb)
    d = oracle_lib.pixel_rays(view, np.array([[0, 0]]))[0]
    eye = np.asarray(view.eye, np.float64)
    x0 = eye + ((0.0 - eye[1]) / d[1]) * d
    path = _catenary_path(1.0 + a0 + G @ x0, G, x0, d)
    exact = path(brentq(lambda xi: (path(xi) - o) @ nrm, 0.0, 1.5))
    errs, hits = [], []
    for ds in (0.02, 0.01, 0.005, 0.0025):
        r = oracle_lib.trace_mesh(md, [view], tris, surf, _step(ds))
        assert r["surface"][0] == 1
        hits.append(r["exit_pos"][0])
        assert abs((r["exit_pos"][0] - o) @ nrm) < 1e-12
        errs.append(np.linalg.norm(r["exit_pos"][0] - exact))
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert errs[0] > 1e-5 and np.all(ratios > 1.6) and np.all(ratios < 2.4), ratios
    assert np.linalg.norm(2.0 * hits[-1] - hits[-2] - exact) < 0.05 * errs[-1]
