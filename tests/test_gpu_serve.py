"""Serving loop on the GPU: continuous batching of mixed multi-view requests.

Every request's outputs must be bitwise identical to a solo hz_trace_views of
the same views, however the scheduler batched it; admission waits for HBM
budget; errors are reported per ticket.
"""
import time

import numpy as np
import pytest
import torch

from paper_2603_02048_amd import workloads as W
from tests.parity import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def haze():
    from paper_2603_02048_amd import haze as h
    h.lib()
    return h


def _wait(ctx, tickets, timeout=60.0):
    lat = {}
    t0 = time.time()
    while len(lat) < len(tickets):
        for t in tickets:
            if t not in lat:
                v = ctx.poll(t)
                if v is not None:
                    lat[t] = v
        assert time.time() - t0 < timeout, "requests did not complete"
        time.sleep(0.001)
    return lat


def _frames(ctx, haze, n=3):
    fields = []
    for k in range(n):
        wl = W.make_small(seed=10 + k, n=4000, width=8, height=8, nviews=1).with_k_gd(150.0)
        fields.append((wl, ctx.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)))
    return fields


def _random_request(rng, grid):
    sizes = [(37, 23), (64, 40), (20, 12), (8, 8)]
    nv = int(rng.integers(1, 4))
    w, h = sizes[int(rng.integers(0, len(sizes)))]
    radius = float(rng.uniform(0.9, 1.6))
    az0 = float(rng.uniform(0, 2 * np.pi))
    return [W.ring_view(grid.lo, grid.hi, az0 + 2 * np.pi * k / nv, radius, w, h, backdrop_beyond=0.6)
            for k in range(nv)]


def test_serve_mix_equals_solo(haze):
    ctx = haze.Context(0)
    try:
        frames = _frames(ctx, haze)
        grid = frames[0][0].grid
        st_a, st_u = W.make_steps(grid)
        ctx.server_start(slots=3, max_batch_rays=1 << 16)
        rng = np.random.default_rng(0)
        reqs = []
        for i in range(24):
            fi = int(rng.integers(0, len(frames)))
            views = _random_request(rng, grid)
            st = st_a if rng.random() < 0.7 else st_u
            t = ctx.submit(frames[fi][1], views, st)
            reqs.append((t, fi, views, st))
            if i % 5 == 4:
                time.sleep(0.002)   # some requests arrive while others run
        lat = _wait(ctx, [r[0] for r in reqs])
        assert all(v > 0 for v in lat.values())
        for t, fi, views, st in reqs:
            got = to_np(ctx.request_outputs(t))
            solo = to_np(ctx.trace_views(frames[fi][1], views, st))
            torch.cuda.synchronize()
            for k in solo:
                assert np.array_equal(got[k].view(np.uint8), solo[k].view(np.uint8)), (t, k)
            assert (got["steps"] > 0).any()
            ctx.request_release(t)
        ms, n = ctx.profile_read("serve_batch")
        print(f"serve: {len(reqs)} requests, latency p50 {np.percentile(list(lat.values()), 50) * 1e3:.2f} ms, "
              f"max {max(lat.values()) * 1e3:.2f} ms", flush=True)
        ctx.server_stop()
    finally:
        ctx.close()


def test_serve_budget_admission_and_errors(haze):
    wl = W.make_small(seed=3, n=3000, width=8, height=8, nviews=1)
    # budget: the field, one launch slot's scratch and outputs for ~1.5 requests
    views = [W.ring_view(wl.grid.lo, wl.grid.hi, 0.3, 1.2, 256, 128)]
    per_req = 256 * 128 * 38
    probe = haze.Context(0)
    f0 = probe.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
    used_with_field, _ = probe.memory()
    probe.close()
    max_batch = 256 * 128
    # slot scratch: hit list (4 B) and length bins (1 B) per queue slot, two
    # sets of 65 counters 256 B apart
    budget = used_with_field + 5 * max_batch + 2 * 65 * 256 + 64 * 1024 + int(1.5 * per_req)
    ctx = haze.Context(0, budget_bytes=budget)
    try:
        f = ctx.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
        with pytest.raises(haze.HazeError) as e:
            ctx.submit(f, views, wl.step_adaptive)
        assert e.value.status == haze.E_INVALID          # no server yet
        ctx.server_start(slots=1, max_batch_rays=max_batch)
        big = [W.ring_view(wl.grid.lo, wl.grid.hi, 0.3, 1.2, 512, 512)]
        with pytest.raises(haze.HazeError) as e:
            ctx.submit(f, big, wl.step_adaptive)        # larger than a launch
        assert e.value.status == haze.E_BUDGET
        with pytest.raises(haze.HazeError) as e:
            ctx.poll(987654321)
        assert e.value.status == haze.E_NOTFOUND
        tickets = [ctx.submit(f, views, wl.step_adaptive) for _ in range(3)]
        done = _wait(ctx, tickets[:1])
        time.sleep(0.05)
        # the second request cannot get output memory while the first holds it
        assert ctx.poll(tickets[1]) is None
        first = to_np(ctx.request_outputs(tickets[0]))
        ctx.request_release(tickets[0])
        _wait(ctx, tickets[1:2])
        ctx.request_release(tickets[1])
        _wait(ctx, tickets[2:3])
        last = to_np(ctx.request_outputs(tickets[2]))
        for k in first:
            assert np.array_equal(first[k].view(np.uint8), last[k].view(np.uint8))
        ctx.request_release(tickets[2])
        with pytest.raises(haze.HazeError) as e:
            ctx.request_release(tickets[2])
        assert e.value.status == haze.E_NOTFOUND
        ctx.server_stop()
    finally:
        ctx.close()


def test_serve_release_refused_while_waiting(haze):
    """hz_field_release and hz_mesh_release refuse a field or mesh that a
    request still waiting in the serving loop reads (HZ_E_INVALID), and both
    succeed once the request has run.  The request is held back by the HBM
    budget: an earlier request's outputs occupy it until released."""
    from tests.test_gpu_scene import _boards
    print("case serve release while waiting: 256x128 mesh requests, one slot", flush=True)
    wl = W.make_small(seed=3, n=3000, width=8, height=8, nviews=1)
    st = wl.step_adaptive
    views = [W.ring_view(wl.grid.lo, wl.grid.hi, 0.3, 1.2, 256, 128)]
    tris = W.tessellate_quads(_boards(wl.grid.lo, wl.grid.hi), 2)
    per_req = 256 * 128 * 38          # the request's outputs, its surface array included
    max_batch = 256 * 128
    probe = haze.Context(0)
    f0 = probe.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
    m0 = probe.mesh_create(*tris, reach=st.ds_max)
    used, _ = probe.memory()
    probe.close()
    budget = used + 5 * max_batch + 2 * 65 * 256 + 64 * 1024 + int(1.5 * per_req)
    ctx = haze.Context(0, budget_bytes=budget)
    try:
        f = ctx.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
        m = ctx.mesh_create(*tris, reach=st.ds_max)
        ctx.server_start(slots=1, max_batch_rays=max_batch)
        t0 = ctx.submit(f, views, st, mesh=m)
        _wait(ctx, [t0])
        t1 = ctx.submit(f, views, st, mesh=m)
        time.sleep(0.05)
        assert ctx.poll(t1) is None                     # waits for output memory
        for obj in (f, m):
            with pytest.raises(haze.HazeError) as e:
                obj.release()
            assert e.value.status == haze.E_INVALID
            assert obj.handle
        first = to_np(ctx.request_outputs(t0))
        ctx.request_release(t0)
        _wait(ctx, [t1])
        second = to_np(ctx.request_outputs(t1))
        for k in first:
            assert np.array_equal(first[k].view(np.uint8), second[k].view(np.uint8)), k
        m.release()                                     # launched: waits for its work
        f.release()
        ctx.request_release(t1)
        ctx.server_stop()
    finally:
        ctx.close()


def test_serve_slots_overlap_on_device(haze):
    """Batches on two slots run at the same time on the device: requests for
    fields of different grids cannot share a launch, so each pair goes to two
    slots, and the dispatch timestamps of the two launches overlap."""
    print("case serve overlap: 3 pairs of 64x32 requests, two grids, 1/64-voxel uniform steps", flush=True)
    ctx = haze.Context(0)
    try:
        a = W.make_small(seed=21, n=4000, res=(48, 40, 32), width=8, height=8, nviews=1)
        b = W.make_small(seed=22, n=4000, res=(40, 48, 32), width=8, height=8, nviews=1)
        fa = ctx.splat_index_field(haze.upload_particles(a.particles), a.grid, a.k_gd, a.h)
        fb = ctx.splat_index_field(haze.upload_particles(b.particles), b.grid, b.k_gd, b.h)
        torch.cuda.synchronize()
        # few rays (8 march workgroups each), many steps: each launch occupies
        # a few CUs for about a millisecond
        _, st_a = W.make_steps(a.grid, uniform_vox=1.0 / 64.0)
        _, st_b = W.make_steps(b.grid, uniform_vox=1.0 / 64.0)
        va = [W.ring_view(a.grid.lo, a.grid.hi, 0.4, 1.2, 64, 32)]
        vb = [W.ring_view(b.grid.lo, b.grid.hi, 1.1, 1.2, 64, 32)]
        ctx.server_start(slots=2, max_batch_rays=1 << 16)
        overlaps = []
        for rep in range(3):
            ta = ctx.submit(fa, va, st_a)
            tb = ctx.submit(fb, vb, st_b)
            _wait(ctx, [ta, tb])
            (s0, e0), (s1, e1) = ctx.request_timing(ta), ctx.request_timing(tb)
            assert e0 > s0 and e1 > s1
            ov = min(e0, e1) - max(s0, s1)
            overlaps.append(ov / min(e0 - s0, e1 - s1))
            print(f"pair {rep}: A [{s0:.3f}, {e0:.3f}] ms, B [{s1:.3f}, {e1:.3f}] ms, overlap {overlaps[-1]:.2f} "
                  f"of the shorter", flush=True)
            got = to_np(ctx.request_outputs(ta))
            solo = to_np(ctx.trace_views(fa, va, st_a))
            torch.cuda.synchronize()
            for k in solo:
                assert np.array_equal(got[k].view(np.uint8), solo[k].view(np.uint8)), k
            ctx.request_release(ta)
            ctx.request_release(tb)
        assert min(overlaps) > 0.2, overlaps
        ctx.server_stop()
    finally:
        ctx.close()


def test_serve_scene_boards_mix_equals_solo(haze):
    """Requests with scene boards (hz_submit_scene) and without, interleaved:
    each result bitwise equal to a solo hz_trace_scene of the same views and
    boards (no boards: the backdrop only, surface 0 or 255)."""
    from tests.test_gpu_scene import _boards
    print("case serve scene boards: 18 requests, three board sets and none", flush=True)
    ctx = haze.Context(0)
    try:
        frames = _frames(ctx, haze, n=2)
        grid = frames[0][0].grid
        st_a, st_u = W.make_steps(grid)
        boards = _boards(grid.lo, grid.hi)
        sets = [None, boards, boards[:2], boards[1:]]
        ctx.server_start(slots=3, max_batch_rays=1 << 16)
        rng = np.random.default_rng(4)
        reqs = []
        for i in range(18):
            fi = int(rng.integers(0, len(frames)))
            views = _random_request(rng, grid)
            q = sets[int(rng.integers(0, len(sets)))]
            st = st_a if rng.random() < 0.6 else st_u
            reqs.append((ctx.submit(frames[fi][1], views, st, quads=q), fi, views, q, st))
        _wait(ctx, [r[0] for r in reqs])
        seen = set()
        for t, fi, views, q, st in reqs:
            got = to_np(ctx.request_outputs(t))
            solo = to_np(ctx.trace_scene(frames[fi][1], views, np.zeros((0, 3, 3)) if q is None else q, st))
            torch.cuda.synchronize()
            for k in solo:
                assert np.array_equal(got[k].view(np.uint8), solo[k].view(np.uint8)), (t, k)
            seen.update(np.unique(got["surface"]).tolist())
            ctx.request_release(t)
        assert {0, 1, 2}.issubset(seen), seen
        ctx.server_stop()
    finally:
        ctx.close()


def test_serve_mesh_mix_equals_solo(haze):
    """Requests against two triangle meshes (hz_submit_mesh) and without a
    scene, interleaved: each result bitwise equal to a solo hz_trace_mesh
    (or hz_trace_views) of the same views; the meshes' surfaces are met."""
    from tests.test_gpu_scene import _boards
    print("case serve meshes: 18 requests, two meshes and none", flush=True)
    ctx = haze.Context(0)
    try:
        frames = _frames(ctx, haze, n=2)
        grid = frames[0][0].grid
        st_a, st_u = W.make_steps(grid)
        reach = max(st_a.ds_max, st_u.ds_uniform)
        boards = _boards(grid.lo, grid.hi)
        meshes = [None, ctx.mesh_create(*W.tessellate_quads(boards, 4), reach=reach),
                  ctx.mesh_create(*W.tessellate_quads(boards[1:], 3), reach=reach)]
        ctx.server_start(slots=3, max_batch_rays=1 << 16)
        rng = np.random.default_rng(6)
        reqs = []
        for i in range(18):
            fi = int(rng.integers(0, len(frames)))
            views = _random_request(rng, grid)
            m = meshes[int(rng.integers(0, len(meshes)))]
            st = st_a if rng.random() < 0.6 else st_u
            reqs.append((ctx.submit(frames[fi][1], views, st, mesh=m), fi, views, m, st))
        _wait(ctx, [r[0] for r in reqs])
        seen = set()
        for t, fi, views, m, st in reqs:
            got = to_np(ctx.request_outputs(t))
            if m is None:
                solo = to_np(ctx.trace_views(frames[fi][1], views, st))
            else:
                solo = to_np(ctx.trace_mesh(frames[fi][1], views, m, st))
                seen.update(np.unique(got["surface"]).tolist())
            torch.cuda.synchronize()
            for k in solo:
                assert np.array_equal(got[k].view(np.uint8), solo[k].view(np.uint8)), (t, k)
            ctx.request_release(t)
        assert {1, 2}.issubset(seen), seen
        ctx.server_stop()
        for m in meshes[1:]:
            m.release()
    finally:
        ctx.close()


def test_serve_mesh_errors(haze):
    """hz_submit_mesh refuses a mesh of another context and steps longer than
    the mesh's reach, at submission."""
    from tests.test_gpu_scene import _boards
    print("case serve mesh errors", flush=True)
    ctx, other = haze.Context(0), haze.Context(0)
    try:
        wl, field = _frames(ctx, haze, n=1)[0]
        st_a, _ = W.make_steps(wl.grid)
        tris = W.tessellate_quads(_boards(wl.grid.lo, wl.grid.hi), 2)
        short = ctx.mesh_create(*tris, reach=0.5 * st_a.ds_max)
        foreign = other.mesh_create(*tris, reach=st_a.ds_max)
        ctx.server_start(slots=1, max_batch_rays=1 << 16)
        views = _random_request(np.random.default_rng(1), wl.grid)
        with pytest.raises(haze.HazeError) as e:
            ctx.submit(field, views, st_a, mesh=short)
        assert e.value.status == haze.E_INVALID
        with pytest.raises(haze.HazeError) as e:
            ctx.submit(field, views, st_a, mesh=foreign)
        assert e.value.status == haze.E_INVALID
        ctx.server_stop()
        short.release()
        foreign.release()
    finally:
        other.close()
        ctx.close()
