"""hz_trace_views_noalloc: the tracer with its launch scratch in the library's
static device array, for callers that cannot allocate.  Two calls in a row
(the second with a smaller input) must give results bitwise equal to
hz_trace_views on the same inputs, without the context allocating anything;
sizes beyond the static array are refused before any work."""
import ctypes as C

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


def _equal(a: dict, b: dict, label: str):
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), f"{label}: {k} differs"


def test_noalloc_matches_trace_views(haze):
    print("case noalloc: two calls (3 views 45x29, then 1 view 17x11), full and subset", flush=True)
    ctx = haze.Context(0)
    try:
        wl = W.make_small(seed=3, n=4000, width=45, height=29, nviews=3).with_k_gd(200.0)
        field = ctx.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
        small = W.make_small(seed=4, n=4000, width=17, height=11, nviews=1)
        torch.cuda.synchronize()
        used0, _ = ctx.memory()
        # first call: three views, all rays
        got1 = to_np(ctx.trace_views_noalloc(field, wl.views, wl.step_adaptive))
        # second call, smaller: one view of another size, uniform step
        got2 = to_np(ctx.trace_views_noalloc(field, small.views, wl.step_uniform))
        # third: a subset of ray ids of the first input
        ids = torch.from_numpy(np.array([0, 5, 44, 45, 1304, 2 * 1305 + 7, 3 * 1305 - 1], np.int64)).cuda()
        got3 = to_np(ctx.trace_views_noalloc(field, wl.views, wl.step_adaptive, ray_ids=ids))
        torch.cuda.synchronize()
        used1, _ = ctx.memory()
        assert used1 == used0, "the no-alloc call changed the context's device memory"
        ref1 = to_np(ctx.trace_views(field, wl.views, wl.step_adaptive))
        ref2 = to_np(ctx.trace_views(field, small.views, wl.step_uniform))
        ref3 = to_np(ctx.trace_views(field, wl.views, wl.step_adaptive, ray_ids=ids))
        torch.cuda.synchronize()
        assert int((ref1["steps"] > 0).sum()) > 100
        _equal(got1, ref1, "first call")
        _equal(got2, ref2, "second (smaller) call")
        _equal(got3, ref3, "subset call")
        field.release()
    finally:
        ctx.close()


def test_noalloc_limits(haze):
    print("case noalloc limits: 65 views, 2^23 + 64 slots", flush=True)
    ctx = haze.Context(0)
    try:
        wl = W.make_small(seed=5, n=2000, width=8, height=8, nviews=1)
        field = ctx.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
        torch.cuda.synchronize()
        views = haze.make_views([wl.views[0]] * 65)
        st = haze.make_step(wl.step_adaptive)
        out = haze.hz_trace_out()
        L = haze.lib()
        rc = L.hz_trace_views_noalloc(C.c_void_p(ctx.handle), C.c_void_p(field.handle), views, 65, C.byref(st),
                                      None, 65 * 64, C.byref(out), None)
        assert rc == haze.E_UNSUPPORTED and "limit" in haze.last_error()
        big = W.View(eye=wl.views[0].eye, fwd=wl.views[0].fwd, up=wl.views[0].up, vfov=wl.views[0].vfov,
                     width=4096, height=2049, plane_p=wl.views[0].plane_p, plane_n=wl.views[0].plane_n)
        rc = L.hz_trace_views_noalloc(C.c_void_p(ctx.handle), C.c_void_p(field.handle), haze.make_views([big]), 1,
                                      C.byref(st), None, 4096 * 2049, C.byref(out), None)
        assert rc == haze.E_UNSUPPORTED and "static scratch" in haze.last_error()
        field.release()
    finally:
        ctx.close()
