"""Failure paths forced from the host: every kernel still exits normally.

The one-pass cell-list scan waits (boundedly) for the tile sums of lower
tiles.  The fault-test knob makes those waits look for tags that never come
with a short bound, so they give up: the library must report HZ_E_DEVICE,
refuse the field the call built, and work normally afterwards."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_02048_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def haze():
    from paper_2603_02048_amd import haze as h
    h.lib()
    return h


def test_scan_give_up_is_reported(haze):
    print("case scan fault test: 4000 particles, h = 0.01 (43 scan tiles)", flush=True)
    ctx = haze.Context(0)
    try:
        wl = W.make_small(seed=7, n=4000, h=0.01)
        parts = haze.upload_particles(wl.particles)
        ctx.tune("splat.scan_fault_test", 1)
        bad = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
        torch.cuda.synchronize()
        ctx.tune("splat.scan_fault_test", 0)
        with pytest.raises(haze.HazeError) as e:
            ctx.field_read(bad)
        assert e.value.status == haze.E_DEVICE and "gave up" in str(e.value), str(e.value)
        # reported once; the field itself stays unusable
        with pytest.raises(haze.HazeError) as e:
            ctx.trace_views(bad, wl.views, wl.step_adaptive)
        assert e.value.status == haze.E_DEVICE and "scan failed" in str(e.value), str(e.value)
        bad.release()
        good = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
        dn = ctx.field_read(good)[0].cpu().numpy().astype(np.float64)
        ref = oracle.splat(wl.particles, wl.grid, wl.k_gd, wl.h)
        err = float(np.max(np.abs(dn - ref)) / np.max(np.abs(ref)))
        print(f"after the fault: rel |d dn| = {err:.2e}", flush=True)
        assert err <= 1e-5
        good.release()
    finally:
        ctx.close()
