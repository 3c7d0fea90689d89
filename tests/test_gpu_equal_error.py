"""Adaptive vs uniform step at equal displacement-map error (Sec. 3.3.3, Eq. 18;
the theta_max accuracy/speed trade-off of Sec. 4.1), through the protocol the
benchmark reports (bench.equal_error_protocol):

  1. E_u = RMS (and max) |disp_GPU,uniform(0.25 voxel) - disp_ref| on a
     4,096-ray subset, where disp_ref is the oracle's converged solution of the
     continuous ray equation through the same FP64 field (step halving +
     Richardson extrapolation).
  2. Sweep theta_max down from the paper's 0.003 (h_max = 1 voxel) and bisect
     in log(theta) for the largest theta whose adaptive RMS error E_a <= E_u.
  3. Time both full-frame traces (ray generation + march) and report rays/s,
     ray-steps/s and the speed ratio at that theta.
Run on the config-2 physical field and on its K_GD x 250 stress variant, where
the adaptive rule binds at the paper's theta.  The numbers are printed as one
JSON line per field.
"""
import json

import pytest

import bench
import oracle
from paper_2603_02048_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def haze():
    from paper_2603_02048_amd import haze as h
    h.lib()
    return h


@pytest.mark.parametrize("kgd", [1.0, 250.0])
def test_equal_error_protocol(haze, kgd):
    wl = W.make_config(2).with_k_gd(kgd)
    print(f"case equal-error config2 kgd x{kgd}", flush=True)
    ctx = haze.Context(0)
    try:
        field = ctx.splat_index_field(haze.upload_particles(wl.particles), wl.grid, wl.k_gd, wl.h)
        md = oracle.field(wl.particles, wl.grid, wl.k_gd, wl.h)
        res = bench.equal_error_protocol(oracle, ctx, field, md, wl)
        assert "error" not in res, res
        res["field"] = f"config2 kgd x{kgd:g}"
        print("EQUAL_ERROR " + json.dumps(res), flush=True)
        # the physical field's reference converges everywhere; on the stress
        # field some rays pass near caustics (reported, not asserted)
        if kgd == 1.0:
            assert res["reference_converged_fraction"] > 0.99
        assert res["E_adaptive_px"]["rms"] <= res["E_uniform_px"]["rms"]
        field.release()
    finally:
        ctx.close()
