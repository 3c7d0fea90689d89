"""The achievable-bandwidth microbenchmarks behind the marcher's roofline.

hz_membench streams a buffer; hz_membench_gather replays the marcher's access
pattern (8-corner gathers along the views' own pinhole rays, walked straight)
with no arithmetic.  Both must return a finite positive rate, count the
samples the straight walks take, and reject arguments outside their
documented ranges without launching anything.
"""
import math

import numpy as np
import pytest

from paper_2603_02048_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def haze():
    from paper_2603_02048_amd import haze as h
    h.lib()
    return h


def test_membench_read(haze):
    with haze.Context(0) as ctx:
        g = ctx.membench(8 << 20, 3)
        assert math.isfinite(g) and g > 0.0


def _expected_samples(grid, views, step):
    """Samples of the straight walks, counted on the host in float64 (the
    kernel's float32 entry/exit parameters can move a count by one)."""
    total = 0
    lo, hi = np.asarray(grid.lo, float), np.asarray(grid.hi, float)
    for v in views:
        fwd = np.asarray(v.fwd, float) / np.linalg.norm(v.fwd)
        r = np.cross(fwd, np.asarray(v.up, float))
        r /= np.linalg.norm(r)
        u = np.cross(r, fwd)
        fpx = 0.5 * v.height / math.tan(0.5 * float(v.vfov))
        p, q = np.meshgrid(np.arange(v.width) + 0.5 - 0.5 * v.width, np.arange(v.height) + 0.5 - 0.5 * v.height)
        d = fpx * fwd[None, None] + p[..., None] * r[None, None] - q[..., None] * u[None, None]
        d /= np.linalg.norm(d, axis=2, keepdims=True)
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (lo - np.asarray(v.eye, float)) / d
            t2 = (hi - np.asarray(v.eye, float)) / d
        a = np.max(np.minimum(t1, t2), axis=2)
        b = np.min(np.maximum(t1, t2), axis=2)
        hit = (a <= b) & (b > 0)
        a = np.maximum(a, 0.0)
        n = np.ceil((b - a) / step)
        total += int(n[hit].sum())
    return total


@pytest.mark.parametrize("voxel_bytes", [16, 8])
def test_membench_gather(haze, voxel_bytes):
    print(f"case membench_gather: 64^3, {voxel_bytes} B voxels, two ring views of 96x64", flush=True)
    grid = W.make_grid((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (64, 64, 64))
    views = [W.ring_view(grid.lo, grid.hi, az, 2.0, 96, 64) for az in (0.0, 0.8)]
    step = grid.voxel
    with haze.Context(0) as ctx:
        used0 = ctx.memory()[0]
        g, n = ctx.membench_gather(grid, voxel_bytes, views, step, 3)
        assert math.isfinite(g) and g > 0.0
        want = _expected_samples(grid, views, step)
        assert abs(n - want) <= 0.002 * want, (n, want)
        # a view whose rays all miss the box: no samples
        off = [W.ring_view(grid.lo + 10.0, grid.hi + 10.0, 0.0, 2.0, 16, 8)]
        with pytest.raises(haze.HazeError):
            ctx.membench_gather(grid, voxel_bytes, off, step, 1)   # no samples: refused
        assert ctx.memory()[0] == used0   # the grid and sink are freed


def test_membench_gather_rejects(haze):
    grid = W.make_grid((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (64, 64, 64))
    views = [W.ring_view(grid.lo, grid.hi, 0.0, 2.0, 32, 16)]
    with haze.Context(0) as ctx:
        bad_res = W.make_grid((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (1, 64, 64))
        big = W.make_grid((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (2048, 2048, 512))
        for args in [(grid, 12, views, grid.voxel, 1), (bad_res, 16, views, grid.voxel, 1),
                     (big, 16, views, grid.voxel, 1), (grid, 16, views, 0.0, 1), (grid, 16, views, 1e9, 1),
                     (grid, 16, views, grid.voxel, 0)]:
            with pytest.raises(haze.HazeError) as e:
                ctx.membench_gather(*args)
            assert e.value.status == haze.E_INVALID, args
