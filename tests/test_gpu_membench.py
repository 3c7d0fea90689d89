"""The achievable-bandwidth microbenchmarks behind the marcher's roofline.

hz_membench streams a buffer; hz_membench_gather replays the marcher's access
pattern (8-corner gathers along straight rays) with no arithmetic.  Both must
return a finite positive rate, and reject arguments outside their documented
ranges without launching anything.
"""
import math

import pytest

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


@pytest.mark.parametrize("voxel_bytes", [16, 8])
def test_membench_gather(haze, voxel_bytes):
    print(f"case membench_gather: 64^3, {voxel_bytes} B voxels, 5000 rays x 60 steps", flush=True)
    with haze.Context(0) as ctx:
        used0 = ctx.memory()[0]
        g = ctx.membench_gather((64, 64, 64), voxel_bytes, 5000, 60, 3)
        assert math.isfinite(g) and g > 0.0
        # rays that run past the far face read clamped (in-grid) cells
        g2 = ctx.membench_gather((2, 3, 2), voxel_bytes, 70, 9, 1)
        assert math.isfinite(g2) and g2 > 0.0
        assert ctx.memory()[0] == used0   # the grid and sink are freed


def test_membench_gather_rejects(haze):
    with haze.Context(0) as ctx:
        for args in [((64, 64, 64), 12, 100, 10, 1), ((1, 64, 64), 16, 100, 10, 1), ((64, 64, 70000), 16, 100, 10, 1),
                     ((64, 64, 64), 16, 0, 10, 1), ((64, 64, 64), 16, 100, 0, 1), ((64, 64, 64), 16, 100, 10, 0),
                     ((2048, 2048, 512), 16, 100, 10, 1)]:
            with pytest.raises(haze.HazeError) as e:
                ctx.membench_gather(*args)
            assert e.value.status == haze.E_INVALID, args
