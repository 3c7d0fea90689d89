"""Library calls spread over several HIP streams.

Fields, the splat and trace scratch buffers and the pool of released field
memory are shared by calls on any stream.  Every call records one completion
event; a call on another stream orders itself after the calls whose memory it
reuses, and a read of a field after the call that wrote it.  The same frames
are run serially and spread over streams with no host synchronisation in
between, and every output must be bitwise identical.
"""
import numpy as np
import pytest
import torch

from paper_2603_02048_amd import workloads as W

pytestmark = pytest.mark.gpu

NFRAMES = 6


@pytest.fixture(scope="module")
def haze():
    from paper_2603_02048_amd import haze as h
    h.lib()
    return h


@pytest.fixture(scope="module")
def frames(haze):
    # different particles every frame, so that a trace of the wrong frame's
    # field (or of one being overwritten) changes the output
    wls = [W.make_small(seed=20 + k, n=150_000, lo=(0.0, 0.0, 0.0), hi=(0.5, 0.5, 0.5), res=(96, 96, 96),
                        h=0.02, width=320, height=240, nviews=2) for k in range(NFRAMES)]
    parts = [haze.upload_particles(wl.particles) for wl in wls]
    torch.cuda.synchronize()
    return wls, parts


def _nrays(wl):
    return sum(v.width * v.height for v in wl.views)


def _bits(out):
    return {k: v.detach().cpu().numpy().view(np.uint8) for k, v in out.items()}


def _run(haze, ctx, wls, parts, streams):
    outs = [haze.alloc_outputs(_nrays(wl)) for wl in wls]
    torch.cuda.synchronize()
    for k, wl in enumerate(wls):
        with torch.cuda.stream(streams[k % len(streams)]):
            f = ctx.splat_index_field(parts[k], wl.grid, wl.k_gd, wl.h)
            ctx.trace_views(f, wl.views, wl.step_adaptive, out=outs[k])
            f.release()
    torch.cuda.synchronize()
    return [_bits(o) for o in outs]


def _field_bytes(wl):
    return int(np.prod(wl.grid.res)) * 16


def _assert_same(a, b, what):
    for k, (x, y) in enumerate(zip(a, b)):
        for name in x:
            assert np.array_equal(x[name], y[name]), f"{what}: frame {k} {name} differs"


def test_frames_on_two_streams_match_serial(haze, frames):
    wls, parts = frames
    print(f"case streams: {NFRAMES} frames, 150000 particles, 96^3, 2 views 320x240", flush=True)
    with haze.Context(0) as ctx:
        serial = _run(haze, ctx, wls, parts, [torch.cuda.current_stream()])
        used_serial = ctx.memory()[0]
    with haze.Context(0) as ctx:
        two = _run(haze, ctx, wls, parts, [torch.cuda.Stream(), torch.cuda.Stream()])
        used_two = ctx.memory()[0]
    _assert_same(serial, two, "two streams")
    # a released field still in use on the other stream is not reused while the
    # budget has room: the frames get a second block and can overlap
    assert used_two >= used_serial + _field_bytes(wls[0])


def test_frames_on_two_streams_tight_budget(haze, frames):
    # with room for one field block only, each frame reuses the block the
    # other stream's frame is still tracing, after that trace
    wls, parts = frames
    with haze.Context(0) as ctx:
        serial = _run(haze, ctx, wls[:1], parts[:1], [torch.cuda.current_stream()])
        budget = ctx.memory()[0] + _field_bytes(wls[0]) // 2
    print(f"case streams tight budget: {budget} bytes", flush=True)
    with haze.Context(0, budget_bytes=budget) as ctx:
        ref = _run(haze, ctx, wls, parts, [torch.cuda.current_stream()])
        three = _run(haze, ctx, wls, parts, [torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()])
        assert ctx.memory()[0] <= budget
    _assert_same(serial, ref[:1], "tight budget, serial")
    _assert_same(ref, three, "tight budget, three streams")


def test_field_written_on_one_stream_read_on_others(haze, frames):
    wls, parts = frames
    wl = wls[0]
    with haze.Context(0) as ctx:
        out_ref = haze.alloc_outputs(_nrays(wl))
        f = ctx.splat_index_field(parts[0], wl.grid, wl.k_gd, wl.h)
        ctx.trace_views(f, wl.views, wl.step_adaptive, out=out_ref)
        arrs_ref = [a.clone() for a in ctx.field_read(f)]
        torch.cuda.synchronize()
        f.release()
        ref = _bits(out_ref)
        a, b, c = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
        out = haze.alloc_outputs(_nrays(wl))
        torch.cuda.synchronize()
        with torch.cuda.stream(a):
            f = ctx.splat_index_field(parts[0], wl.grid, wl.k_gd, wl.h)
        with torch.cuda.stream(b):
            ctx.trace_views(f, wl.views, wl.step_adaptive, out=out)
        with torch.cuda.stream(c):
            arrs = ctx.field_read(f)
        torch.cuda.synchronize()
        f.release()
        got = _bits(out)
        for name in ref:
            assert np.array_equal(ref[name], got[name]), name
        for x, y in zip(arrs_ref, arrs):
            assert torch.equal(x.view(torch.int32), y.view(torch.int32))


def test_many_calls_over_streams(haze):
    # more calls than the 64 completion events the context keeps in its ring:
    # issuing a call's event waits for the one 64 calls back, and older calls
    # count as complete; outputs still match a serial run bit for bit
    wl = W.make_small(seed=40, n=4000, width=24, height=16, nviews=1)
    parts = haze.upload_particles(wl.particles)
    torch.cuda.synchronize()
    nframes = 90
    print(f"case streams: {nframes} small frames over three streams", flush=True)
    with haze.Context(0) as ctx:
        ref = _run(haze, ctx, [wl], [parts], [torch.cuda.current_stream()])[0]
        streams = [torch.cuda.Stream() for _ in range(3)]
        outs = [haze.alloc_outputs(_nrays(wl)) for _ in range(nframes)]
        torch.cuda.synchronize()
        for k in range(nframes):
            with torch.cuda.stream(streams[k % 3]):
                f = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
                ctx.trace_views(f, wl.views, wl.step_adaptive, out=outs[k])
                f.release()
        torch.cuda.synchronize()
    for k in range(nframes):
        got = _bits(outs[k])
        for name in ref:
            assert np.array_equal(ref[name], got[name]), (k, name)


def test_profile_select(haze):
    wl = W.make_small(seed=41, n=3000)
    parts = haze.upload_particles(wl.particles)
    with haze.Context(0) as ctx:
        with pytest.raises(haze.HazeError) as e:
            ctx.profile_select("splat,nonsense")
        assert e.value.status == haze.E_INVALID
        ctx.profile_select("splat")
        ctx.profile_enable(True)
        f = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h)
        ctx.trace_views(f, wl.views, wl.step_adaptive)
        torch.cuda.synchronize()
        ctx.profile_enable(False)
        ms, n = ctx.profile_read("splat")
        assert n == 1 and ms > 0.0
        for g in ("cell_list", "grad_pack", "raygen", "march"):
            assert ctx.profile_read(g)[1] == 0, g
        ctx.profile_select(None)
        ctx.profile_enable(True)
        ctx.trace_views(f, wl.views, wl.step_adaptive)
        torch.cuda.synchronize()
        ctx.profile_enable(False)
        assert ctx.profile_read("march")[1] == 1 and ctx.profile_read("raygen")[1] == 1
        f.release()
