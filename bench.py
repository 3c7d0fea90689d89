#!/usr/bin/env python
"""Benchmark of the splat-and-trace path on one MI355X.

A step is one pass of the whole path over one frame of synthetic input:
SPH particles -> delta-n grid with its gradient (cell list, splat gather,
gradient/pack) -> every pixel of every view traced through the field (ray
generation, adaptive march, backdrop displacement).  Inputs are resident in
HBM before the timed region starts.

Workload (default): 262,144 particles in a 1 x 1 x 2 m box (main plume + 3
seeded plumes), 128^3 FP32 grid, one 1280x720 view, adaptive step with
theta_max = 0.003 and h_max = 1 voxel; the fixed-step trace (0.25 voxel) is
timed the same way for the adaptive-vs-uniform comparison.

Prints one JSON line (rank 0).  `--gpus N` with N > 1 is refused: the library
and this benchmark run on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rays/s & ray-steps/s, adaptive vs uniform step, 1 MI355X; p50/p99 view latency"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed FP32 instructions (the kernels are built with
# them disabled): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 78.6
BYTES_PER_STEP = {"f32": 128, "f16": 64, "bf16": 64}   # 8 corners x 4 channels
COUNTERS = os.path.join(ROOT, "profiles", "counters_config2_f32.json")
KERNEL_SOURCE = {"k_splat": "paper_2603_02048_amd/csrc/splat.hip",
                 "k_march": "paper_2603_02048_amd/csrc/trace.hip"}


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def code_digest(path: str) -> str:
    """SHA-256 of a source file's code: comments dropped, whitespace runs
    collapsed (so an edit of comments alone keeps the digest)."""
    import hashlib
    import re
    with open(path, encoding="utf-8") as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return hashlib.sha256(" ".join(src.split()).encode()).hexdigest()


def measured_traffic(kernel: str, row: str, config: int, dtype: str):
    """HBM/fabric bytes per launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's readings), or None when
    the workload differs from the counted one or the kernel's code has
    changed since the counters were taken."""
    if config != 2 or dtype != "f32" or not os.path.exists(COUNTERS):
        return None
    with open(COUNTERS) as f:
        c = json.load(f)
    src = KERNEL_SOURCE[kernel]
    if code_digest(os.path.join(ROOT, src)) != c.get("code_sha256", {}).get(src):
        return None
    k = c["kernels"][row]
    return {"bytes": k["fetch_bytes"] + k["write_bytes"], "read_bytes": k["fetch_bytes"],
            "write_bytes": k["write_bytes"], "fetch_scale": c["calibration"]["fetch_scale"],
            "write_scale": c["calibration"]["write_scale"], "source": "profiles/counters_config2_f32.md"}


def per_view_steps(out, wl) -> list:
    """Per view (rays concatenated in view order): rays that enter the volume,
    their mean and largest step count, and a histogram of their step counts in
    bins of 32 steps."""
    steps = out["steps"].cpu().numpy().astype(np.int64)
    res, o = [], 0
    for v in wl.views:
        s = steps[o:o + v.nrays]
        o += v.nrays
        s = s[s > 0]
        hist = np.bincount(s // 32).tolist() if s.size else []
        res.append({"rays_in_volume": int(s.size), "mean_steps": float(s.mean()) if s.size else 0.0,
                    "max_steps": int(s.max()) if s.size else 0, "hist32": hist})
    return res


def time_steps(ctx, torch, fn, steps: int, warmup: int, kernels=(), live=("splat",), live_every: int = 4):
    """ms per step over exactly `steps` steps (host clock between two device
    synchronisations) with the `live` kernel groups timed by their own
    dispatch events inside those steps (every `live_every`-th step, the first
    included); then a second pass of the same length for per-step latencies
    and the other groups' times.  Every timed launch and every event record
    costs the stream microseconds, so the timed pass carries only what the
    roofline needs."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ctx.profile_read("march", reset=True)
    ctx.profile_select(live)
    t0 = time.perf_counter()
    for i in range(steps):
        ctx.profile_enable(i % live_every == 0)
        fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile_enable(False)
    kt_live = {k: ctx.profile_read(k) for k in live}
    ctx.profile_read("march", reset=True)
    ctx.profile_select(None)
    ctx.profile_enable(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ctx.profile_enable(False)
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    kt = {k: ctx.profile_read(k) for k in kernels}
    ctx.profile_read("march", reset=True)
    kt.update(kt_live)
    return (t1 - t0) * 1e3 / steps, per, kt


def count_pairs(torch, parts, grid, h: float) -> int:
    """(voxel, particle) pairs closer than 2h: the splat's algorithmic work units."""
    R = 2.0 * h
    lo = torch.tensor(np.asarray(grid.lo, np.float64), device="cuda")
    sp = torch.tensor(np.asarray(grid.spacing, np.float64), device="cuda")
    res = torch.tensor(np.asarray(grid.res, np.int64), device="cuda")
    p = torch.stack([parts.x, parts.y, parts.z], 1).double()
    base = torch.floor((p - lo) / sp - 0.5).long()
    r = [int(math.ceil(R / float(s))) + 1 for s in grid.spacing]
    total = 0
    for dk in range(-r[2], r[2] + 2):
        for dj in range(-r[1], r[1] + 2):
            off = torch.tensor([0, dj, dk], device="cuda")
            for di in range(-r[0], r[0] + 2):
                off[0] = di
                v = base + off
                inside = ((v >= 0) & (v < res)).all(1)
                c = lo + (v.double() + 0.5) * sp
                d2 = ((c - p) ** 2).sum(1)
                total += int(((d2 < R * R) & inside).sum())
    return total


def pipelined(ctx, torch, make_step_on, steps: int, warmup: int) -> float:
    """ms per frame when frame i+1's splat overlaps frame i's trace (two streams)."""
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for i in range(warmup):
        make_step_on(streams[i % 2], i % 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        make_step_on(streams[i % 2], i % 2)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def serving_leg(haze, torch, W, args) -> dict:
    """Config 5: resident per-frame F16 fields, Poisson requests at 200/s."""
    wl = W.make_config(5)
    ctx = haze.Context(0)
    try:
        fields = []
        for fr in W.advect_frames(wl.particles, wl.grid.lo, wl.grid.hi, nframes=args.serve_frames, device="cuda"):
            parts = haze.upload_particles(fr)
            fields.append(ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h, dtype="f16", store_scale=1e4))
        torch.cuda.synchronize()
        reqs = W.serving_requests(wl.grid.lo, wl.grid.hi, args.serve_seconds, rate_hz=200.0,
                                  nframes=args.serve_frames)
        ctx.server_start(slots=4, max_batch_rays=1 << 24)
        # warm-up: one request of each resolution
        warm = [ctx.submit(fields[0], r.views, wl.step_adaptive) for r in reqs[:3]]
        while any(ctx.poll(t) is None for t in warm):
            time.sleep(0.001)
        for t in warm:
            ctx.request_release(t)
        log(f"bench: serving {len(reqs)} requests over {args.serve_seconds:.1f} s on {len(fields)} resident frames")
        outstanding, lat, rays_done = {}, [], 0
        i = 0
        t0 = time.perf_counter()
        t_last = t0
        while i < len(reqs) or outstanding:
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i].t_arrive <= now:
                r = reqs[i]
                outstanding[ctx.submit(fields[r.frame], r.views, wl.step_adaptive)] = sum(v.nrays for v in r.views)
                i += 1
            for t in list(outstanding):
                v = ctx.poll(t)
                if v is not None:
                    lat.append(v)
                    rays_done += outstanding.pop(t)
                    ctx.request_release(t)
                    t_last = time.perf_counter()
            if now > args.serve_seconds * 4 + 30:
                raise RuntimeError("serving run did not drain")
            time.sleep(0.0002)
        ctx.server_stop()
        lat_ms = np.array(lat) * 1e3
        offered = sum(sum(v.nrays for v in r.views) for r in reqs) / args.serve_seconds
        return {"requests": len(reqs), "frames_resident": len(fields), "field_dtype": "f16",
                "rate_hz": 200.0, "latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                                                 "p99": float(np.percentile(lat_ms, 99)),
                                                 "max": float(lat_ms.max())},
                "sustained_rays_per_s": rays_done / (t_last - t0), "offered_rays_per_s": offered,
                "workload": "config5: 1,048,576 particles advected 60 frames, 256^3 F16 fields resident, "
                            "1-5 views of 640x360/1280x720/1920x1080 per request"}
    finally:
        ctx.close()


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, args) -> dict:
    """The FP64 oracle on the host cores: full splat + a bounded ray sample,
    then the same ray sample (a quarter of it) on one thread."""
    import oracle
    oracle.build()
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    md = oracle.field(wl.particles, wl.grid, wl.k_gd, wl.h, "cells")
    t_splat = time.perf_counter() - t0
    rng = np.random.default_rng(12345)
    ns = min(wl.nrays, args.cpu_rays)
    ids = np.sort(rng.choice(wl.nrays, size=ns, replace=False)).astype(np.int64)
    t0 = time.perf_counter()
    r = oracle.trace_views(md, wl.views, wl.step_adaptive, ray_ids=ids)
    t_trace = time.perf_counter() - t0
    frame_s = t_splat + t_trace * wl.nrays / ns
    oracle.set_num_threads(1)
    try:
        ids1 = ids[::4]
        t0 = time.perf_counter()
        r1 = oracle.trace_views(md, wl.views, wl.step_adaptive, ray_ids=ids1)
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    return {"value": wl.nrays / frame_s, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle: full splat of the {tuple(int(x) for x in wl.grid.res)} grid "
                       f"({t_splat:.2f} s) + {ns} random rays of the {wl.nrays}-ray frame, adaptive "
                       f"({t_trace:.2f} s), scaled to one frame"),
            "ray_steps_per_s": float(r["steps"].sum()) / t_trace, "frame_s": frame_s,
            "voxels_per_s": wl.grid.nvox / t_splat,
            "single_thread": {"rays": int(ids1.size), "rays_per_s": ids1.size / t1,
                              "ray_steps_per_s": float(r1["steps"].sum()) / t1},
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 4])
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--theta", type=float, default=None, help="override theta_max of the adaptive step")
    ap.add_argument("--cpu-rays", type=int, default=65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pairs", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=3.0, help="length of the serving run (0: skip)")
    ap.add_argument("--serve-frames", type=int, default=60)
    ap.add_argument("--no-membench", action="store_true")
    ap.add_argument("--no-pipelined", action="store_true",
                    help="skip the two-stream leg (whose splats overlap marches), e.g. under a kernel-trace profiler")
    ap.add_argument("--splat", default="gather", choices=["gather", "scatter"])
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); on several "
              f"GPUs the path would split views or pixel tiles with the field replicated on each",
              file=sys.stderr)
        return 2

    import torch
    from paper_2603_02048_amd import haze
    from paper_2603_02048_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 3
    torch.cuda.set_device(0)
    wl = W.make_config(args.config)
    st_a, st_u = wl.step_adaptive, wl.step_uniform
    if args.theta is not None:
        st_a, _ = W.make_steps(wl.grid, theta_max=args.theta)
    scale = 1e4 if args.dtype != "f32" else 1.0
    log(f"bench: {wl.name} particles={wl.particles.n} grid={tuple(int(r) for r in wl.grid.res)} "
        f"views={len(wl.views)} rays={wl.nrays} dtype={args.dtype}")

    ctx = haze.Context(0)
    parts = haze.upload_particles(wl.particles)
    out = haze.alloc_outputs(wl.nrays)
    nrays = wl.nrays

    def make_step(st):
        def fn():
            f = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h, dtype=args.dtype, store_scale=scale)
            ctx.trace_views(f, wl.views, st, out=out)
            f.release()
        return fn

    if args.calib_copy_mib > 0:
        a = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {args.calib_copy_mib} MiB done")
        del a, b
    kernels = ("cell_list", "splat", "grad_pack", "raygen", "march")
    ctx.tune("splat.method", 2 if args.splat == "scatter" else 1)
    res = {}
    for name, st in (("adaptive", st_a), ("uniform", st_u)):
        ms, per, kt = time_steps(ctx, torch, make_step(st), args.steps, args.warmup, kernels)
        steps_total = int(out["steps"].sum().item())
        hits = int((out["steps"] > 0).sum().item())
        res[name] = dict(ms=ms, per=per, kt=kt, steps=steps_total, hits=hits, per_view=per_view_steps(out, wl))
        log(f"bench: {name}: {ms:.3f} ms/step (p50 {np.percentile(per, 50):.3f}, p99 {np.percentile(per, 99):.3f}), "
            f"ray-steps {steps_total}, rays in volume {hits}; kernels " +
            ", ".join(f"{k} {v[0] / max(v[1], 1):.3f} ms" for k, v in kt.items()))

    # the other splat kernel, for comparison (same field, same checks in the tests)
    other = "gather" if args.splat == "scatter" else "scatter"
    ctx.tune("splat.method", 2 if other == "scatter" else 1)
    for _ in range(3):
        ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h, dtype=args.dtype, store_scale=scale).release()
    torch.cuda.synchronize()
    ctx.profile_read("splat", reset=True)
    ctx.profile_enable(True)
    for _ in range(10):
        ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h, dtype=args.dtype, store_scale=scale).release()
    torch.cuda.synchronize()
    ctx.profile_enable(False)
    other_ms = ctx.profile_read("splat", reset=True)[0] / 10
    ctx.tune("splat.method", 2 if args.splat == "scatter" else 1)
    log(f"bench: splat kernel {args.splat} {res['adaptive']['kt']['splat'][0] / max(res['adaptive']['kt']['splat'][1], 1):.3f} ms, "
        f"{other} {other_ms:.3f} ms")

    def step_on(stream, k):
        with torch.cuda.stream(stream):
            f = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h, dtype=args.dtype, store_scale=scale)
            ctx.trace_views(f, wl.views, st_a, out=out_pipe[k])
            f.release()
    pipe_ms = None
    if not args.no_pipelined:
        out_pipe = [haze.alloc_outputs(wl.nrays), haze.alloc_outputs(wl.nrays)]
        pipe_ms = pipelined(ctx, torch, step_on, args.steps, args.warmup)
        log(f"bench: pipelined (two streams, splat of frame i+1 under trace of frame i): {pipe_ms:.3f} ms/frame")
    achievable = None
    if not args.no_membench:
        fb = wl.grid.nvox * (16 if args.dtype == "f32" else 8)
        achievable = {"hbm_read_GBps": ctx.membench(4 << 30, 5),
                      "field_sized_read_GBps": ctx.membench(fb, 50),
                      "field_bytes": fb}
        # the marcher's own pattern with no arithmetic: as many straight rays as
        # enter the volume, each taking the mean number of steps of the adaptive trace
        hits = max(1, res["adaptive"]["hits"])
        walk = max(1, round(res["adaptive"]["steps"] / hits))
        achievable["field_sized_gather_GBps"] = ctx.membench_gather(wl.grid.res, fb // wl.grid.nvox, hits, walk, 20)
        achievable["gather_walk"] = {"walkers": hits, "steps": walk}
        log(f"bench: achievable read bandwidth: 4 GiB buffer {achievable['hbm_read_GBps']:.0f} GB/s, "
            f"field-sized ({fb >> 20} MiB) {achievable['field_sized_read_GBps']:.0f} GB/s, "
            f"marcher-pattern gathers ({hits} rays x {walk} steps) {achievable['field_sized_gather_GBps']:.0f} GB/s")

    A, U = res["adaptive"], res["uniform"]
    rays_s = nrays / (A["ms"] * 1e-3)
    # dominant kernel of the adaptive step
    avg = {k: v[0] / max(v[1], 1) for k, v in A["kt"].items()}
    dominant = max(avg, key=avg.get)
    roofline = None
    march_ms = avg["march"]
    march_gbs = A["steps"] * BYTES_PER_STEP[args.dtype] / (march_ms * 1e-3) / 1e9
    march_roof = {"kernel": "k_march", "bound": "hbm", "achieved": march_gbs, "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": march_gbs / HBM_PEAK_GBS, "traffic": None,
                  "per_unit": f"{BYTES_PER_STEP[args.dtype]} B gathered per ray-step (8 corners x 4 channels)",
                  "launch_ms": march_ms,
                  "launch_timing": "dispatch events in a second pass of the same steps (latency pass)"}
    tr = measured_traffic("k_march", "k_march (adaptive)", args.config, args.dtype)
    if tr is not None and args.theta is None:
        march_roof["traffic"] = tr["bytes"]
        march_roof["traffic_detail"] = tr
    if achievable:
        march_roof["achievable_GBps_field_sized"] = achievable["field_sized_read_GBps"]
        march_roof["frac_of_achievable"] = march_gbs / achievable["field_sized_read_GBps"]
        march_roof["achievable_GBps_gather"] = achievable["field_sized_gather_GBps"]
        march_roof["frac_of_achievable_gather"] = march_gbs / achievable["field_sized_gather_GBps"]
    pairs = None
    splat_roof = None
    if not args.no_pairs:
        pairs = count_pairs(torch, parts, wl.grid, wl.h)
        tf = pairs * 25.0 / (avg["splat"] * 1e-3) / 1e12
        splat_roof = {"kernel": "k_splat_scatter" if args.splat == "scatter" else "k_splat", "bound": "alu",
                      "achieved": tf, "peak": FP32_PEAK_TFLOPS,
                      "unit": "TFLOP/s", "frac": tf / FP32_PEAK_TFLOPS, "traffic": None,
                      "per_unit": "25 FP32 flops per (voxel, particle) pair within 2h",
                      "launch_ms": avg["splat"], "units_per_launch": pairs,
                      "launch_timing": "dispatch events of the kernel in every 4th of the timed steps"}
        tr = measured_traffic("k_splat", "k_splat", args.config, args.dtype)
        if tr is not None and args.splat == "gather":
            splat_roof["traffic"] = tr["bytes"]
            splat_roof["traffic_detail"] = tr
    roofline = splat_roof if dominant == "splat" else march_roof

    line = {
        "metric": METRIC,
        "value": rays_s,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": A["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": (f"{wl.name}: {wl.particles.n} SPH particles, "
                                f"{'x'.join(str(int(r)) for r in wl.grid.res)} grid, {len(wl.views)} view(s) "
                                f"{wl.views[0].width}x{wl.views[0].height}, splat + adaptive trace per step"),
                   "theta_max": st_a.theta_max, "h_max_voxel": 1.0, "uniform_step_voxel": 0.25,
                   "parallelism": "single GPU"},
        "ray_steps_per_s": A["steps"] / (A["ms"] * 1e-3),
        "latency_ms": {"p50": float(np.percentile(A["per"], 50)), "p99": float(np.percentile(A["per"], 99))},
        "adaptive": {"rays_per_s": rays_s, "ray_steps": A["steps"], "rays_in_volume": A["hits"],
                     "per_view": A["per_view"],
                     "trace_rays_per_s": nrays / ((avg["raygen"] + avg["march"]) * 1e-3),
                     "trace_ray_steps_per_s": A["steps"] / ((avg["raygen"] + avg["march"]) * 1e-3)},
        "uniform": {"rays_per_s": nrays / (U["ms"] * 1e-3), "ms_per_step": U["ms"], "ray_steps": U["steps"],
                    "ray_steps_per_s": U["steps"] / (U["ms"] * 1e-3),
                    "latency_ms": {"p50": float(np.percentile(U["per"], 50)),
                                   "p99": float(np.percentile(U["per"], 99))}},
        "kernel_ms": {k: round(v, 5) for k, v in avg.items()},
        "splat_ms_by_method": {args.splat: avg["splat"], other: other_ms},
        "march_gather_GBps": march_gbs,
        "splat_pairs": pairs,
        "roofline": roofline,
        "rooflines": {"k_splat": splat_roof, "k_march": march_roof},
        "pipelined": None if pipe_ms is None else {
            "ms_per_frame": pipe_ms, "rays_per_s": nrays / (pipe_ms * 1e-3),
            "note": "two streams: the splat of frame i+1 overlaps the trace of frame i"},
        "achievable_bandwidth": achievable,
        "serving": None,
        "cpu_baseline": None,
    }
    if pairs is not None:
        line["splat_pairs_per_s"] = pairs / (avg["splat"] * 1e-3)
    ctx.close()
    if args.serve_seconds > 0:
        line["serving"] = serving_leg(haze, torch, W, args)
        sv = line["serving"]
        log(f"bench: serving p50 {sv['latency_ms']['p50']:.2f} ms, p99 {sv['latency_ms']['p99']:.2f} ms, "
            f"sustained {sv['sustained_rays_per_s'] / 1e6:.0f} M rays/s (offered {sv['offered_rays_per_s'] / 1e6:.0f})")
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host (cpu_baseline)")
        line["cpu_baseline"] = cpu_baseline(wl, args)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
