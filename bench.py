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
timed the same way.  On this physical field theta_max = 0.003 never binds, so
that pair is not an equal-error comparison: the oracle leg runs the
equal-error protocol (uniform step's error against the oracle's converged
reference, theta_max bisected to the same error, both traces timed) on this
field and on its K_GD x 250 stress variant, and reports the timed result's
error against the FP64 oracle.

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
# MI355X published FP32 vector peak (with packed FP32 instructions), and the
# peak this build can reach: its kernels are compiled with packed FP32
# disabled, so 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3
FP32_UNPACKED_PEAK_TFLOPS = 78.6
# wave64 VALU instructions the chip can issue per second: 256 CUs x 4 SIMDs x
# 2.4 GHz / 4 clocks per wave64 instruction
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
BYTES_PER_STEP = {"f32": 128, "f16": 64, "bf16": 64}   # 8 corners x 4 channels
LATENCY_SAMPLES = 100
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


def measured_counters(kernel: str, row: str, config: int, dtype: str):
    """Counter readings per launch from the committed summary of this workload
    (profiles/counters_config<N>_<dtype>.json): fabric (HBM/MALL) bytes from
    FETCH_SIZE + WRITE_SIZE scaled by a plain copy's readings, VALU wave
    instructions, L2 hit rate.  None when there is no summary for the
    workload or the kernel's code has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"counters_config{config}_{dtype}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        c = json.load(f)
    src = KERNEL_SOURCE[kernel]
    if code_digest(os.path.join(ROOT, src)) != c.get("code_sha256", {}).get(src):
        return None
    k = c["kernels"].get(row)
    if k is None:
        return None
    return {"bytes": k["fetch_bytes"] + k["write_bytes"], "read_bytes": k["fetch_bytes"],
            "write_bytes": k["write_bytes"], "fetch_scale": c["calibration"]["fetch_scale"],
            "write_scale": c["calibration"]["write_scale"], "valu_wave_instructions": k.get("valu_wave_instructions"),
            "l2_hit_rate": k.get("l2_hit_rate"), "source": os.path.relpath(path, ROOT)[:-5] + ".md"}


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


def time_steps(ctx, torch, fn, steps: int, warmup: int, kernels=(), live=("splat",), live_every: int = 4,
               latency_samples: int = LATENCY_SAMPLES):
    """ms per step over exactly `steps` steps (host clock between two device
    synchronisations) with the `live` kernel groups timed by their own
    dispatch events inside those steps (every `live_every`-th step, the first
    included); then a second pass of max(steps, LATENCY_SAMPLES) steps for
    per-step latencies (so p99 is not the largest of a few samples) and the
    other groups' times.  Every timed launch and every event record costs the
    stream microseconds, so the timed pass carries only what the roofline
    needs."""
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
    nlat = max(steps, latency_samples)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nlat + 1)]
    ev[0].record(stream)
    for i in range(nlat):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ctx.profile_enable(False)
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(nlat)])
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


def _rms_max(a: np.ndarray) -> dict:
    a = a[np.isfinite(a)]
    return {"max": float(a.max()) if a.size else None, "rms": float(np.sqrt(np.mean(a ** 2))) if a.size else None}


def trace_time(ctx, field, views, st, reps: int = 5) -> dict:
    """One full-frame trace (ray generation + march) timed by the kernels'
    dispatch events, mean of `reps` launches."""
    out = ctx.trace_views(field, views, st)
    import torch
    torch.cuda.synchronize()
    ctx.profile_read("march", reset=True)
    ctx.profile_select(("raygen", "march"))
    ctx.profile_enable(True)
    for _ in range(reps):
        ctx.trace_views(field, views, st, out=out)
    torch.cuda.synchronize()
    ctx.profile_enable(False)
    ms = (ctx.profile_read("raygen")[0] + ctx.profile_read("march")[0]) / reps
    ctx.profile_read("march", reset=True)
    ctx.profile_select(None)
    steps = int(out["steps"].sum().item())
    nrays = sum(v.nrays for v in views)
    return dict(ms=ms, rays_per_s=nrays / (ms * 1e-3), ray_steps_per_s=steps / (ms * 1e-3), ray_steps=steps)


def equal_error_protocol(oracle, ctx, field, md, wl, dtype: str = "f32", log_fn=None) -> dict:
    """Adaptive against uniform step at equal displacement-map error (Eq. 18's
    theta_max trade-off):
      1. E_u = RMS (and max) |disp_GPU,uniform(0.25 voxel) - disp_ref| over the
         rays of the workload's subset whose reference converged, where
         disp_ref is the oracle's solution of the continuous ray equation
         through its FP64 field (step halving to 2e-5 px between levels, then
         Richardson extrapolation; on stress fields rays near caustics do not
         converge and are left out, and their share is reported);
      2. theta_max swept down from the paper's 0.003 (h_max = 1 voxel) by
         factors of 3, then bisected in log(theta) for the largest theta whose
         adaptive RMS error E_a <= E_u (same rays);
      3. full-frame traces timed at that theta, at the paper's theta and with
         the uniform step."""
    import torch
    from paper_2603_02048_amd import workloads as W
    ids_np = wl.subset
    t0 = time.perf_counter()
    ref = oracle.reference_views(md, wl.views, wl.step_uniform, ray_ids=ids_np, max_levels=10, tol_px=2e-5,
                                 tol_dir=1e-7)
    t_ref = time.perf_counter() - t0
    ids = torch.from_numpy(ids_np).cuda()

    conv = ref["converged"].astype(bool)

    def err_of(st, only_converged=True):
        out = ctx.trace_views(field, wl.views, st, ray_ids=ids)
        d = out["disp"].cpu().numpy().astype(np.float64)
        e = np.linalg.norm(d - ref["disp"], axis=1)
        if only_converged:
            e = e[conv]
        e = e[np.isfinite(e)]
        return (float(np.sqrt(np.mean(e ** 2))), float(np.max(e))), int(out["steps"].sum().item())

    e_u, steps_u = err_of(wl.step_uniform)
    sweep = {}
    theta = 0.003
    while theta > 1e-9:
        st, _ = W.make_steps(wl.grid, theta_max=theta)
        sweep[theta] = err_of(st)
        if sweep[theta][0][0] <= e_u[0]:
            break
        theta /= 3.0
    if sweep[theta][0][0] > e_u[0]:
        return {"error": "no theta in the sweep reached the uniform step's error"}
    lo_t, hi_t = theta, (theta * 3.0 if theta < 0.003 else theta)
    for _ in range(6):
        if hi_t <= lo_t:
            break
        mid = math.sqrt(lo_t * hi_t)
        st, _ = W.make_steps(wl.grid, theta_max=mid)
        sweep[mid] = err_of(st)
        if sweep[mid][0][0] <= e_u[0]:
            lo_t = mid
        else:
            hi_t = mid
    theta_eq = lo_t
    st_eq, _ = W.make_steps(wl.grid, theta_max=theta_eq)
    t_a = trace_time(ctx, field, wl.views, st_eq)
    t_p = trace_time(ctx, field, wl.views, wl.step_adaptive)
    t_u = trace_time(ctx, field, wl.views, wl.step_uniform)
    # the same errors over all rays of the subset, converged or not (on
    # stress fields rays near caustics keep moving by more than the
    # convergence bar under step halving; there these numbers compare
    # against an unconverged reference)
    e_ua = err_of(wl.step_uniform, False)[0]
    e_aa = err_of(st_eq, False)[0]
    res = {"subset_rays": int(ids_np.size), "reference_converged_fraction": float(np.mean(conv)),
           "rays_compared": int(conv.sum()), "reference_s": t_ref, "theta_eq": theta_eq,
           "all_rays_including_unconverged": {"E_uniform_px": {"rms": e_ua[0], "max": e_ua[1]},
                                              "E_adaptive_px": {"rms": e_aa[0], "max": e_aa[1]}},
           "E_uniform_px": {"rms": e_u[0], "max": e_u[1]},
           "E_adaptive_px": {"rms": sweep[theta_eq][0][0], "max": sweep[theta_eq][0][1]},
           "E_adaptive_at_paper_theta_px": {"rms": sweep[0.003][0][0], "max": sweep[0.003][0][1]},
           "uniform": t_u, "adaptive_at_theta_eq": t_a, "adaptive_at_paper_theta": t_p,
           "speed_ratio": t_u["ms"] / t_a["ms"],
           "sweep": {f"{k:.3g}": {"rms_px": v[0][0], "max_px": v[0][1], "subset_steps": v[1]}
                     for k, v in sorted(sweep.items(), reverse=True)}}
    if log_fn:
        log_fn(f"bench: equal error: E_u {e_u[0]:.3g} px rms, theta_eq {theta_eq:.3g} (E_a {sweep[theta_eq][0][0]:.3g}), "
               f"uniform {t_u['ms']:.3f} ms, adaptive at theta_eq {t_a['ms']:.3f} ms: ratio {res['speed_ratio']:.2f}")
    return res


def cpu_baseline_leg(wl, args, ctx, parts, run_step, st_a, out, dtype: str, scale: float) -> dict:
    """The FP64 oracle on the host cores (the only leg that runs it):
      * cpu_baseline: full splat + a bounded random ray sample, adaptive, timed
        on all host threads and (a quarter of the sample) on one;
      * error_vs_oracle: the timed configuration's GPU result (one more step
        of the benchmark, run_step, into `out`) against the oracle on the same
        sampled rays;
      * equal_error (the default workload): the equal-error protocol on the
        physical field and on its K_GD x 250 stress variant."""
    import oracle
    import torch
    oracle.build()
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    md = oracle.field(wl.particles, wl.grid, wl.k_gd, wl.h, "cells")
    t_splat = time.perf_counter() - t0
    rng = np.random.default_rng(12345)
    ns = min(wl.nrays, args.cpu_rays)
    ids = np.sort(rng.choice(wl.nrays, size=ns, replace=False)).astype(np.int64)
    t0 = time.perf_counter()
    r = oracle.trace_views(md, wl.views, st_a, ray_ids=ids)
    t_trace = time.perf_counter() - t0
    frame_s = t_splat + t_trace * wl.nrays / ns
    oracle.set_num_threads(1)
    try:
        ids1 = ids[::4]
        t0 = time.perf_counter()
        r1 = oracle.trace_views(md, wl.views, st_a, ray_ids=ids1)
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    base = {"value": wl.nrays / frame_s, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle: full splat of the {tuple(int(x) for x in wl.grid.res)} grid "
                       f"({t_splat:.2f} s) + {ns} random rays of the {wl.nrays}-ray frame, adaptive "
                       f"({t_trace:.2f} s), scaled to one frame"),
            "ray_steps_per_s": float(r["steps"].sum()) / t_trace, "frame_s": frame_s,
            "voxels_per_s": wl.grid.nvox / t_splat,
            "single_thread": {"rays": int(ids1.size), "rays_per_s": ids1.size / t1,
                              "ray_steps_per_s": float(r1["steps"].sum()) / t1},
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}

    # the timed step once more, its outputs against the oracle's on the sample
    run_step()
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    g = {k: v[ids] for k, v in g.items()}
    vox = wl.grid.voxel
    e_pos = np.linalg.norm(g["exit_pos"].astype(np.float64) - r["exit_pos"], axis=1) / vox
    e_dir = np.linalg.norm(g["exit_dir"].astype(np.float64) - r["exit_dir"], axis=1)
    d_g, d_r = g["disp"].astype(np.float64), r["disp"]
    e_px = np.where(np.isnan(d_g) & np.isnan(d_r), 0.0, np.abs(d_g - d_r)).max(axis=1)
    err = {"rays": int(ns), "dtype": dtype, "pos_voxel": _rms_max(e_pos), "dir_rad": _rms_max(e_dir),
           "disp_px": _rms_max(e_px), "status_equal_fraction": float(np.mean(g["status"] == r["status"])),
           "steps_max_diff": int(np.abs(g["steps"].astype(np.int64) - r["steps"].astype(np.int64)).max()),
           "tolerance": {"pos_voxel": 1e-3, "dir_rad": 1e-5, "disp_px": 0.02},
           "rays_sampled": "the cpu_baseline sample"}
    log(f"bench: error vs the FP64 oracle ({dtype}, {ns} rays): max {err['pos_voxel']['max']:.2e} voxel, "
        f"{err['dir_rad']['max']:.2e} rad, {err['disp_px']['max']:.2e} px")

    eq = None
    if wl.name == "config2" and not args.no_equal_error:
        from paper_2603_02048_amd import workloads as W
        eq = {}
        for factor in (1.0, 250.0):
            wlk = wl if factor == 1.0 else wl.with_k_gd(factor)
            mdk = md if factor == 1.0 else oracle.field(wlk.particles, wlk.grid, wlk.k_gd, wlk.h, "cells")
            field = ctx.splat_index_field(parts, wlk.grid, wlk.k_gd, wlk.h, dtype=dtype, store_scale=scale)
            name = "physical" if factor == 1.0 else "kgd_x250"
            eq[name] = equal_error_protocol(oracle, ctx, field, mdk, wlk, dtype, log_fn=log)
            eq[name]["field"] = f"{wl.name} K_GD x {factor:g}, {dtype}"
            field.release()
    return {"cpu_baseline": base, "error_vs_oracle": err, "equal_error": eq}


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
    ap.add_argument("--trace-stream", action="store_true",
                    help="run each step's trace on a second stream, so that its ray generation overlaps the cell "
                         "list and the splat")
    ap.add_argument("--splat", default="gather", choices=["gather", "scatter"])
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--no-equal-error", action="store_true", help="skip the equal-error protocol of the oracle leg")
    ap.add_argument("--latency-samples", type=int, default=LATENCY_SAMPLES,
                    help="steps of the latency pass (at least --steps); fewer under a profiler")
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

    # With --trace-stream a step's trace runs on a second stream (default
    # priority): its ray generation reads no field data and runs beside the
    # cell list and the splat; the library makes the march wait for the field.
    # The step still ends only when both streams are done.  (Config 3: 1.53
    # against 1.59 ms; config 2: 0.584 against 0.577, the two cross-stream
    # waits costing more than its 22 us of ray generation.)
    trace_stream = torch.cuda.Stream() if args.trace_stream else None

    def make_step(st):
        def fn():
            if trace_stream is None:
                f = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h, dtype=args.dtype, store_scale=scale)
                ctx.trace_views(f, wl.views, st, out=out)
                f.release()
                return
            main = torch.cuda.current_stream()
            trace_stream.wait_stream(main)          # the previous step is done
            f = ctx.splat_index_field(parts, wl.grid, wl.k_gd, wl.h, dtype=args.dtype, store_scale=scale)
            ctx.trace_views(f, wl.views, st, out=out, stream=trace_stream)
            main.wait_stream(trace_stream)
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
        ms, per, kt = time_steps(ctx, torch, make_step(st), args.steps, args.warmup, kernels,
                                 latency_samples=args.latency_samples)
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
        # the marcher's own pattern with no arithmetic: the benchmarked views'
        # pinhole rays walked straight through the grid in steps of h_max
        # (the step the adaptive rule takes on this field), 8 corners a sample
        g, n = ctx.membench_gather(wl.grid, fb // wl.grid.nvox, wl.views, st_a.ds_max, 20)
        achievable["view_gather_GBps"] = g
        achievable["view_gather_samples"] = n
        achievable["view_gather_note"] = ("the benchmarked views' entering rays in the tracer's length-sorted "
                                          "hit-list order, walked straight, one sample per h_max (8 corners "
                                          "per sample)")
        log(f"bench: achievable read bandwidth: 4 GiB buffer {achievable['hbm_read_GBps']:.0f} GB/s, "
            f"field-sized ({fb >> 20} MiB) {achievable['field_sized_read_GBps']:.0f} GB/s, "
            f"the views' rays walked straight ({n} samples) {g:.0f} GB/s")

    A, U = res["adaptive"], res["uniform"]
    rays_s = nrays / (A["ms"] * 1e-3)
    # dominant kernel of the adaptive step
    avg = {k: v[0] / max(v[1], 1) for k, v in A["kt"].items()}
    dominant = max(avg, key=avg.get)
    roofline = None
    march_ms = avg["march"]
    march_gbs = A["steps"] * BYTES_PER_STEP[args.dtype] / (march_ms * 1e-3) / 1e9
    # The march's gathers are served by the caches (neighbouring rays share
    # cells): its bound is the achievable rate of the same gathers with no
    # arithmetic, and its instruction issue; HBM/MALL traffic comes from the
    # counters.
    march_roof = {"kernel": "k_march", "bound": "cache gathers (L1/L2, MALL behind)", "achieved": march_gbs,
                  "peak": achievable["view_gather_GBps"] if achievable else None, "unit": "GB/s",
                  "frac": march_gbs / achievable["view_gather_GBps"] if achievable else None,
                  "peak_is": "achievable gather rate of the same views' rays walked straight, no arithmetic "
                             "(hz_membench_gather)",
                  "per_unit": f"{BYTES_PER_STEP[args.dtype]} B gathered per ray-step (8 corners x 4 channels)",
                  "units_per_launch": A["steps"], "launch_ms": march_ms,
                  "launch_timing": "dispatch events in the latency pass of the same steps", "traffic": None}
    tr = measured_counters("k_march", "k_march (adaptive)", args.config, args.dtype)
    if tr is not None and args.theta is None:
        fabric_gbs = tr["bytes"] / (march_ms * 1e-3) / 1e9
        march_roof["traffic"] = tr["bytes"]
        march_roof["traffic_detail"] = tr
        march_roof["hbm"] = {"achieved": fabric_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": fabric_gbs / HBM_PEAK_GBS,
                             "note": "counter-measured fabric bytes (L2 misses to MALL/HBM) per launch / launch time"}
        if tr.get("valu_wave_instructions"):
            iss = tr["valu_wave_instructions"] / (march_ms * 1e-3)
            march_roof["valu_issue"] = {"achieved": iss, "peak": VALU_ISSUE_PEAK, "unit": "wave64 instr/s",
                                        "frac": iss / VALU_ISSUE_PEAK,
                                        "per_ray_step": tr["valu_wave_instructions"] / A["steps"]}
    pairs = None
    splat_roof = None
    if not args.no_pairs:
        pairs = count_pairs(torch, parts, wl.grid, wl.h)
        tf = pairs * 25.0 / (avg["splat"] * 1e-3) / 1e12
        splat_roof = {"kernel": "k_splat_scatter" if args.splat == "scatter" else "k_splat", "bound": "alu",
                      "achieved": tf, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / FP32_PEAK_TFLOPS,
                      "peak_is": "MI355X published FP32 vector peak (packed FP32)",
                      "peak_unpacked": FP32_UNPACKED_PEAK_TFLOPS, "frac_of_unpacked": tf / FP32_UNPACKED_PEAK_TFLOPS,
                      "peak_unpacked_is": ("256 CUs x 4 SIMDs x 16 lanes x FMA x 2.4 GHz: the ceiling of this "
                                           "build, whose kernels are compiled without packed FP32"),
                      "traffic": None,
                      "per_unit": "25 FP32 flops per (voxel, particle) pair within 2h",
                      "launch_ms": avg["splat"], "units_per_launch": pairs,
                      "launch_timing": "dispatch events of the kernel in every 4th of the timed steps"}
        tr = measured_counters("k_splat", "k_splat", args.config, args.dtype)
        if tr is not None and args.splat == "gather":
            splat_roof["traffic"] = tr["bytes"]
            splat_roof["traffic_detail"] = tr
            if tr.get("valu_wave_instructions"):
                iss = tr["valu_wave_instructions"] / (avg["splat"] * 1e-3)
                splat_roof["valu_issue"] = {"achieved": iss, "peak": VALU_ISSUE_PEAK, "unit": "wave64 instr/s",
                                            "frac": iss / VALU_ISSUE_PEAK,
                                            "lane_instr_per_pair": 64.0 * tr["valu_wave_instructions"] / pairs}
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
        "latency_ms": {"p50": float(np.percentile(A["per"], 50)), "p99": float(np.percentile(A["per"], 99)),
                       "samples": int(A["per"].size), "what": "whole step (splat + trace of the frame), device time"},
        "adaptive_vs_uniform_note": ("'adaptive' is the paper's rule at theta_max = 0.003, which on this physical "
                                     "field never binds (every step is h_max = 1 voxel), against a 0.25-voxel "
                                     "uniform step: not an equal-error comparison.  equal_error holds that one."),
        "adaptive": {"rays_per_s": rays_s, "ray_steps": A["steps"], "rays_in_volume": A["hits"],
                     "per_view": A["per_view"],
                     "trace_rays_per_s": nrays / ((avg["raygen"] + avg["march"]) * 1e-3),
                     "trace_ray_steps_per_s": A["steps"] / ((avg["raygen"] + avg["march"]) * 1e-3)},
        "uniform": {"rays_per_s": nrays / (U["ms"] * 1e-3), "ms_per_step": U["ms"], "ray_steps": U["steps"],
                    "ray_steps_per_s": U["steps"] / (U["ms"] * 1e-3),
                    "latency_ms": {"p50": float(np.percentile(U["per"], 50)),
                                   "p99": float(np.percentile(U["per"], 99)), "samples": int(U["per"].size)}},
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
        "error_vs_oracle": None,
        "equal_error": None,
    }
    if pairs is not None:
        line["splat_pairs_per_s"] = pairs / (avg["splat"] * 1e-3)
    if not args.no_cpu_baseline:
        log("bench: the FP64 oracle on the host (cpu_baseline, error_vs_oracle, equal_error)")
        leg = cpu_baseline_leg(wl, args, ctx, parts, make_step(st_a), st_a, out, args.dtype, scale)
        line.update(leg)
    ctx.close()
    if args.serve_seconds > 0:
        line["serving"] = serving_leg(haze, torch, W, args)
        sv = line["serving"]
        log(f"bench: serving p50 {sv['latency_ms']['p50']:.2f} ms, p99 {sv['latency_ms']['p99']:.2f} ms, "
            f"sustained {sv['sustained_rays_per_s'] / 1e6:.0f} M rays/s (offered {sv['offered_rays_per_s'] / 1e6:.0f})")
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
