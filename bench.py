"""Benchmark of the SGM hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--extras none|batch|all] [--serve-seconds S]

A step is one pass of the whole path (Census of both views, Hamming costs,
8-path aggregation, WTA + right-view disparity + left-right check, 3x3
median, U-/V-maps) over one synthetic 1242x375 pair with D = 128 (the
KITTI-shaped workload), inputs already in device memory.  Steps go through
sgm_submit on one library stream (frames run back to back, up to 8 queued);
the timed region is bracketed by torch.cuda.synchronize().

Prints ONE JSON line: the throughput in Mdisp-evals/s (W*H*D*paths per
second), the aggregation kernel's roofline position (its average launch time
from HIP events the library records around it on its own stream), the CPU
oracle timed on a bounded sample of the same workload, and secondary
measurements (per-frame stage calls, a batch of 32 mixed pairs, a batch of 8
1920x1080 D=256 pairs, and the multi-camera request loop).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
ALG_BYTES_PER_EVAL = 4         # read + write of a uint16 running sum per path and cell
HEADLINE_STREAMS = 4           # the library context's default stream count


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kitti_params(sgm, W=1242, H=375, D=128):
    return sgm.Params(width=W, height=H, max_disp=D, census_w=9, census_h=7, path_mask=0xFF,
                      p1=10, p2=120, lr_check=1, median=3)


def time_submit_stream(torch, sgm, ctx, frames_fn, steps, warmup, depth=8):
    """Run `steps` submits of one batch each, keeping up to `depth` in flight
    (how they overlap on the GPU depends on the context's stream count).
    Returns (seconds, list of per-step Frame lists)."""
    outs = [frames_fn(i) for i in range(depth)]

    def run(n):
        inflight = []
        for s in range(n):
            if len(inflight) >= depth:
                sgm.sgm_wait(ctx, inflight.pop(0))
            inflight.append(sgm.sgm_submit(ctx, outs[s % depth]))
        for t in inflight:
            sgm.sgm_wait(ctx, t)

    run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, outs


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(left, right, p, seconds_target=12.0):
    """The oracle on the host: whole pairs with OpenMP over scanlines on all
    the cores it gets (the reported value), then one thread on a 94-row crop
    of the same pair (a bounded sample, scaled to the same unit)."""
    from oracle import oracle as O
    threads = O.threads()
    runs, t_total = 0, 0.0
    while t_total < seconds_target or runs == 0:
        t0 = time.perf_counter()
        O.sgm(left, right, p.max_disp, p.census_w, p.census_h, p.path_mask, p.p1, p.p2, True,
              p.lr_max_diff, p.median, p.inv())
        t_total += time.perf_counter() - t0
        runs += 1
        if runs >= 5:
            break
    rows = min(94, p.height)
    O.set_threads(1)
    try:
        t0 = time.perf_counter()
        O.sgm(left[:rows], right[:rows], p.max_disp, p.census_w, p.census_h, p.path_mask, p.p1, p.p2, True,
              p.lr_max_diff, p.median, p.inv())
        t1 = time.perf_counter() - t0
    finally:
        O.set_threads(threads)
    one = p.width * rows * p.max_disp * bin(p.path_mask).count("1") / t1 / 1e6
    return {"value": round(runs * p.disp_evals() / t_total / 1e6, 2), "unit": "Mdisp-evals/s",
            "cores": threads, "kind": "oracle",
            "sample": "%d full %dx%d D=%d 8-path pairs through the C oracle (-O2, OpenMP over "
                      "scanlines), %.1f s" % (runs, p.width, p.height, p.max_disp, t_total),
            "single_thread": {"value": round(one, 2), "sample": "one %dx%d crop, one thread, %.1f s"
                              % (p.width, rows, t1)},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def bench_small(torch, sgm, ctx, synthetic, steps=200):
    """320x240, D=64, Census 5x5, L->R/R->L/T->B/B->T, WTA only: one pair per
    step on one stream, then with 4 streams."""
    L, R, _ = synthetic.make_pair("small", 1000)
    p = sgm.Params(width=320, height=240, max_disp=64, census_w=5, census_h=5, path_mask=0x0F,
                   p1=10, p2=120, lr_check=0, median=0)
    Lt, Rt = torch.from_numpy(L).cuda(), torch.from_numpy(R).cuda()
    h = sgm.sgm_autotune(ctx, sgm.Frame.alloc(p, Lt, Rt), reps=5)[0]
    prof_on = True
    sgm.sgm_profile(ctx, False)
    res = {"h_lanes": h}
    for streams in (1, 4):
        sgm.sgm_set_streams(ctx, streams)
        dt, _ = time_submit_stream(torch, sgm, ctx, lambda i: [sgm.Frame.alloc(p, Lt, Rt)], steps, 10)
        res["streams%d_mdisp_evals_per_s" % streams] = p.disp_evals() * steps / dt / 1e6
        res["streams%d_fps" % streams] = steps / dt
    sgm.sgm_set_streams(ctx, 1)
    sgm.sgm_profile(ctx, prof_on)
    return res


def bench_paper_settings(torch, sgm, ctx, synthetic, steps=100):
    """The paper's own setting (640x360, D in [0,60), 5x5 support, the four
    forward paths of its figure 2, LR check, 5x5 median; section 4.1) with
    the Census cost (P1=8, P2=32) and with SAD (P1=200, P2=800): one pair per
    step on one stream.  The paper's FPGA ran this at 29 Hz (section 4.1)."""
    L, R, _ = synthetic.make_pair("paper", 7)
    Lt, Rt = torch.from_numpy(L).cuda(), torch.from_numpy(R).cuda()
    res = {"paper_fpga_hz": 29.0}
    sgm.sgm_profile(ctx, False)
    sgm.sgm_set_streams(ctx, 1)
    for name, kw in (("census", dict(cost=sgm.COST_CENSUS, p1=8, p2=32)),
                     ("sad", dict(cost=sgm.COST_SAD, p1=200, p2=800))):
        p = sgm.Params(width=640, height=360, max_disp=60, census_w=5, census_h=5,
                       path_mask=sgm.PATHS_PAPER4, lr_check=1, median=5, **kw)
        sgm.sgm_autotune(ctx, sgm.Frame.alloc(p, Lt, Rt), reps=3)
        dt, _ = time_submit_stream(torch, sgm, ctx, lambda i: [sgm.Frame.alloc(p, Lt, Rt)], steps, 10)
        res[name] = {"fps": steps / dt, "mdisp_evals_per_s": p.disp_evals() * steps / dt / 1e6,
                     "ms_per_frame": dt / steps * 1e3}
    res["census_sweep"] = bench_sweep(torch, sgm, ctx, synthetic)
    res["census_rectified"] = bench_rectified(torch, sgm, ctx, synthetic, steps)
    res["uv_filter"] = bench_uv_filter(torch, sgm, ctx, synthetic)
    sgm.sgm_profile(ctx, True)
    return res


def bench_uv_filter(torch, sgm, ctx, synthetic, reps=200):
    """Obstacle-map filtering (threshold, 3x3 dilation, 5x5 binomial blur,
    region of interest) of one frame's U-map [60][640] and V-map [360][60]
    in one launch, timed with events on the stream it runs on."""
    L, R, _ = synthetic.make_pair("paper", 7)
    p = sgm.Params(width=640, height=360, max_disp=60, census_w=5, census_h=5, path_mask=sgm.PATHS_PAPER4,
                   lr_check=1, median=5, p1=8, p2=32)
    f = sgm.Frame.alloc(p, torch.from_numpy(L).cuda(), torch.from_numpy(R).cuda())
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
    u_out = torch.empty((60, 640), dtype=torch.uint8, device="cuda")
    v_out = torch.empty((360, 60), dtype=torch.uint8, device="cuda")
    jobs = [sgm.filter_job(f.umap, u_out, 20, 1, 2, (1, 60, 0, 640)),
            sgm.filter_job(f.vmap, v_out, 30, 1, 2, (120, 360, 0, 60))]
    stream = torch.cuda.current_stream()
    for _ in range(10):
        sgm.uv_filter(ctx, jobs, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        sgm.uv_filter(ctx, jobs, stream)
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    cells = 60 * 640 + 360 * 60
    return {"us_per_frame": us, "cells": cells, "algorithmic_bytes": 3 * cells,
            "gb_per_s": 3 * cells / (us * 1e-6) / 1e9}


def bench_sweep(torch, sgm, ctx, synthetic, batch=256, reps=3):
    """The paper's Census setting through the single-pass sweep (one block
    per frame, nothing but the disparity maps written) against the
    per-direction kernels: one frame per submit, and batches of `batch`
    frames (a frame per CU)."""
    L, R, _ = synthetic.make_pair("paper", 7)
    Lt, Rt = torch.from_numpy(L).cuda(), torch.from_numpy(R).cuda()
    p = sgm.Params(width=640, height=360, max_disp=60, census_w=5, census_h=5, path_mask=sgm.PATHS_PAPER4,
                   lr_check=1, median=5, p1=8, p2=32)
    h = sgm.sgm_get_schedule(ctx, p)
    res = {"batch": batch}
    for name, sweep in (("direction_kernels", False), ("sweep", True)):
        sgm.sgm_set_schedule(ctx, p, h, sweep=sweep)
        one = [sgm.Frame.alloc(p, Lt, Rt)]
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, one))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, one))
        single_ms = (time.perf_counter() - t0) / reps * 1e3
        frames = [sgm.Frame.alloc(p, Lt, Rt) for _ in range(batch)]
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
        dt = (time.perf_counter() - t0) / reps
        res[name] = {"single_frame_ms": single_ms, "batch_ms": dt * 1e3, "batch_fps": batch / dt}
        del frames
    sgm.sgm_set_schedule(ctx, p, h, sweep=False)
    return res


def bench_rectified(torch, sgm, ctx, synthetic, steps):
    """Raw 672x380 pairs rectified to 640x360 by synthetic calibration maps
    (section 3.1.1), then the paper's Census setting: sgm_submit_rectify per
    pair, and the rectification kernel alone (both views, one launch) timed
    with events on the stream it runs on."""
    w, h, D, sw, sh = 640, 360, 60, 672, 380
    raw_l, raw_r, _ = synthetic.make_pair("paper", 8, sw, sh, D)
    RL, RR = torch.from_numpy(raw_l).cuda(), torch.from_numpy(raw_r).cuda()
    maps = [tuple(torch.from_numpy(m).cuda() for m in synthetic.rectification_maps(w, h, sw, sh, seed=s))
            for s in (1, 2)]
    p = sgm.Params(width=w, height=h, max_disp=D, census_w=5, census_h=5, path_mask=sgm.PATHS_PAPER4,
                   lr_check=1, median=5, p1=8, p2=32)
    frames = [sgm.Frame.alloc(p, torch.empty((h, w), dtype=torch.uint8, device="cuda"),
                              torch.empty((h, w), dtype=torch.uint8, device="cuda")) for _ in range(8)]
    remaps = [(RL, *maps[0]), (RR, *maps[1])]

    def run(n):
        inflight = []
        for s in range(n):
            if len(inflight) >= 8:
                sgm.sgm_wait(ctx, inflight.pop(0))
            inflight.append(sgm.sgm_submit_rectify(ctx, [frames[s % 8]], remaps))
        for t in inflight:
            sgm.sgm_wait(ctx, t)

    run(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    jobs = [sgm.remap_job(RL, *maps[0], frames[0].left), sgm.remap_job(RR, *maps[1], frames[0].right)]
    stream = torch.cuda.current_stream()
    for _ in range(10):
        sgm.sgm_rectify(ctx, jobs, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 200
    e0.record(stream)
    for _ in range(reps):
        sgm.sgm_rectify(ctx, jobs, stream)
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    # algorithmic bytes of one launch: per rectified pixel two 16-bit map
    # entries and one output byte, plus each raw image read once
    algo = 2 * (w * h * 5 + sw * sh)
    return {"fps": steps / dt, "ms_per_frame": dt / steps * 1e3, "raw": "%dx%d" % (sw, sh),
            "rectify_us_per_pair": us, "rectify_algorithmic_bytes": algo,
            "rectify_gb_per_s": algo / (us * 1e-6) / 1e9}


def bench_batch32(torch, sgm, ctx, synthetic):
    specs = synthetic.mixed_batch_specs(32, seed=2000)
    frames = []
    for (W, H, D, seed) in specs:
        L, R, _ = synthetic.make_pair("kitti", seed, W, H, D)
        p = kitti_params(sgm, W, H, D)
        frames.append(sgm.Frame.alloc(p, torch.from_numpy(L).cuda(), torch.from_numpy(R).cuda()))
    evals = sum(f.p.disp_evals() for f in frames)
    res = {}
    sgm.sgm_profile(ctx, False)
    # autotune each distinct shape once on its first frame
    tuned = {}
    for f in frames:
        key = (f.p.width, f.p.height, f.p.max_disp)
        if key not in tuned:
            tuned[key] = sgm.sgm_autotune(ctx, f, reps=3)[0]
    res["schedules"] = {"%dx%d D%d" % k: v for k, v in tuned.items()}
    # one submit of all 32
    for _ in range(2):
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    batched = [f.disp.clone() for f in frames]
    sgm.sgm_set_graphs(ctx, True)
    for _ in range(2):
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
    torch.cuda.synchronize()
    tg = (time.perf_counter() - t0) / reps
    sgm.sgm_set_graphs(ctx, False)
    same_graph = all(torch.equal(a, f.disp) for a, f in zip(batched, frames))
    # 32 sequential per-frame submits, each waited for
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for f in frames:
            sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / reps
    same = all(torch.equal(a, f.disp) for a, f in zip(batched, frames))
    # 32 sequential per-frame stage-call pipelines
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in frames:
        sgm.run_stages(ctx, f.p, f.left, f.right)
    torch.cuda.synchronize()
    tst = time.perf_counter() - t0
    res.update(frames=32, disp_evals=evals, batched_ms=tb * 1e3,
               batched_mdisp_evals_per_s=evals / tb / 1e6,
               sequential_submit_ms=ts * 1e3, sequential_submit_mdisp_evals_per_s=evals / ts / 1e6,
               sequential_stage_calls_ms=tst * 1e3,
               sequential_stage_calls_mdisp_evals_per_s=evals / tst / 1e6,
               batched_equals_sequential=bool(same), graph_batched_ms=tg * 1e3,
               graph_batched_mdisp_evals_per_s=evals / tg / 1e6, graph_equals_direct=bool(same_graph))
    sgm.sgm_profile(ctx, True)
    return res


def bench_large(torch, sgm, ctx, synthetic, nframes=8):
    """Eight 1920x1080 D=256 pairs (8 paths, LR, 3x3 median, U/V): one submit
    of all eight vs eight sequential one-frame submits on the same inputs
    (outputs compared), and the aggregation kernel's roofline position, with
    the HBM bytes it actually moves when the committed counter record for
    this workload matches the kernel sources."""
    frames = []
    for i in range(nframes):
        L, R, _ = synthetic.make_pair("large", 4000 + i)
        p = kitti_params(sgm, 1920, 1080, 256)
        p.invalid = 65535
        frames.append(sgm.Frame.alloc(p, torch.from_numpy(L).cuda(), torch.from_numpy(R).cuda()))
    evals = sum(f.p.disp_evals() for f in frames)
    h_lanes = sgm.sgm_autotune(ctx, frames[0], reps=2)[0]
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
    batched = [f.disp.clone() for f in frames]
    sgm.sgm_profile_read(ctx, reset=True)
    torch.cuda.synchronize()
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    prof = sgm.sgm_profile_read(ctx, reset=True)
    agg_ms, agg_n = prof["aggregate"]
    agg_avg = agg_ms / max(agg_n, 1)
    achieved = ALG_BYTES_PER_EVAL * evals / (agg_avg * 1e-3) / 1e9
    # the same frames one submit at a time (queued back to back)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ts = [sgm.sgm_submit(ctx, [f]) for f in frames]
        for tk in ts:
            sgm.sgm_wait(ctx, tk)
    torch.cuda.synchronize()
    tseq = (time.perf_counter() - t0) / reps
    same = all(torch.equal(a, f.disp) for a, f in zip(batched, frames))
    res = {"frames": nframes, "width": 1920, "height": 1080, "max_disp": 256, "paths": 8,
           "h_lanes": h_lanes,
           "batch_ms": t * 1e3, "mdisp_evals_per_s": evals / t / 1e6, "fps": nframes / t,
           "sequential_submits_ms": tseq * 1e3, "sequential_mdisp_evals_per_s": evals / tseq / 1e6,
           "batched_equals_sequential": bool(same),
           "aggregate_launch_ms": agg_avg,
           "aggregate_alg_GBs": achieved, "aggregate_hbm_frac": achieved / HBM_PEAK_GBS,
           "stage_ms_per_batch": {k: v[0] / reps for k, v in prof.items()}}
    moved = measured_traffic("agg_kernel<16, %d, %d, 0, unsigned char" % (256 // h_lanes, h_lanes),
                             "traffic_agg_1920x1080_d256_batch8.json")
    if moved is not None:
        res["aggregate_measured_bytes"] = moved
        res["aggregate_measured_GBs"] = moved / (agg_avg * 1e-3) / 1e9
        res["aggregate_measured_hbm_frac"] = res["aggregate_measured_GBs"] / HBM_PEAK_GBS
    return res


def bench_serve(torch, sgm, synthetic, ctx, seconds, stress_cameras=48, stress_seconds=4.0):
    """The 4-camera request loop at 30 fps per camera (640x480 and 1242x375,
    D=128, 8 paths), continuous batching vs one frame at a time on the
    identical trace; then the same with `stress_cameras` cameras, a load at
    which one-at-a-time processing queues up.  Also checks that every frame's
    disparity map is identical in both modes (alone vs in the mix)."""
    from paper_1807_06271_amd import serve
    base = []
    for cam in range(4):
        sc = synthetic.camera_scene(cam)
        pairs = [synthetic.render_pair(sc, k)[:2] for k in range(3)]
        p = kitti_params(sgm, sc.width, sc.height, 128)
        base.append((p, pairs))
    out = {}
    # autotune both frame shapes once (kept by the context)
    for p, pairs in base[1:3]:
        f = sgm.Frame.alloc(p, torch.from_numpy(pairs[0][0]).cuda(), torch.from_numpy(pairs[0][1]).cuda())
        sgm.sgm_autotune(ctx, f, reps=3)
    for label, ncam, secs in (("4cams_30fps", 4, seconds), ("%dcams_30fps" % stress_cameras, stress_cameras, stress_seconds)):
        cams = [serve.Camera(base[c % 4][0], base[c % 4][1]) for c in range(ncam)]
        trace = synthetic.poisson_trace(ncam, 30.0, secs, seed=3000 + ncam)
        serve.serve(ctx, cams, [(0.0, c, 0) for c in range(min(ncam, 8))], continuous=True)  # warm-up
        res = {"cameras": ncam, "fps_per_camera": 30, "seconds": secs, "frames": len(trace)}
        maps = {}
        for mode, cont in (("continuous_batching", True), ("per_frame", False)):
            stats, done = serve.serve(ctx, cams, trace, continuous=cont)
            log("served %s %s: p50 %.3f ms, p99 %.3f ms" % (label, mode, stats["p50_ms"], stats["p99_ms"]))
            res[mode] = stats
            maps[mode] = done
        a, b = maps["continuous_batching"], maps["per_frame"]
        res["mix_equals_alone"] = bool(a.keys() == b.keys() and all(
            all(torch.equal(x, y) for x, y in zip(a[k], b[k])) for k in a))
        out[label] = res
    return out


def served_p99(extras):
    """p50 / p99 latency of the 4-camera request loop in both modes, or None
    when the request loop was not run."""
    run = extras.get("served", {}).get("4cams_30fps")
    if run is None:
        return None
    return {mode: {"p50": round(run[mode]["p50_ms"], 4), "p99": round(run[mode]["p99_ms"], 4)}
            for mode in ("continuous_batching", "per_frame")}


def measured_traffic(kernel_prefix, record="traffic_agg_1242x375_d128.json"):
    """HBM bytes per launch of an aggregation kernel from a committed
    FETCH_SIZE / WRITE_SIZE counter record (scaled by a copy of known size), or
    None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(path):
        return None
    from paper_1807_06271_amd.profiling import source_hash
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash():
        return None
    for name, k in rec["kernels"].items():
        if kernel_prefix in name:
            return int(k["fetch_bytes"] + k["write_bytes"])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--extras", choices=["none", "large", "batch", "serve", "all"], default="all",
                    help="secondary measurements: none; large (the 8 x 1920x1080 batch only); "
                         "batch (all batch forms); serve (the request loop only); "
                         "all (batch forms and the request loop)")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of a known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(frames would shard across GPUs with no exchange between them)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from gen import synthetic
    from paper_1807_06271_amd import sgm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    sgm.lib()  # raises if libsgm.so is missing: no fallback
    # The library's contexts are created before torch puts anything on the
    # device: the HIP runtime spreads streams over its hardware queues (4 per
    # process by default) in the order they appear, and contexts created
    # after torch's own streams had two of their four streams on one queue,
    # which cost the four-stream loop ~10 % (0.27 instead of 0.24 ms/frame).
    ctx = sgm.Context(0)
    serve_ctx = sgm.Context(0)

    left, right, _ = synthetic.make_pair("kitti", 1001)
    p = kitti_params(sgm)
    L = torch.from_numpy(left).cuda()
    R = torch.from_numpy(right).cuda()
    if args.calibrate_copy:
        from paper_1807_06271_amd.profiling import CALIBRATION_BYTES
        src = torch.ones(CALIBRATION_BYTES, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # autotune the schedule of this shape once (the winner stays in the context)
    h_lanes, tune_ms = sgm.sgm_autotune(ctx, sgm.Frame.alloc(p, L, R), reps=5)
    log("autotuned h_lanes", h_lanes, tune_ms)
    log("main: 1242x375 D=128 8 paths, steps", args.steps)
    # one stream first: the frames run strictly back to back, nothing else
    # shares the GPU (kernel durations in a trace of this loop are clean)
    sgm.sgm_set_streams(ctx, 1)
    sgm.sgm_profile(ctx, False)
    dt1, outs = time_submit_stream(torch, sgm, ctx, lambda i: [sgm.Frame.alloc(p, L, R)],
                                   args.steps, args.warmup)
    # the same loop again with per-stage HIP events (they add a marker per
    # stage boundary, so they stay out of the timed loops); the aggregation
    # kernel's event-timed duration gives the roofline position
    sgm.sgm_profile(ctx, True)
    sgm.sgm_profile_read(ctx, reset=True)
    dtp, _ = time_submit_stream(torch, sgm, ctx, lambda i: [sgm.Frame.alloc(p, L, R)],
                                args.steps, args.warmup)
    prof = sgm.sgm_profile_read(ctx, reset=True)
    # the headline: the context's default of 4 streams, one frame per
    # submit; consecutive frames overlap on the GPU (one frame's
    # aggregation next to the next frame's Census and the previous one's
    # disparity selection)
    sgm.sgm_profile(ctx, False)
    sgm.sgm_set_streams(ctx, HEADLINE_STREAMS)
    dt, outs4 = time_submit_stream(torch, sgm, ctx, lambda i: [sgm.Frame.alloc(p, L, R)],
                                   args.steps, args.warmup)
    same_as_one_stream = all(torch.equal(a[0].disp, b[0].disp) and torch.equal(a[0].umap, b[0].umap)
                             and torch.equal(a[0].vmap, b[0].vmap) for a, b in zip(outs, outs4))
    # and in graph mode (captured batches replayed from the graph cache)
    sgm.sgm_set_streams(ctx, 1)
    sgm.sgm_set_graphs(ctx, True)
    dtg, _ = time_submit_stream(torch, sgm, ctx, lambda i: [sgm.Frame.alloc(p, L, R)],
                                args.steps, args.warmup)
    sgm.sgm_set_graphs(ctx, False)
    # the secondary measurements below choose their own stream counts; the
    # batch comparisons run on one stream
    evals = p.disp_evals()
    value = evals * args.steps / dt / 1e6
    # per-stage averages over the profiled loop (warm-up + timed steps)
    n_batches = args.steps + args.warmup
    stage_avg_ms = {k: v[0] / max(v[1], 1) for k, v in prof.items()}
    agg_ms = stage_avg_ms["aggregate"]
    achieved = ALG_BYTES_PER_EVAL * evals / (agg_ms * 1e-3) / 1e9

    # frame latency of the fused path, one frame at a time (no stage
    # markers: they would add their own cost to every frame)
    lat = []
    for _ in range(200):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, outs[0]))
        lat.append(time.perf_counter() - t0)
    lat_ms = np.array(lat) * 1e3

    # per-frame stage-call path (materialised cost and S volumes)
    for _ in range(2):
        sgm.run_stages(ctx, p, L, R)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nst = 10
    for _ in range(nst):
        sgm.run_stages(ctx, p, L, R)
    torch.cuda.synchronize()
    stage_path = evals * nst / (time.perf_counter() - t0) / 1e6

    sgm.sgm_profile(ctx, True)  # the extras read stage times
    extras = {}
    if args.extras in ("batch", "all"):
        log("320x240 D=64 5x5 4 paths, WTA only")
        extras["small_320x240_d64_4path_wta"] = bench_small(torch, sgm, ctx, synthetic)
        log("paper settings 640x360 D=60, Census and SAD")
        extras["paper_640x360_d60_4path"] = bench_paper_settings(torch, sgm, ctx, synthetic)
        log("batch of 32 mixed pairs")
        extras["batch32_mixed"] = bench_batch32(torch, sgm, ctx, synthetic)
    if args.extras in ("large", "batch", "all"):
        log("batch of 8 1920x1080 D=256")
        extras["batch8_1920x1080_d256"] = bench_large(torch, sgm, ctx, synthetic)
    if args.extras in ("serve", "all"):
        log("request loop, 4 cameras,", args.serve_seconds, "s per mode")
        extras["served"] = bench_serve(torch, sgm, synthetic, serve_ctx, args.serve_seconds)
    ctx.close()
    serve_ctx.close()

    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(left, right, p, args.cpu_seconds)
    # the aggregation kernel instance the schedule selects: K = 8 disparities
    # per lane over 16 lanes (D = 128), K * 16 / h_lanes on the horizontal paths
    traffic = measured_traffic("agg_kernel<8, %d, %d, 0, unsigned char" % (128 // h_lanes, h_lanes))

    line = {
        "metric": "SGM Mdisp-evals/s (W\u00b7H\u00b7D\u00b7paths) + p99 frame latency, batched vs per-frame",
        "value": round(value, 2),
        "unit": "Mdisp-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": "1242x375 uint8 pair, D=128, Census 9x7, 8 paths, P1=10, P2=120, "
                               "LR |dL-dR|<=1, 3x3 median, U/V maps (KITTI-shaped slanted planes)",
                   "frames_per_step": 1, "streams": HEADLINE_STREAMS,
                   "path": "sgm_submit (fused kernels), up to 8 frames in flight",
                   "schedule": {"h_lanes": h_lanes, "autotune_ms": tune_ms}},
        "fps": round(args.steps / dt, 1),
        "frame_latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        # the request loop's frame latency (arrival to result) at 4 cameras x
        # 30 fps: continuous batching vs one frame at a time, same trace
        "served_p99_ms": served_p99(extras),
        "stage_avg_ms": {k: round(v, 5) for k, v in stage_avg_ms.items()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "agg_kernel<8, %d, %d, 0, unsigned char> (8 directions, uint8 costs, uint8 path costs)"
                               % (128 // h_lanes, h_lanes),
                     "alg_bytes_per_launch": ALG_BYTES_PER_EVAL * evals,
                     "avg_launch_ms": round(agg_ms, 5), "launches": prof["aggregate"][1],
                     "batches_profiled": n_batches},
        "per_frame_stage_calls_mdisp_evals_per_s": round(stage_path, 2),
        "one_stream_mdisp_evals_per_s": round(evals * args.steps / dt1 / 1e6, 2),
        "one_stream_ms_per_step": round(dt1 / args.steps * 1e3, 4),
        "headline_outputs_equal_one_stream": same_as_one_stream,
        "profiled_loop_mdisp_evals_per_s": round(evals * args.steps / dtp / 1e6, 2),
        "graph_mode_mdisp_evals_per_s": round(evals * args.steps / dtg / 1e6, 2),
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
