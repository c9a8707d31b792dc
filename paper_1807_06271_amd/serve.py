"""Multi-camera request loop over sgm_submit / sgm_poll.

Simulated cameras deliver frame pairs at seeded Poisson arrival times.  Each
arriving pair is copied host-to-device from pinned memory and queued.  The
loop then does continuous batching: whenever frames are queued it submits
them (as many as the context's memory budget admits next to the batches
still on the GPU), polls the batches in flight, and records each frame's
latency from its scheduled arrival to the moment a poll sees it finished
(the loop polls without sleeping while batches are in flight).  Batches go
to the context's own streams, so work of a batch submitted while others run
overlaps on the device.

The per-frame baseline serves the identical trace one frame at a time: each
frame is submitted alone and waited for before the next one starts.
"""
from __future__ import annotations

import collections
import gc
import time

import numpy as np
import torch

from . import sgm


class Camera:
    """Pre-rendered, pinned frame pairs of one camera, replayed cyclically."""

    def __init__(self, params: sgm.Params, pairs):
        self.p = params
        self.host = [(torch.from_numpy(l).pin_memory(), torch.from_numpy(r).pin_memory()) for l, r in pairs]

    def pair(self, k: int):
        return self.host[k % len(self.host)]


def _percentiles(lat_s):
    a = np.asarray(lat_s) * 1e3
    return {"p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
            "mean_ms": float(a.mean()), "max_ms": float(a.max())}


def serve(ctx: sgm.Context, cameras, trace, continuous: bool = True, max_batch: int = 8):
    """Replay `trace` [(t, camera, frame)] in real time.  Returns statistics
    and, per (camera, frame), the disparity map computed (on the GPU, not
    copied back) for later comparison."""
    dev = torch.device("cuda", ctx.device)
    copy_stream = torch.cuda.Stream(device=dev)
    queued = collections.deque()   # (t_arrival, cam, k, Frame)
    inflight = []                  # (ticket, [(t_arrival, cam, k, Frame)])
    lat, done_frames = [], {}
    i = 0
    n = len(trace)
    finished = 0
    evals = 0
    # no garbage-collector pauses inside the timed loop
    gc_was_enabled = gc.isenabled()
    gc.disable()
    t0 = time.perf_counter()

    def arrive(ev):
        t, ci, k = ev
        cam = cameras[ci]
        hl, hr = cam.pair(k)
        with torch.cuda.stream(copy_stream):
            L = hl.to(dev, non_blocking=True)
            R = hr.to(dev, non_blocking=True)
        copy_stream.synchronize()
        f = sgm.Frame.alloc(cam.p, L, R)
        return (t, ci, k, f)

    try:
        while finished < n:
            now = time.perf_counter() - t0
            # arrivals
            while i < n and trace[i][0] <= now:
                queued.append(arrive(trace[i]))
                i += 1
            # completions
            still = []
            for ticket, items in inflight:
                if sgm.sgm_poll(ctx, ticket):
                    tdone = time.perf_counter() - t0
                    for (ta, ci, k, f) in items:
                        lat.append(tdone - ta)
                        done_frames[(ci, k)] = f.disp
                        evals += f.p.disp_evals()
                        finished += 1
                else:
                    still.append((ticket, items))
            inflight = still
            # admission
            if queued and (continuous or not inflight):
                take = min(len(queued), max_batch if continuous else 1)
                items = [queued[j] for j in range(take)]
                ticket = sgm.try_submit(ctx, [it[3] for it in items])
                if ticket is not None:
                    for _ in range(take):
                        queued.popleft()
                    if continuous:
                        inflight.append((ticket, items))
                    else:
                        sgm.sgm_wait(ctx, ticket)
                        tdone = time.perf_counter() - t0
                        for (ta, ci, k, f) in items:
                            lat.append(tdone - ta)
                            done_frames[(ci, k)] = f.disp
                            evals += f.p.disp_evals()
                            finished += 1
                    continue
            if not queued and not inflight and i < n:
                # idle until the next arrival: sleep until shortly before it,
                # then poll, so that a late wake-up of the host thread does not
                # delay the frame
                dt = trace[i][0] - (time.perf_counter() - t0)
                if dt > 0.003:
                    time.sleep(dt - 0.002)
            # with batches in flight the loop polls without sleeping: a sleep
            # of the host thread adds its wake-up delay to every latency
    finally:
        if gc_was_enabled:
            gc.enable()
    wall = time.perf_counter() - t0
    stats = _percentiles(lat)
    stats.update(frames=finished, wall_s=wall, fps=finished / wall,
                 mdisp_evals_per_s=evals / wall / 1e6)
    return stats, done_frames
