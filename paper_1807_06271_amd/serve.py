"""Multi-camera request loop over sgm_submit / sgm_poll.

Simulated cameras deliver frame pairs at seeded Poisson arrival times.  Each
arriving pair is copied host-to-device from pinned memory, in one
asynchronous copy, into a free slot of its camera's device buffers (input
pair and output maps, allocated once and reused) and queued with an event
recorded after the copy; the batch that takes the frame waits for that event
on the GPU (sgm_submit_after), so the host never blocks on a copy.  The
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
    """Pre-rendered frame pairs of one camera, replayed cyclically; each pair
    is one pinned [2][H][W] buffer (left, right), so that one copy moves both
    views."""

    def __init__(self, params: sgm.Params, pairs):
        self.p = params
        self.host = []
        for l, r in pairs:
            t = torch.empty((2,) + tuple(l.shape), dtype=torch.uint8, pin_memory=True)
            t[0].copy_(torch.from_numpy(l))
            t[1].copy_(torch.from_numpy(r))
            self.host.append(t)

    def pair(self, k: int):
        t = self.host[k % len(self.host)]
        return t[0], t[1]


class _Slot:
    """Device buffers for one frame of a camera: the input pair, the output
    maps, and the marshalled sgm_frame that points at them."""

    __slots__ = ("inp", "frame", "args", "reuse_after")

    def __init__(self, p: sgm.Params, dev):
        self.inp = torch.empty((2, p.height, p.width), dtype=torch.uint8, device=dev)
        self.frame = sgm.Frame.alloc(p, self.inp[0], self.inp[1])
        self.args = self.frame.c()
        self.reuse_after = None  # event after the last read of the outputs


def _percentiles(lat_s):
    a = np.asarray(lat_s) * 1e3
    return {"p50_ms": float(np.percentile(a, 50)), "p99_ms": float(np.percentile(a, 99)),
            "mean_ms": float(a.mean()), "max_ms": float(a.max())}


def serve(ctx: sgm.Context, cameras, trace, continuous: bool = True, max_batch: int = 8,
          keep_maps: bool = True):
    """Replay `trace` [(t, camera, frame)] in real time.  Returns statistics
    and, with keep_maps, per (camera, frame) device copies (disparity map,
    U-map, V-map) of the maps computed, for later comparison (the copies are
    taken after the frame's latency is recorded)."""
    dev = torch.device("cuda", ctx.device)
    copy_stream = torch.cuda.Stream(device=dev)
    queued = collections.deque()   # (t_arrival, cam, k, slot, input-ready event)
    inflight = []                  # (ticket, [(t_arrival, cam, k, slot, event)])
    # idle slots per camera: a few allocated up front, more only if a camera
    # has more frames queued or in flight at once
    free = [[_Slot(cam.p, dev) for _ in range(4)] for cam in cameras]
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
        slot = free[ci].pop() if free[ci] else _Slot(cam.p, dev)
        ready = torch.cuda.Event()
        with torch.cuda.stream(copy_stream):
            if slot.reuse_after is not None:  # the last copy of its outputs
                copy_stream.wait_event(slot.reuse_after)
            slot.inp.copy_(cam.host[k % len(cam.host)], non_blocking=True)
            ready.record(copy_stream)
        return (t, ci, k, slot, ready)

    def finish(items, tdone):
        nonlocal evals, finished
        for (ta, ci, k, slot, _) in items:
            lat.append(tdone - ta)
            evals += slot.frame.p.disp_evals()
            finished += 1
        for (ta, ci, k, slot, _) in items:
            if keep_maps:
                f = slot.frame
                done_frames[(ci, k)] = (f.disp.clone(), f.umap.clone(), f.vmap.clone())
                slot.reuse_after = torch.cuda.Event()
                slot.reuse_after.record()
            free[ci].append(slot)

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
                    finish(items, time.perf_counter() - t0)
                else:
                    still.append((ticket, items))
            inflight = still
            # admission
            if queued and (continuous or not inflight):
                take = min(len(queued), max_batch if continuous else 1)
                items = [queued[j] for j in range(take)]
                ticket = sgm.try_submit(ctx, [it[3].args for it in items], after=[it[4] for it in items])
                if ticket is not None:
                    for _ in range(take):
                        queued.popleft()
                    if continuous:
                        inflight.append((ticket, items))
                    else:
                        sgm.sgm_wait(ctx, ticket)
                        finish(items, time.perf_counter() - t0)
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
