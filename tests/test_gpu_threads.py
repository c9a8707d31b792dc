"""Concurrent use of the library (GPU required): several host threads
submitting and polling batches on one context, and two contexts running
stage calls on two streams at once, give the same results as the frames run
one at a time.  The C entry points serialise on a per-context lock and every
batch has its own scratch, so results must not depend on the interleaving."""
import threading
import time

import numpy as np
import pytest

from gen import synthetic
from gpu_util import announce, assert_equal, gpu_or_skip, to_dev, to_np

pytestmark = pytest.mark.gpu

SHAPES = [(320, 240, 64, 0x0F), (200, 90, 128, 0xFF), (160, 100, 60, 0x55), (97, 33, 32, 0x03)]


def frames_for(torch, sgm, k):
    W, H, D, mask = SHAPES[k % len(SHAPES)]
    left, right, _ = synthetic.make_pair("kitti", 900 + k, W, H, D)
    p = sgm.Params(width=W, height=H, max_disp=D, census_w=5, census_h=5, path_mask=mask, median=3)
    return p, to_dev(torch, left), to_dev(torch, right)


def test_threads_sharing_one_context():
    torch = gpu_or_skip()
    from paper_1807_06271_amd import sgm
    announce("4 threads x 6 batches on one context")
    inputs = [frames_for(torch, sgm, k) for k in range(8)]
    with sgm.Context(0) as ctx:
        # reference: every frame alone
        ref = []
        for p, L, R in inputs:
            f = sgm.Frame.alloc(p, L, R)
            sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
            ref.append((to_np(f.disp), to_np(f.umap), to_np(f.vmap)))
        torch.cuda.synchronize()
        errors, results = [], {}

        def worker(t):
            try:
                for rep in range(6):
                    ks = [(t + rep + i) % len(inputs) for i in range(1 + (t + rep) % 3)]
                    fs = [sgm.Frame.alloc(*inputs[k]) for k in ks]
                    tk = sgm.sgm_submit(ctx, fs)
                    while not sgm.sgm_poll(ctx, tk):
                        pass
                    results[(t, rep)] = [(k, to_np(f.disp), to_np(f.umap), to_np(f.vmap)) for k, f in zip(ks, fs)]
            except Exception as e:  # reported below, in the main thread
                errors.append(repr(e))

        threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
        for th in threads:
            th.start()
        for th in threads:
            th.join(timeout=120)
        assert not any(th.is_alive() for th in threads), "a worker did not finish"
        assert not errors, errors
        assert len(results) == 24
        for key, outs in results.items():
            for k, d, u, v in outs:
                assert_equal(d, ref[k][0], "disp frame %d in %s" % (k, key))
                assert_equal(u, ref[k][1], "umap frame %d in %s" % (k, key))
                assert_equal(v, ref[k][2], "vmap frame %d in %s" % (k, key))


def test_two_contexts_stage_calls_on_two_streams():
    torch = gpu_or_skip()
    from paper_1807_06271_amd import sgm
    announce("2 contexts, stage calls on 2 streams")
    inputs = [frames_for(torch, sgm, k) for k in (0, 1)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ctxs = [sgm.Context(0), sgm.Context(0)]
    try:
        alone = []
        for (p, L, R), c in zip(inputs, ctxs):
            alone.append(to_np(sgm.run_stages(c, p, L, R)["disp"]))
        torch.cuda.synchronize()
        outs = [None, None]

        def worker(i):
            p, L, R = inputs[i]
            with torch.cuda.stream(streams[i]):
                res = []
                for _ in range(5):
                    res.append(sgm.run_stages(ctxs[i], p, L, R, stream=streams[i])["disp"])
                streams[i].synchronize()
                outs[i] = [to_np(r) for r in res]

        threads = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
        for th in threads:
            th.start()
        for th in threads:
            th.join(timeout=120)
        for i in range(2):
            assert outs[i] is not None, "worker %d did not finish" % i
            for r in outs[i]:
                assert_equal(r, alone[i], "context %d" % i)
    finally:
        torch.cuda.synchronize()
        for c in ctxs:
            c.close()


def test_wait_does_not_hold_up_other_threads():
    # while one thread waits on a long batch, another thread's submit must
    # return at once (the waiting thread polls without holding the context's
    # lock), and both results must still equal the frames run alone
    torch = gpu_or_skip()
    from paper_1807_06271_amd import sgm
    announce("sgm_wait on a 16-frame batch while another thread submits")
    big = frames_for(torch, sgm, 1)
    W, H, D = 1242, 375, 128
    left, right, _ = synthetic.make_pair("kitti", 950, W, H, D)
    pb = sgm.Params(width=W, height=H, max_disp=D, census_w=9, census_h=7, path_mask=0xFF, median=3)
    Lb, Rb = to_dev(torch, left), to_dev(torch, right)
    with sgm.Context(0) as ctx:
        ref_big = sgm.Frame.alloc(pb, Lb, Rb)
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [ref_big]))
        ref_small = sgm.Frame.alloc(*big)
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [ref_small]))
        torch.cuda.synchronize()
        batch = [sgm.Frame.alloc(pb, Lb, Rb) for _ in range(16)]
        small = sgm.Frame.alloc(*big)
        submitted = threading.Event()
        times, errors = {}, []

        def waiter():
            try:
                tk = sgm.sgm_submit(ctx, batch)
                submitted.set()
                sgm.sgm_wait(ctx, tk)
                times["wait_returned"] = time.perf_counter()
            except Exception as e:  # reported below, in the main thread
                errors.append(repr(e))
                submitted.set()

        th = threading.Thread(target=waiter)
        th.start()
        assert submitted.wait(60)
        time.sleep(0.0005)  # the waiter is inside sgm_wait by now
        tk = sgm.sgm_submit(ctx, [small])
        times["submit_returned"] = time.perf_counter()
        sgm.sgm_wait(ctx, tk)
        th.join(timeout=120)
        assert not th.is_alive(), "the waiting thread did not finish"
        assert not errors, errors
        assert times["submit_returned"] < times["wait_returned"], "submit waited for the other thread's batch"
        for f in batch:
            assert_equal(to_np(f.disp), to_np(ref_big.disp), "batch frame disp")
        assert_equal(to_np(small.disp), to_np(ref_small.disp), "small frame disp")
