"""The allocation-free disparity selection (GPU required): sgm_disparity_noalloc
gives the same maps as sgm_disparity, bit for bit, on consecutive calls that
share the library's fixed scratch (the second with a smaller frame), and
rejects frames whose scratch exceeds it before enqueuing anything."""
import numpy as np
import pytest

from gen import synthetic
from gpu_util import announce, assert_equal, gpu_or_skip, to_dev, to_np

pytestmark = pytest.mark.gpu


def aggregated(torch, sgm, ctx, seed, W, H, D, **kw):
    left, right, _ = synthetic.make_pair("kitti", seed, W, H, D)
    p = sgm.Params(width=W, height=H, max_disp=D, **kw)
    out = sgm.run_stages(ctx, p, to_dev(torch, left), to_dev(torch, right), keep=True)
    torch.cuda.synchronize()
    return p, out["aggr"]


def test_noalloc_disparity_equals_disparity_on_consecutive_calls():
    torch = gpu_or_skip()
    from paper_1807_06271_amd import sgm
    with sgm.Context(0) as ctx:
        # a full 1242x375 D=128 frame (LR check inside the median), then a
        # smaller frame with other settings: the second call reuses the
        # scratch the first one left behind
        cases = [aggregated(torch, sgm, ctx, 71, 1242, 375, 128, median=3),
                 aggregated(torch, sgm, ctx, 72, 301, 97, 64, median=5),
                 aggregated(torch, sgm, ctx, 73, 150, 40, 60, lr_check=1, median=0),
                 aggregated(torch, sgm, ctx, 74, 97, 31, 32, lr_check=0, median=3)]
        stream = torch.cuda.current_stream()
        for rep in range(2):
            for p, S in cases:
                tag = "%dx%d D%d lr %d median %d (pass %d)" % (p.width, p.height, p.max_disp, p.lr_check,
                                                                 p.median, rep)
                announce("noalloc disparity", tag)
                want = torch.empty((p.height, p.width), dtype=torch.uint16, device="cuda")
                got = torch.empty_like(want)
                sgm.sgm_disparity(ctx, p, S, want, stream)
                sgm.sgm_disparity_noalloc(ctx, p, S, got, stream)
                torch.cuda.synchronize()
                assert_equal(to_np(got), to_np(want), "noalloc vs sgm_disparity " + tag)


def test_noalloc_disparity_rejects_oversized_frames():
    torch = gpu_or_skip()
    from paper_1807_06271_amd import sgm
    announce("noalloc disparity size limit")
    with sgm.Context(0) as ctx:
        p = sgm.Params(width=4096, height=4096, max_disp=64)   # 64 MiB of maps alone
        S = torch.empty((1, 1, 1), dtype=torch.uint16, device="cuda")
        out = torch.empty((1, 1), dtype=torch.uint16, device="cuda")
        rc = sgm.lib().sgm_disparity_noalloc(ctx.handle, sgm.ctypes.byref(p.c()), S.data_ptr(),
                                             out.data_ptr(), None)
        assert rc == sgm.SGM_ENOMEM
        assert b"fixed scratch" in sgm.lib().sgm_last_error()
