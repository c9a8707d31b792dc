"""The two-pass stripe schedule (GPU required): T->B and TL->BR in a
top-down pass over stripes of 64 or 32 columns, B->T and BR->TL with the sum
over all 8 paths and the disparity selection in a bottom-up pass (section
3.1.3), the four other paths in per-direction kernels.  Every shape -- one
stripe or many, a ragged last stripe, padded disparity rows, every
disparities-per-lane width, with and without the LR check and median --
must give the oracle's disparity map and U/V maps bit for bit."""
import numpy as np
import pytest

from gen import synthetic
from gpu_util import announce, assert_equal, gpu_or_skip, to_dev, to_np
from oracle import oracle as O

pytestmark = pytest.mark.gpu

# W, H, D, census, p1, p2, lr_check, median
SHAPES = [
    (203, 61, 128, (9, 7), 10, 120, 1, 3),     # 4 wide stripes, the last ragged
    (64, 20, 64, (5, 5), 8, 32, 1, 3),         # exactly one wide stripe
    (97, 33, 256, (9, 7), 10, 120, 1, 5),
    (140, 37, 100, (9, 7), 10, 120, 1, 3),     # padded disparity rows
    (120, 30, 192, (9, 7), 10, 120, 0, 0),     # 12 disparities per lane, no LR, no median
    (33, 9, 60, (5, 5), 7, 90, 1, 0),          # LR check without a median
    (1, 5, 64, (5, 5), 10, 120, 1, 3),         # one column
    (300, 1, 128, (9, 7), 10, 120, 1, 3),      # one row
    (257, 40, 250, (9, 7), 10, 120, 1, 3),
    (1, 6, 120, (9, 7), 10, 120, 1, 3),        # one column, 8 disparities per lane (code records too)
    (65, 3, 256, (9, 7), 10, 120, 1, 3),       # a second wide stripe with one live column
]


@pytest.fixture(scope="module")
def env():
    torch = gpu_or_skip()
    from paper_1807_06271_amd import sgm
    ctx = sgm.Context(0)
    yield torch, sgm, ctx
    torch.cuda.synchronize()
    ctx.close()


def params(sgm, W, H, D, cw, ch, p1, p2, lr, med):
    return sgm.Params(width=W, height=H, max_disp=D, census_w=cw, census_h=ch, path_mask=0xFF, p1=p1, p2=p2,
                      lr_check=lr, median=med, invalid=65535 if D > 255 else 255)


def oracle_maps(p, left, right):
    out = O.sgm(left, right, p.max_disp, p.census_w, p.census_h, p.path_mask, p.p1, p.p2, bool(p.lr_check),
                p.lr_max_diff, p.median, p.inv())
    return out["disp"], out["umap"], out["vmap"]


def check(f, want, tag):
    assert_equal(to_np(f.disp), want[0], "disp " + tag)
    assert_equal(to_np(f.umap), want[1], "umap " + tag)
    assert_equal(to_np(f.vmap), want[2], "vmap " + tag)


# a batch runs its two-pass frames as such only with at least this many
# stripes in all (else on the per-direction kernels)
MIN_STRIPES = 128


def copies_for(W, mode):
    stripes = -(-W // (64 if mode == "wide" else 32))
    return -(-MIN_STRIPES // stripes)


def lanes_k(D):
    # disparities per lane of a 16-lane pixel
    return 4 if D <= 64 else 8 if D <= 128 else 12 if D <= 192 else 16


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("mode", ["wide", "narrow"])
@pytest.mark.parametrize("costs", ["volume", "codes"])
def test_two_pass_matches_oracle(env, shape, mode, costs):
    # the frame submitted as many times as it takes to reach the stripe
    # threshold (one launch then holds several job tables, each with its own
    # ticket counter); every copy must equal the oracle.  costs: the stripe
    # passes read the cost volume, or (64-lane horizontals on Census code
    # records, 8 or 16 disparities per lane) form the costs from the records
    torch, sgm, ctx = env
    W, H, D, (cw, ch), p1, p2, lr, med = shape
    if costs == "codes" and lanes_k(D) not in (8, 16):
        pytest.skip("Census code records exist for 8 or 16 disparities per lane")
    n = copies_for(W, mode)
    announce("two-pass", mode, costs, shape, n, "copies")
    left, right, _ = synthetic.make_pair("kitti", W + 7 * D + H, W, H, D)
    p = params(sgm, W, H, D, cw, ch, p1, p2, lr, med)
    tp = sgm.TWOPASS_WIDE if mode == "wide" else sgm.TWOPASS_NARROW
    if costs == "codes":
        sgm.sgm_set_schedule(ctx, p, 64, h_costs=sgm.HCOSTS_CODES, two_pass=tp)
        assert sgm.schedule_of(ctx, p)[3] == sgm.HCOSTS_CODES
    else:
        sgm.sgm_set_schedule(ctx, p, 0, h_costs=sgm.HCOSTS_VOLUME, two_pass=tp)
        assert sgm.schedule_of(ctx, p)[3] == sgm.HCOSTS_VOLUME
    assert sgm.schedule_of(ctx, p)[4] == tp
    L, R = to_dev(torch, left), to_dev(torch, right)
    frames = [sgm.Frame.alloc(p, L, R) for _ in range(n)]
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
    want = oracle_maps(p, left, right)
    for i, f in enumerate(frames):
        check(f, want, "%s %s copy %d" % (mode, shape, i))


def test_two_pass_does_not_apply_elsewhere(env):
    # 4 paths, SAD costs, 16-bit path costs: per-direction kernels whatever
    # the schedule says
    torch, sgm, ctx = env
    announce("two-pass fallback")
    for kw in (dict(width=90, height=20, max_disp=64, path_mask=0x55),
               dict(width=90, height=20, max_disp=64, census_w=5, census_h=5, cost=sgm.COST_SAD, p1=200, p2=800),
               dict(width=90, height=20, max_disp=64, p2=300)):
        p = sgm.Params(**kw)
        sgm.sgm_set_schedule(ctx, p, 0, two_pass=sgm.TWOPASS_WIDE)
        assert sgm.schedule_of(ctx, p)[4] == sgm.TWOPASS_OFF, kw
        left, right, _ = synthetic.make_pair("kitti", 5, p.width, p.height, p.max_disp)
        f = sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right))
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
        want = O.sgm(left, right, p.max_disp, p.census_w, p.census_h, p.path_mask, p.p1, p.p2, True, 1, 3,
                     cost_kind=p.cost)
        assert_equal(to_np(f.disp), want["disp"], "disp %s" % kw)


def test_mixed_batch_repeated_split_and_graphs(env):
    # frames on the two-pass schedule next to frames on the per-direction
    # kernels in one batch; the same batch again on the same scratch (stale
    # edge words of the previous launch must never be taken), split over the
    # context's streams, and replayed in graph mode
    torch, sgm, ctx = env
    announce("two-pass mixed batch")
    # six shapes, each frame 16 times (the two-pass ones: 160 stripes or
    # more); the last two-pass shape forms its stripe passes' costs from
    # Census code records, the others read the cost volume: separate
    # launches within each pass
    specs = [(150, 40, 128, 0xFF, sgm.TWOPASS_WIDE, False), (150, 40, 64, 0xFF, sgm.TWOPASS_NARROW, False),
             (130, 30, 128, 0x0F, sgm.TWOPASS_WIDE, False), (90, 44, 256, 0xFF, sgm.TWOPASS_OFF, False),
             (70, 25, 64, 0xFF, sgm.TWOPASS_WIDE, False), (160, 36, 256, 0xFF, sgm.TWOPASS_WIDE, True)]
    frames, want = [], []
    for i, (W, H, D, mask, tp, codes) in enumerate(specs):
        left, right, _ = synthetic.make_pair("kitti", 300 + i, W, H, D)
        p = sgm.Params(width=W, height=H, max_disp=D, path_mask=mask, invalid=65535 if D > 255 else 255)
        if codes:
            sgm.sgm_set_schedule(ctx, p, 64, h_costs=sgm.HCOSTS_CODES, two_pass=tp)
            assert sgm.schedule_of(ctx, p)[3] == sgm.HCOSTS_CODES
        else:
            sgm.sgm_set_schedule(ctx, p, 0, h_costs=sgm.HCOSTS_VOLUME, two_pass=tp)
        o = O.sgm(left, right, D, 9, 7, mask, 10, 120, True, 1, 3, p.inv())
        L, R = to_dev(torch, left), to_dev(torch, right)
        for _ in range(16):
            frames.append(sgm.Frame.alloc(p, L, R))
            want.append((o["disp"], o["umap"], o["vmap"]))
    try:
        for split in (1, 4):
            sgm.sgm_set_split(ctx, split)
            for rep in range(3):
                for f in frames:
                    f.disp.view(torch.int16).fill_(7)
                torch.cuda.synchronize()
                sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
                for i, f in enumerate(frames):
                    check(f, want[i], "split %d rep %d frame %d" % (split, rep, i))
        sgm.sgm_set_split(ctx, 1)
        sgm.sgm_set_graphs(ctx, True)
        for rep in range(3):
            for f in frames:
                f.disp.view(torch.int16).fill_(7)
            torch.cuda.synchronize()
            sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
            for i, f in enumerate(frames):
                check(f, want[i], "graph replay %d frame %d" % (rep, i))
    finally:
        sgm.sgm_set_graphs(ctx, False)
        sgm.sgm_set_split(ctx, 4)


def test_many_frames_in_one_launch(env):
    # 30 frames of two shapes: more stripe workgroups than the chip holds at
    # once in one launch (tickets keep the waits finite); two tables of jobs
    torch, sgm, ctx = env
    announce("two-pass 30 frames")
    frames, want = [], []
    for i in range(30):
        W, H, D = (640, 48, 128) if i % 2 == 0 else (333, 61, 64)
        left, right, _ = synthetic.make_pair("kitti", 500 + i, W, H, D)
        p = sgm.Params(width=W, height=H, max_disp=D)
        sgm.sgm_set_schedule(ctx, p, 0, two_pass=sgm.TWOPASS_NARROW)
        frames.append(sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right)))
        if i < 4:
            o = O.sgm(left, right, D, 9, 7, 0xFF, 10, 120, True, 1, 3)
            want.append((o["disp"], o["umap"], o["vmap"]))
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
    for i in range(4):
        check(frames[i], want[i], "frame %d" % i)
    # the rest equal the same frames run alone on the per-direction kernels
    for i in range(4, 30, 5):
        f = frames[i]
        sgm.sgm_set_schedule(ctx, f.p, 0, two_pass=sgm.TWOPASS_OFF)
        g = sgm.Frame.alloc(f.p, f.left, f.right)
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [g]))
        assert np.array_equal(to_np(g.disp), to_np(f.disp)), i
        assert np.array_equal(to_np(g.umap), to_np(f.umap)), i


def test_a_stripe_wait_that_gives_up_fails_the_batch(env):
    # the failure path forced from the host: stripes publish no edge records
    # and every wait gives up after 64 polls (the kernels still end); the
    # batch reports SGM_EHIP, and the context then works as before
    torch, sgm, ctx = env
    announce("two-pass failure path")
    W, H, D = 256, 24, 64  # 4 wide stripes per frame, 32 frames: 128
    p = sgm.Params(width=W, height=H, max_disp=D)
    left, right, _ = synthetic.make_pair("kitti", 77, W, H, D)
    L, R = to_dev(torch, left), to_dev(torch, right)
    frames = [sgm.Frame.alloc(p, L, R) for _ in range(32)]
    sgm.sgm_set_schedule(ctx, p, 0, two_pass=sgm.TWOPASS_WIDE)
    try:
        sgm.sgm_set_stripe_wait(ctx, 64, True)
        with pytest.raises(sgm.SgmError) as e:
            sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
        assert e.value.status == sgm.SGM_EHIP and "gave up waiting" in str(e.value)
    finally:
        sgm.sgm_set_stripe_wait(ctx, 0, False)
    with pytest.raises(sgm.SgmError):
        sgm.sgm_set_stripe_wait(ctx, -1, False)
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
    want = oracle_maps(params(sgm, W, H, D, 9, 7, 10, 120, 1, 3), left, right)
    for i, f in enumerate(frames):
        check(f, want, "frame %d after the failed batch" % i)
