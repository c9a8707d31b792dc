"""Schedules and the autotuner (GPU required): every aggregation lane layout
gives output bit-identical to the oracle, and the autotuner keeps a valid
schedule for the shape."""
import numpy as np
import pytest

from gen import synthetic
from gpu_util import announce, assert_equal, gpu_or_skip, to_dev, to_np
from oracle import oracle as O

pytestmark = pytest.mark.gpu

SHAPES = [  # W, H, D, census, mask, p1, p2
    (203, 61, 128, (9, 7), 0xFF, 10, 120),
    (150, 40, 64, (5, 5), 0x0F, 10, 120),
    (97, 33, 256, (9, 7), 0x03, 10, 120),
    (120, 30, 192, (9, 7), 0xFF, 10, 120),
    (131, 47, 60, (5, 5), 0x55, 8, 32),     # padded disparity rows
    (90, 25, 100, (9, 7), 0xFF, 20, 300),   # padded, 16-bit path costs
    (140, 37, 100, (9, 7), 0xFF, 10, 120),  # padded, 8-bit path costs (one pair per lane at 64 lanes)
]
# SAD costs (16-bit cost volume, 16-bit path costs): W, H, D, window, mask
SAD_SHAPES = [(160, 40, 60, (5, 5), 0x55), (97, 21, 128, (5, 5), 0x0F), (70, 30, 64, (3, 3), 0xFF),
              (50, 12, 200, (5, 5), 0x03)]


@pytest.fixture(scope="module")
def env():
    torch = gpu_or_skip()
    from paper_1807_06271_amd import sgm
    ctx = sgm.Context(0)
    yield torch, sgm, ctx
    torch.cuda.synchronize()
    ctx.close()


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("h_lanes", [16, 32, 64])
def test_every_lane_layout_matches_oracle(env, shape, h_lanes):
    torch, sgm, ctx = env
    W, H, D, (cw, ch), mask, p1, p2 = shape
    announce("schedule", h_lanes, shape)
    left, right, _ = synthetic.make_pair("kitti", W + D + mask, W, H, D)
    p = sgm.Params(width=W, height=H, max_disp=D, census_w=cw, census_h=ch, path_mask=mask, p1=p1, p2=p2)
    sgm.sgm_set_schedule(ctx, p, h_lanes)
    used = sgm.sgm_get_schedule(ctx, p)
    assert used in (16, 32, 64) and (used == h_lanes or used < h_lanes)
    f = sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right))
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
    want = O.sgm(left, right, D, cw, ch, mask, p1, p2, True, 1, 3, p.inv())
    assert_equal(to_np(f.disp), want["disp"], "disp h_lanes=%d" % h_lanes)
    assert_equal(to_np(f.umap), want["umap"], "umap")
    assert_equal(to_np(f.vmap), want["vmap"], "vmap")


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("h_lanes", [16, 32, 64])
def test_census_cost_source_matches_oracle(env, shape, h_lanes):
    # the aggregation computes the Hamming costs from the Census codes (no
    # cost volume); frames whose path costs need 16 bits keep the volume
    torch, sgm, ctx = env
    W, H, D, (cw, ch), mask, p1, p2 = shape
    announce("census cost source", h_lanes, shape)
    left, right, _ = synthetic.make_pair("kitti", W + D + mask + 7, W, H, D)
    p = sgm.Params(width=W, height=H, max_disp=D, census_w=cw, census_h=ch, path_mask=mask, p1=p1, p2=p2)
    sgm.sgm_set_schedule(ctx, p, h_lanes, cost_source=sgm.COSTS_CENSUS)
    fits8 = p.nbits + p2 <= 255
    assert sgm.schedule_of(ctx, p)[2] == (sgm.COSTS_CENSUS if fits8 else sgm.COSTS_VOLUME)
    f = sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right))
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
    want = O.sgm(left, right, D, cw, ch, mask, p1, p2, True, 1, 3, p.inv())
    assert_equal(to_np(f.disp), want["disp"], "disp h_lanes=%d" % h_lanes)
    assert_equal(to_np(f.umap), want["umap"], "umap")
    assert_equal(to_np(f.vmap), want["vmap"], "vmap")


@pytest.mark.parametrize("W,H,D,mask", [(1, 1, 1, 0xFF), (5, 40, 64, 0xFF), (63, 9, 64, 0x0F), (70, 20, 256, 0xFF),
                                        (257, 3, 256, 0x03), (20, 300, 128, 0xF0), (33, 33, 60, 0x55)])
def test_census_cost_source_near_the_left_border(env, W, H, D, mask):
    # frames narrower than (or close to) the disparity range: most costs
    # belong to right-view pixels left of the image (cost N_b), on every
    # path direction and lane layout
    torch, sgm, ctx = env
    announce("census cost source, narrow frame", W, H, D, hex(mask))
    left, right, _ = synthetic.make_pair("kitti", 5 * W + H, W, H, D)
    p = sgm.Params(width=W, height=H, max_disp=D, census_w=9, census_h=7, path_mask=mask,
                   invalid=65535 if D == 256 else 255)
    for h_lanes in (16, 64):
        sgm.sgm_set_schedule(ctx, p, h_lanes, cost_source=sgm.COSTS_CENSUS)
        f = sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right))
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
        want = O.sgm(left, right, D, 9, 7, mask, 10, 120, True, 1, 3, p.inv())
        assert_equal(to_np(f.disp), want["disp"], "disp h_lanes=%d" % h_lanes)
        assert_equal(to_np(f.umap), want["umap"], "umap h_lanes=%d" % h_lanes)


@pytest.mark.parametrize("graphs", [False, True])
def test_batch_mixing_cost_sources_matches_oracle(env, graphs):
    # one submit holding frames that take their costs from the volume, from
    # the Census codes, and from SAD (which always uses its volume)
    torch, sgm, ctx = env
    announce("mixed cost sources, graphs" if graphs else "mixed cost sources")
    specs = [(211, 57, 128, dict(), sgm.COSTS_CENSUS), (187, 40, 128, dict(median=5), sgm.COSTS_VOLUME),
             (96, 30, 64, dict(census_w=5, census_h=5, path_mask=0x0F, lr_check=0), sgm.COSTS_CENSUS),
             (120, 33, 60, dict(census_w=5, census_h=5, path_mask=0x55, p1=200, p2=800, cost=sgm.COST_SAD),
              sgm.COSTS_CENSUS),
             (64, 24, 256, dict(invalid=65535), sgm.COSTS_CENSUS)]
    items = []
    for k, (W, H, D, kw, src) in enumerate(specs):
        left, right, _ = synthetic.make_pair("kitti", 900 + k, W, H, D)
        p = sgm.Params(width=W, height=H, max_disp=D, **kw)
        sgm.sgm_set_schedule(ctx, p, 0, cost_source=src)
        items.append((p, left, right, sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right))))
    sgm.sgm_set_graphs(ctx, graphs)
    try:
        for rep in range(2 if graphs else 1):
            frames = [sgm.Frame.alloc(p, f.left, f.right) for p, _, _, f in items]
            sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
            for (p, left, right, _), f in zip(items, frames):
                want = O.sgm(left, right, p.max_disp, p.census_w, p.census_h, p.path_mask, p.p1, p.p2,
                             bool(p.lr_check), p.lr_max_diff, p.median, p.inv(), cost_kind=p.cost)
                tag = "%dx%d D%d rep %d" % (p.width, p.height, p.max_disp, rep)
                assert_equal(to_np(f.disp), want["disp"], "disp " + tag)
                assert_equal(to_np(f.umap), want["umap"], "umap " + tag)
                assert_equal(to_np(f.vmap), want["vmap"], "vmap " + tag)
    finally:
        sgm.sgm_set_graphs(ctx, False)


@pytest.mark.parametrize("shape", SAD_SHAPES)
@pytest.mark.parametrize("h_lanes", [16, 32, 64])
def test_every_lane_layout_matches_oracle_sad(env, shape, h_lanes):
    torch, sgm, ctx = env
    W, H, D, (cw, ch), mask = shape
    announce("schedule sad", h_lanes, shape)
    left, right, _ = synthetic.make_pair("kitti", W + D + mask + 1, W, H, D)
    p = sgm.Params(width=W, height=H, max_disp=D, census_w=cw, census_h=ch, path_mask=mask, p1=200, p2=800,
                   cost=sgm.COST_SAD, median=5)
    sgm.sgm_set_schedule(ctx, p, h_lanes)
    f = sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right))
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
    want = O.sgm(left, right, D, cw, ch, mask, 200, 800, True, 1, 5, p.inv(), cost_kind=1)
    assert_equal(to_np(f.disp), want["disp"], "disp h_lanes=%d" % h_lanes)
    assert_equal(to_np(f.umap), want["umap"], "umap")


def test_autotune_keeps_a_valid_schedule(env):
    torch, sgm, ctx = env
    announce("autotune")
    W, H, D = 300, 90, 128
    left, right, _ = synthetic.make_pair("kitti", 77, W, H, D)
    p = sgm.Params(width=W, height=H, max_disp=D)
    f = sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right))
    best, ms = sgm.sgm_autotune(ctx, f, reps=2)
    assert best in ms and set(ms) == {16, 32, 64}
    assert all(v > 0 for v in ms.values())
    assert best == min(ms, key=ms.get)
    assert sgm.sgm_get_schedule(ctx, p) == best
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
    want = O.sgm(left, right, D, 9, 7, 0xFF, 10, 120, True, 1, 3)
    assert_equal(to_np(f.disp), want["disp"], "disp after autotune")


def test_schedule_rejects_bad_values(env):
    torch, sgm, ctx = env
    with pytest.raises(sgm.SgmError):
        sgm.sgm_set_schedule(ctx, None, 48)
    with pytest.raises(sgm.SgmError):
        sgm.sgm_set_schedule(ctx, None, 0, cost_source=3)
