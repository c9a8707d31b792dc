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


# shapes whose horizontal scanlines can form their costs from Census codes
# (64 lanes, 2 or 4 disparities per lane): W, H, D, census, mask, p1, p2
HCODE_SHAPES = [
    (203, 61, 128, (9, 7), 0xFF, 10, 120),
    (97, 33, 256, (9, 7), 0x03, 10, 120),
    (140, 37, 100, (9, 7), 0xFF, 10, 120),   # padded disparity rows
    (300, 20, 250, (9, 7), 0x03, 10, 120),   # padded, D = 250
    (64, 40, 128, (5, 5), 0x03, 10, 120),    # narrower than D: every pixel near the left border
    (1, 3, 256, (9, 7), 0x03, 10, 120),
    (257, 9, 200, (7, 7), 0x02, 7, 90),      # right to left alone
    (1500, 4, 128, (9, 7), 0x01, 10, 120),   # left to right alone, long rows
]


@pytest.mark.parametrize("shape", HCODE_SHAPES)
def test_horizontal_costs_from_census_codes_match_oracle(env, shape):
    torch, sgm, ctx = env
    W, H, D, (cw, ch), mask, p1, p2 = shape
    announce("horizontal costs from codes", shape)
    left, right, _ = synthetic.make_pair("kitti", W + 3 * D + mask, W, H, D)
    p = sgm.Params(width=W, height=H, max_disp=D, census_w=cw, census_h=ch, path_mask=mask, p1=p1, p2=p2,
                   invalid=65535 if D == 256 else 255)
    sgm.sgm_set_schedule(ctx, p, 64, h_costs=sgm.HCOSTS_CODES)
    assert sgm.schedule_of(ctx, p)[3] == sgm.HCOSTS_CODES
    f = sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right))
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
    want = O.sgm(left, right, D, cw, ch, mask, p1, p2, True, 1, 3, p.inv())
    assert_equal(to_np(f.disp), want["disp"], "disp")
    assert_equal(to_np(f.umap), want["umap"], "umap")
    assert_equal(to_np(f.vmap), want["vmap"], "vmap")


def test_horizontal_code_costs_fall_back_where_they_do_not_apply(env):
    # 32 lanes, D = 64 (one disparity per lane pair), 16-bit path costs, SAD:
    # the horizontal scanlines read the cost volume whatever the schedule says
    torch, sgm, ctx = env
    announce("horizontal costs fallback")
    for kw in (dict(width=120, height=30, max_disp=128), dict(width=120, height=30, max_disp=64),
               dict(width=120, height=30, max_disp=128, p2=300),
               dict(width=120, height=30, max_disp=128, census_w=5, census_h=5, cost=sgm.COST_SAD, p1=200, p2=800)):
        p = sgm.Params(**kw)
        h = 32 if kw["max_disp"] == 128 and "p2" not in kw and "cost" not in kw else 64
        sgm.sgm_set_schedule(ctx, p, h, h_costs=sgm.HCOSTS_CODES)
        assert sgm.schedule_of(ctx, p)[3] == sgm.HCOSTS_VOLUME, kw
        left, right, _ = synthetic.make_pair("kitti", 61, p.width, p.height, p.max_disp)
        f = sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right))
        sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
        want = O.sgm(left, right, p.max_disp, p.census_w, p.census_h, p.path_mask, p.p1, p.p2, True, 1, 3,
                     cost_kind=p.cost)
        assert_equal(to_np(f.disp), want["disp"], "disp %s" % kw)


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
    # first lanes (16, 32, 64 with costs from the volume, 64 with costs from
    # Census windows), then the disparity block size; no two-pass stripes
    # (one 300-column frame has 5 or 10 stripes, below the 128 a batch needs)
    # and no sweep (9x7 codes, D = 128)
    stage1 = ("h_lanes=16", "h_lanes=32", "h_lanes=64", "h_costs=codes")
    want = set(stage1) | {"disp_threads=256", "disp_threads=512", "disp_threads=1024"}
    assert best["two_pass"] == "off"
    assert set(ms) == want
    assert all(v > 0 for v in ms.values())
    first = min(stage1, key=lambda k: ms[k])
    assert best["h_lanes"] == (64 if first == "h_costs=codes" else int(first.split("=")[1]))
    assert (best["h_costs"] == "codes") == (first == "h_costs=codes") and not best["sweep"]
    overall = min(ms.values())
    if best["two_pass"] != "off":
        chosen = "two_pass=" + best["two_pass"]
    else:
        chosen = "disp_threads=%d" % best["disp_threads"] if best["disp_threads"] else first
    assert ms[chosen] == overall
    hc = sgm.HCOSTS_CODES if best["h_costs"] == "codes" else sgm.HCOSTS_VOLUME
    assert sgm.schedule_of(ctx, p)[:4] == (best["h_lanes"], False, best["disp_threads"], hc)
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
    want = O.sgm(left, right, D, 9, 7, 0xFF, 10, 120, True, 1, 3)
    assert_equal(to_np(f.disp), want["disp"], "disp after autotune")


def test_autotune_on_a_batch_sample(env):
    # the sample may be a batch of frames of one shape (tuned as one submit);
    # frames of another shape are refused
    torch, sgm, ctx = env
    announce("autotune on a batch")
    W, H, D = 260, 70, 256
    p = sgm.Params(width=W, height=H, max_disp=D, invalid=65535)
    frames, inputs = [], []
    for k in range(3):
        left, right, _ = synthetic.make_pair("kitti", 81 + k, W, H, D)
        frames.append(sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right)))
        inputs.append((left, right))
    best, ms = sgm.sgm_autotune(ctx, frames, reps=1)
    assert ms and all(v > 0 for v in ms.values()) and best["h_lanes"] in (16, 32, 64)
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
    for (left, right), f in zip(inputs, frames):
        want = O.sgm(left, right, D, 9, 7, 0xFF, 10, 120, True, 1, 3, 65535)
        assert_equal(to_np(f.disp), want["disp"], "disp after batch autotune")
    other = sgm.Params(width=W + 1, height=H, max_disp=D, invalid=65535)
    odd = sgm.Frame.alloc(other, to_dev(torch, synthetic.make_pair("kitti", 90, W + 1, H, D)[0]),
                          to_dev(torch, synthetic.make_pair("kitti", 90, W + 1, H, D)[1]))
    with pytest.raises(sgm.SgmError) as e:
        sgm.sgm_autotune(ctx, [frames[0], odd], reps=1)
    assert e.value.status == sgm.SGM_EINVAL


def test_autotune_considers_two_pass_on_large_batches(env):
    # 32 frames of 260 columns: 5 wide or 9 narrow stripes each, 160 and 288
    # in all, so both stripe widths are timed; the kept schedule gives the
    # oracle's maps for every frame
    torch, sgm, ctx = env
    announce("autotune with two-pass candidates")
    W, H, D = 260, 40, 256
    p = sgm.Params(width=W, height=H, max_disp=D, invalid=65535)
    left, right, _ = synthetic.make_pair("kitti", 95, W, H, D)
    L, R = to_dev(torch, left), to_dev(torch, right)
    frames = [sgm.Frame.alloc(p, L, R) for _ in range(32)]
    best, ms = sgm.sgm_autotune(ctx, frames, reps=1)
    assert {"two_pass=wide", "two_pass=narrow"} <= set(ms)
    assert best["two_pass"] in ("off", "wide", "narrow")
    for f in frames:
        f.disp.view(torch.int16).fill_(7)
    torch.cuda.synchronize()
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, frames))
    want = O.sgm(left, right, D, 9, 7, 0xFF, 10, 120, True, 1, 3, 65535)
    for i, f in enumerate(frames):
        assert_equal(to_np(f.disp), want["disp"], "disp frame %d after autotune" % i)
        assert_equal(to_np(f.vmap), want["vmap"], "vmap frame %d after autotune" % i)


def test_schedule_rejects_bad_values(env):
    torch, sgm, ctx = env
    with pytest.raises(sgm.SgmError):
        sgm.sgm_set_schedule(ctx, None, 48)
    with pytest.raises(sgm.SgmError):
        sgm.sgm_set_schedule(ctx, None, 0, h_costs=3)
    with pytest.raises(sgm.SgmError):
        sgm.sgm_set_schedule(ctx, None, 0, disp_threads=300)
