"""Bit-exact parity of each C-ABI stage with the CPU oracle (GPU required).

Every stage output is integer, so the bar is exact equality on every element.
Sizes span several tiles / waves with ragged tails, plus the degenerate
shapes (1 x 1 images, single rows/columns, D larger than W, D not a multiple
of 64, D = 256)."""
import numpy as np
import pytest

from gen import synthetic
from gpu_util import announce, assert_equal, gpu_or_skip, to_dev, to_np
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = gpu_or_skip()
    from paper_1807_06271_amd import sgm
    ctx = sgm.Context(0)
    yield torch, sgm, ctx
    torch.cuda.synchronize()
    ctx.close()


def params(sgm, W, H, D, **kw):
    return sgm.Params(width=W, height=H, max_disp=D, **kw)


@pytest.mark.parametrize("W,H", [(1, 1), (5, 3), (67, 33), (320, 240)])
@pytest.mark.parametrize("cw,ch", [(5, 5), (9, 7), (3, 3), (1, 3), (13, 5)])
def test_census(env, W, H, cw, ch):
    torch, sgm, ctx = env
    announce("census", W, H, cw, ch)
    rng = np.random.default_rng(W * 1000 + H + cw)
    pitch = W + 7
    img = synthetic.random_image(rng, H, pitch, levels=8)  # few levels: many ties
    d_img = to_dev(torch, img)
    out = torch.empty((H, W), dtype=torch.uint64, device="cuda")
    p = params(sgm, W, H, 16, census_w=cw, census_h=ch)
    sgm.sgm_census(ctx, p, d_img[:, :pitch], out)
    torch.cuda.synchronize()
    assert_equal(to_np(out), O.census(img[:, :W], cw, ch), "census")


@pytest.mark.parametrize("W,H,D", [(7, 3, 1), (7, 3, 16), (200, 17, 60), (333, 41, 129),
                                   (130, 9, 256), (64, 2, 64)])
def test_cost(env, W, H, D):
    torch, sgm, ctx = env
    announce("cost", W, H, D)
    rng = np.random.default_rng(W + H + D)
    nb = 62
    cl = rng.integers(0, 1 << nb, size=(H, W), dtype=np.uint64)
    cr = rng.integers(0, 1 << nb, size=(H, W), dtype=np.uint64)
    out = torch.empty((H, W, D), dtype=torch.uint16, device="cuda")
    sgm.sgm_cost(ctx, params(sgm, W, H, D), to_dev(torch, cl), to_dev(torch, cr), out)
    torch.cuda.synchronize()
    assert_equal(to_np(out), O.cost(cl, cr, D, nb), "cost")


AGG_SHAPES = [(1, 1, 1), (9, 1, 5), (1, 9, 7), (37, 23, 64), (23, 37, 65), (70, 31, 128),
              (31, 70, 130), (45, 20, 200), (40, 26, 256), (3, 50, 100)]


@pytest.mark.parametrize("bit", range(8))
@pytest.mark.parametrize("W,H,D", AGG_SHAPES)
def test_aggregate_single_path(env, bit, W, H, D):
    torch, sgm, ctx = env
    announce("aggregate", "dir", bit, W, H, D)
    rng = np.random.default_rng(bit * 7919 + W * 31 + H * 7 + D)
    p = params(sgm, W, H, D, path_mask=1 << bit, p1=7, p2=90)
    c = synthetic.random_cost(rng, H, W, D, p.nbits)
    out = torch.empty((H, W, D), dtype=torch.uint16, device="cuda")
    sgm.sgm_aggregate(ctx, p, to_dev(torch, c), out)
    torch.cuda.synchronize()
    assert_equal(to_np(out), O.aggregate(c, 1 << bit, 7, 90), "L_r dir %d" % bit)


@pytest.mark.parametrize("D", [64, 60, 61])
def test_aggregate_cost_at_odd_address(env, D):
    # a uint16 cost volume starting 2 bytes past a 4-byte boundary: the
    # aggregation must not take its vector cost loads there
    torch, sgm, ctx = env
    W, H = 45, 19
    announce("aggregate odd address", W, H, D)
    rng = np.random.default_rng(D)
    p = params(sgm, W, H, D, path_mask=0xFF, p1=7, p2=90)
    c = synthetic.random_cost(rng, H, W, D, p.nbits)
    flat = torch.zeros(H * W * D + 1, dtype=torch.uint16, device="cuda")
    flat[1:] = to_dev(torch, c).view(-1)
    out = torch.empty((H, W, D), dtype=torch.uint16, device="cuda")
    sgm.sgm_aggregate(ctx, p, flat[1:].view(H, W, D), out)
    torch.cuda.synchronize()
    assert_equal(to_np(out), O.aggregate(c, 0xFF, 7, 90), "S")


@pytest.mark.parametrize("mask", [0x0F, 0xFF, 0x55, 0xF0, 0x03])
@pytest.mark.parametrize("W,H,D,cw,ch,p1,p2", [
    (97, 61, 64, 5, 5, 10, 120),
    (130, 47, 128, 9, 7, 10, 120),
    (61, 40, 60, 5, 5, 8, 32),
    (50, 33, 100, 9, 7, 30, 400),   # N_b + P2 > 255: 16-bit path costs
    (20, 30, 256, 9, 7, 0, 0),      # zero penalties: S = P * C
])
def test_aggregate_masks(env, mask, W, H, D, cw, ch, p1, p2):
    torch, sgm, ctx = env
    announce("aggregate mask", hex(mask), W, H, D, p1, p2)
    rng = np.random.default_rng(mask + W + D + p2)
    p = params(sgm, W, H, D, census_w=cw, census_h=ch, path_mask=mask, p1=p1, p2=p2)
    c = synthetic.random_cost(rng, H, W, D, p.nbits)
    out = torch.empty((H, W, D), dtype=torch.uint16, device="cuda")
    sgm.sgm_aggregate(ctx, p, to_dev(torch, c), out)
    torch.cuda.synchronize()
    assert_equal(to_np(out), O.aggregate(c, mask, p1, p2), "S mask %x" % mask)


# the wide shapes split rows into 2, 3 and 4 segments (the last one ragged);
# the right-view keys of pixels near a segment border come from two segments
@pytest.mark.parametrize("W,H,D", [(1, 1, 1), (5, 4, 16), (97, 13, 60), (64, 9, 64), (100, 7, 100),
                                   (131, 11, 128), (77, 5, 256), (3, 6, 40), (600, 5, 32), (1100, 3, 128),
                                   (1601, 2, 200)])
@pytest.mark.parametrize("lr,med", [(0, 0), (1, 0), (1, 3), (1, 5), (0, 5)])
def test_disparity(env, W, H, D, lr, med):
    torch, sgm, ctx = env
    announce("disparity", W, H, D, lr, med)
    rng = np.random.default_rng(W * 13 + H + D + 100 * lr + med)
    s = synthetic.random_cost(rng, H, W, D, 6)  # narrow range: many ties in WTA and D_R
    s[rng.random((H, W, D)) < 0.02] = 1000
    p = params(sgm, W, H, D, lr_check=lr, median=med, lr_max_diff=1)
    out = torch.empty((H, W), dtype=torch.uint16, device="cuda")
    sgm.sgm_disparity(ctx, p, to_dev(torch, s), out)
    torch.cuda.synchronize()
    dl = O.wta(s)
    dlr = O.lr_check(dl, O.right_disparity(s), 1, p.inv()) if lr else dl
    want = O.median(dlr, med) if med else dlr
    assert_equal(to_np(out), want, "disparity")


@pytest.mark.parametrize("maxdiff", [0, 2])
def test_disparity_lr_max_diff(env, maxdiff):
    torch, sgm, ctx = env
    announce("disparity maxdiff", maxdiff)
    rng = np.random.default_rng(maxdiff)
    W, H, D = 90, 10, 32
    s = synthetic.random_cost(rng, H, W, D, 40)
    p = params(sgm, W, H, D, lr_check=1, median=0, lr_max_diff=maxdiff, invalid=999)
    out = torch.empty((H, W), dtype=torch.uint16, device="cuda")
    sgm.sgm_disparity(ctx, p, to_dev(torch, s), out)
    torch.cuda.synchronize()
    assert_equal(to_np(out), O.lr_check(O.wta(s), O.right_disparity(s), maxdiff, 999), "lr")


@pytest.mark.parametrize("W,H,D", [(1, 1, 1), (63, 5, 64), (65, 130, 128), (200, 3, 256), (7, 300, 16)])
def test_uv_maps(env, W, H, D):
    torch, sgm, ctx = env
    announce("uv", W, H, D)
    rng = np.random.default_rng(W + H + D)
    disp = rng.integers(0, D, size=(H, W)).astype(np.uint16)
    inv = 255 if D <= 255 else 65535
    disp[rng.random((H, W)) < 0.15] = inv
    p = params(sgm, W, H, D)
    u = torch.empty((D, W), dtype=torch.uint16, device="cuda")
    v = torch.empty((H, D), dtype=torch.uint16, device="cuda")
    sgm.uv_maps(ctx, p, to_dev(torch, disp), u, v)
    torch.cuda.synchronize()
    wu, wv = O.uv_maps(disp, D)
    assert_equal(to_np(u), wu, "U")
    assert_equal(to_np(v), wv, "V")


def test_stage_errors_are_reported(env):
    torch, sgm, ctx = env
    p = params(sgm, 16, 8, 16)
    host = torch.empty((8, 16), dtype=torch.uint64)
    img = torch.zeros((8, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(TypeError):
        sgm.sgm_census(ctx, p, img, host)
    bad = params(sgm, 16, 8, 16, median=4)
    out = torch.empty((8, 16), dtype=torch.uint64, device="cuda")
    with pytest.raises(sgm.SgmError) as e:
        sgm.sgm_census(ctx, bad, img, out)
    assert e.value.status == sgm.SGM_EINVAL
