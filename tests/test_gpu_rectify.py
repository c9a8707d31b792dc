"""Rectification by remap maps (section 3.1.1) on the GPU: sgm_rectify
against the oracle's gather, bit-exact, on synthetic calibration maps with
ragged widths, pitched and unaligned buffers, out-of-image entries and
batches of more images than one launch holds; then rectification ahead of
the whole disparity path."""
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


def raw_image(seed, src_w, src_h):
    return synthetic.random_image(np.random.default_rng(seed), src_h, src_w)


# (rectified w, h, raw w, h): one pixel, ragged tails, the paper's and a KITTI-like size
SIZES = [(1, 1, 1, 1), (7, 3, 9, 5), (37, 11, 40, 13), (129, 40, 140, 44), (640, 360, 672, 380),
         (1242, 375, 1280, 384)]


@pytest.mark.parametrize("w,h,sw,sh", SIZES)
def test_rectify_matches_oracle(env, w, h, sw, sh):
    torch, sgm, ctx = env
    announce("rectify", w, h, sw, sh)
    src = raw_image(w + h, sw, sh)
    mx, my = synthetic.rectification_maps(w, h, sw, sh, seed=w * h)
    out = torch.full((h, w), 77, dtype=torch.uint8, device="cuda")
    sgm.sgm_rectify(ctx, [(to_dev(torch, src), to_dev(torch, mx), to_dev(torch, my), out)])
    torch.cuda.synchronize()
    assert_equal(to_np(out), O.rectify(src, mx, my), "rectified %dx%d" % (w, h))


def test_rectify_pitched_unaligned_and_out_of_range(env):
    torch, sgm, ctx = env
    announce("rectify pitched/unaligned")
    w, h, sw, sh = 101, 23, 120, 30
    src = raw_image(5, sw, sh)
    mx, my = synthetic.rectification_maps(w, h, sw, sh, seed=9, angle_deg=8.0)
    mx[0, :5] = 65535                 # explicit "no source pixel"
    my[3, 7] = sh                     # first row beyond the image
    mx[4, 8] = sw                     # first column beyond the image
    src_big = torch.zeros((sh, sw + 13), dtype=torch.uint8, device="cuda")
    src_big[:, :sw] = to_dev(torch, src)
    flat_x = torch.zeros(w * h + 1, dtype=torch.uint16, device="cuda")
    flat_y = torch.zeros(w * h + 1, dtype=torch.uint16, device="cuda")
    flat_x[1:] = to_dev(torch, mx).view(-1)
    flat_y[1:] = to_dev(torch, my).view(-1)
    mx_u, my_u = flat_x[1:].view(h, w), flat_y[1:].view(h, w)   # 2-byte aligned maps
    out_big = torch.full((h, w + 6), 200, dtype=torch.uint8, device="cuda")
    out = out_big[:, 3:3 + w]                                      # pitched, unaligned output
    sgm.sgm_rectify(ctx, [(src_big[:, :sw], mx_u, my_u, out)])
    torch.cuda.synchronize()
    want = O.rectify(src, mx, my)
    assert_equal(to_np(out), want, "rectified")
    ob = to_np(out_big)
    assert (ob[:, :3] == 200).all() and (ob[:, 3 + w:] == 200).all(), "wrote outside the output rows"
    assert want[0, :5].max() == 0 and want[3, 7] == 0 and want[4, 8] == 0


def test_rectify_batch_of_many_images(env):
    # 30 images of mixed sizes: more than one launch's job table
    torch, sgm, ctx = env
    announce("rectify batch 30")
    rng = np.random.default_rng(3)
    jobs, want = [], []
    for i in range(30):
        w, h = int(rng.integers(1, 90)), int(rng.integers(1, 40))
        sw, sh = w + int(rng.integers(0, 20)), h + int(rng.integers(0, 10))
        src = raw_image(100 + i, sw, sh)
        mx, my = synthetic.rectification_maps(w, h, sw, sh, seed=i)
        out = torch.zeros((h, w), dtype=torch.uint8, device="cuda")
        jobs.append((to_dev(torch, src), to_dev(torch, mx), to_dev(torch, my), out))
        want.append(O.rectify(src, mx, my))
    sgm.sgm_rectify(ctx, jobs)
    sgm.sgm_rectify(ctx, [])          # empty batch: nothing enqueued
    torch.cuda.synchronize()
    for i, (j, wnt) in enumerate(zip(jobs, want)):
        assert_equal(to_np(j[3]), wnt, "image %d" % i)


def test_rectify_rejects_bad_jobs(env):
    torch, sgm, ctx = env
    announce("rectify validation")
    src = torch.zeros((10, 10), dtype=torch.uint8, device="cuda")
    m = torch.zeros((4, 4), dtype=torch.uint16, device="cuda")
    out = torch.zeros((4, 4), dtype=torch.uint8, device="cuda")
    good = sgm.remap_job(src, m, m, out)
    for field, value in [("w", 0), ("h", 16385), ("src_w", 0), ("src_h", 65536), ("src_pitch", 9),
                         ("out_pitch", 3)]:
        bad = sgm.remap_job(src, m, m, out)
        setattr(bad, field, value)
        with pytest.raises(sgm.SgmError) as e:
            sgm.sgm_rectify(ctx, [good, bad])
        assert e.value.status == sgm.SGM_EINVAL and "job 1" in str(e.value)
    host = np.zeros(16, np.uint16)
    bad = sgm.remap_job(src, m, m, out)
    bad.map_x = host.ctypes.data
    with pytest.raises(sgm.SgmError) as e:
        sgm.sgm_rectify(ctx, [bad])
    assert e.value.status == sgm.SGM_EINVAL


def paper_census(sgm, w=640, h=360, D=60):
    return sgm.Params(width=w, height=h, max_disp=D, census_w=5, census_h=5, path_mask=sgm.PATHS_PAPER4,
                      p1=8, p2=32, lr_check=1, median=5)


def oracle_rectified(sgm, p, raw_l, raw_r, maps):
    left, right = O.rectify(raw_l, *maps[0]), O.rectify(raw_r, *maps[1])
    O.set_threads(16)
    want = O.sgm(left, right, p.max_disp, p.census_w, p.census_h, p.path_mask, p.p1, p.p2, bool(p.lr_check),
                 p.lr_max_diff, p.median, p.inv())
    return left, right, want


def test_rectified_pair_through_the_whole_path(env):
    # raw pair -> rectification -> disparity path, the paper's setting, two
    # ways: sgm_rectify on the caller's stream, a host wait, sgm_submit; and
    # sgm_submit_rectify, which runs the rectification as the batch's first
    # stage.  Both against the oracle's rectify followed by its path.
    torch, sgm, ctx = env
    announce("rectify + submit, paper setting")
    w, h, D, sw, sh = 640, 360, 60, 672, 380
    raw_l, raw_r, _ = synthetic.make_pair("paper", 21, sw, sh, D)
    maps = [synthetic.rectification_maps(w, h, sw, sh, seed=1), synthetic.rectification_maps(w, h, sw, sh, seed=2)]
    dmaps = [tuple(to_dev(torch, m) for m in mm) for mm in maps]
    RL, RR = to_dev(torch, raw_l), to_dev(torch, raw_r)
    p = paper_census(sgm, w, h, D)
    left, right, want = oracle_rectified(sgm, p, raw_l, raw_r, maps)

    L = torch.empty((h, w), dtype=torch.uint8, device="cuda")
    R = torch.empty((h, w), dtype=torch.uint8, device="cuda")
    sgm.sgm_rectify(ctx, [(RL, *dmaps[0], L), (RR, *dmaps[1], R)])
    torch.cuda.synchronize()
    f = sgm.Frame.alloc(p, L, R)
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
    assert_equal(to_np(L), left, "rectified left")
    assert_equal(to_np(R), right, "rectified right")
    assert_equal(to_np(f.disp), want["disp"], "disp")

    L2 = torch.zeros((h, w + 32), dtype=torch.uint8, device="cuda")   # pitched view buffers
    R2 = torch.zeros((h, w + 32), dtype=torch.uint8, device="cuda")
    # the fills run on torch's stream; sgm_submit_rectify does not wait for it
    torch.cuda.synchronize()
    g = sgm.Frame.alloc(p, L2, R2)
    sgm.sgm_wait(ctx, sgm.sgm_submit_rectify(ctx, [g], [(RL, *dmaps[0]), (RR, *dmaps[1])]))
    assert_equal(to_np(L2)[:, :w], left, "rectified left (in batch)")
    assert_equal(to_np(R2)[:, :w], right, "rectified right (in batch)")
    assert_equal(to_np(g.disp), want["disp"], "disp (in batch)")
    assert_equal(to_np(g.umap), want["umap"], "umap (in batch)")
    assert_equal(to_np(g.vmap), want["vmap"], "vmap (in batch)")


@pytest.mark.parametrize("graphs", [False, True])
def test_submit_rectify_mixed_batch(env, graphs):
    # three frames of different sizes and costs, each with its own maps;
    # graph mode replays the captured batch with new raw images in between
    torch, sgm, ctx = env
    announce("submit_rectify mixed, graphs=%d" % graphs)
    sgm.sgm_set_graphs(ctx, graphs)
    try:
        specs = [(640, 360, 60, 672, 380, dict(census_w=5, census_h=5, path_mask=sgm.PATHS_PAPER4, p1=8, p2=32,
                                                    median=5)),
                 (203, 61, 128, 220, 64, dict(census_w=9, census_h=7)),
                 (90, 25, 60, 100, 30, dict(census_w=5, census_h=5, cost=sgm.COST_SAD, p1=200, p2=800,
                                            path_mask=sgm.PATHS_PAPER4))]
        for rep in range(3 if graphs else 1):
            frames, remaps, wants = [], [], []
            for k, (w, h, D, sw, sh, kw) in enumerate(specs):
                raw_l, raw_r, _ = synthetic.make_pair("kitti", 50 + 7 * k + rep, sw, sh, D)
                maps = [synthetic.rectification_maps(w, h, sw, sh, seed=2 * k),
                        synthetic.rectification_maps(w, h, sw, sh, seed=2 * k + 1)]
                p = sgm.Params(width=w, height=h, max_disp=D, **kw)
                frames.append(sgm.Frame.alloc(p, torch.empty((h, w), dtype=torch.uint8, device="cuda"),
                                              torch.empty((h, w), dtype=torch.uint8, device="cuda")))
                remaps += [(to_dev(torch, raw_l), *(to_dev(torch, m) for m in maps[0])),
                           (to_dev(torch, raw_r), *(to_dev(torch, m) for m in maps[1]))]
                left, right = O.rectify(raw_l, *maps[0]), O.rectify(raw_r, *maps[1])
                wants.append(O.sgm(left, right, D, p.census_w, p.census_h, p.path_mask, p.p1, p.p2,
                                   bool(p.lr_check), p.lr_max_diff, p.median, p.inv(), cost_kind=p.cost))
            sgm.sgm_wait(ctx, sgm.sgm_submit_rectify(ctx, frames, remaps))
            torch.cuda.synchronize()
            for f, want in zip(frames, wants):
                tag = "%dx%d rep %d" % (f.p.width, f.p.height, rep)
                assert_equal(to_np(f.disp), want["disp"], "disp " + tag)
                assert_equal(to_np(f.umap), want["umap"], "umap " + tag)
                assert_equal(to_np(f.vmap), want["vmap"], "vmap " + tag)
    finally:
        sgm.sgm_set_graphs(ctx, False)


def test_submit_rectify_rejects_mismatched_views(env):
    torch, sgm, ctx = env
    announce("submit_rectify validation")
    w, h, sw, sh = 64, 20, 70, 24
    p = sgm.Params(width=w, height=h, max_disp=16, census_w=5, census_h=5)
    raw = torch.zeros((sh, sw), dtype=torch.uint8, device="cuda")
    m = torch.zeros((h, w), dtype=torch.uint16, device="cuda")
    f = sgm.Frame.alloc(p, torch.empty((h, w), dtype=torch.uint8, device="cuda"),
                        torch.empty((h, w), dtype=torch.uint8, device="cuda"))
    other = torch.empty((h, w), dtype=torch.uint8, device="cuda")
    bad = [sgm.remap_job(raw, m, m, other), sgm.remap_job(raw, m, m, f.right)]
    with pytest.raises(sgm.SgmError) as e:
        sgm.sgm_submit_rectify(ctx, [f], bad)
    assert e.value.status == sgm.SGM_EINVAL and "job 0" in str(e.value)
    with pytest.raises(ValueError):
        sgm.sgm_submit_rectify(ctx, [f], bad[:1])
