"""Graph mode of sgm_submit (GPU required): batches captured into HIP graphs
and replayed from the cache give the same outputs as direct launches, on
every replay, with unrelated eager GPU work and synchronisations between
replays."""
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


def batch(sgm, torch, seed):
    specs = [(320, 240, 64, dict(census_w=5, census_h=5, path_mask=0x0F, lr_check=0, median=0)),
             (257, 61, 128, dict()),
             (131, 47, 60, dict(census_w=5, census_h=5, path_mask=0x55, p1=8, p2=32, median=5))]
    out = []
    for i, (W, H, D, kw) in enumerate(specs):
        left, right, _ = synthetic.make_pair("kitti", seed + i, W, H, D)
        p = sgm.Params(width=W, height=H, max_disp=D, **kw)
        out.append((p, left, right, sgm.Frame.alloc(p, to_dev(torch, left), to_dev(torch, right))))
    return out


def test_graph_replays_match_direct_launches_and_oracle(env):
    torch, sgm, ctx = env
    announce("graphs")
    sgm.sgm_set_graphs(ctx, False)
    ref = batch(sgm, torch, 500)
    sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f for *_, f in ref]))
    want = [to_np(f.disp) for *_, f in ref]
    for (p, left, right, f), w in zip(ref, want):
        o = O.sgm(left, right, p.max_disp, p.census_w, p.census_h, p.path_mask, p.p1, p.p2,
                  bool(p.lr_check), p.lr_max_diff, p.median, p.inv())
        assert_equal(w, o["disp"], "direct vs oracle")
    sgm.sgm_set_graphs(ctx, True)
    h0, m0 = sgm.sgm_graph_stats(ctx)
    scratch = torch.zeros(1 << 20, device="cuda")
    for rep in range(4):
        # fresh output buffers each time: the cached graph must be updated
        frames = [sgm.Frame.alloc(p, f.left, f.right) for p, _, _, f in ref]
        t = sgm.sgm_submit(ctx, frames)
        scratch.add_(1.0)          # unrelated eager work between replays
        sgm.sgm_wait(ctx, t)
        torch.cuda.synchronize()
        for f, w in zip(frames, want):
            assert_equal(to_np(f.disp), w, "graph replay %d" % rep)
        ref_u = [to_np(f.umap) for *_, f in ref]
        for f, u in zip(frames, ref_u):
            assert_equal(to_np(f.umap), u, "graph replay %d umap" % rep)
    h1, m1 = sgm.sgm_graph_stats(ctx)
    assert m1 - m0 == 1 and h1 - h0 == 3
    assert float(scratch[0]) == 4.0
    sgm.sgm_set_graphs(ctx, False)


def test_graph_cache_keeps_census_and_sad_batches_apart(env):
    # two batches identical in every parameter but the cost kind: they launch
    # different kernels, so each must get its own cached graph, and replays
    # in turn must keep matching the oracle
    torch, sgm, ctx = env
    announce("graphs: Census and SAD batches of one shape")
    W, H, D = 192, 64, 64
    items = {}
    for kind, seed in ((sgm.COST_CENSUS, 610), (sgm.COST_SAD, 611)):
        left, right, _ = synthetic.make_pair("kitti", seed, W, H, D)
        p = sgm.Params(width=W, height=H, max_disp=D, census_w=5, census_h=5, path_mask=sgm.PATHS_PAPER4,
                       p1=200, p2=800, lr_check=1, median=5, cost=kind)
        o = O.sgm(left, right, D, 5, 5, p.path_mask, 200, 800, True, 1, 5, cost_kind=kind)
        items[kind] = (p, to_dev(torch, left), to_dev(torch, right), o)
    sgm.sgm_set_graphs(ctx, True)
    try:
        h0, m0 = sgm.sgm_graph_stats(ctx)
        for rep in range(3):
            for kind in (sgm.COST_CENSUS, sgm.COST_SAD):
                p, L, R, o = items[kind]
                f = sgm.Frame.alloc(p, L, R)
                sgm.sgm_wait(ctx, sgm.sgm_submit(ctx, [f]))
                torch.cuda.synchronize()
                tag = "replay %d cost %d" % (rep, kind)
                assert_equal(to_np(f.disp), o["disp"], "disp " + tag)
                assert_equal(to_np(f.umap), o["umap"], "umap " + tag)
                assert_equal(to_np(f.vmap), o["vmap"], "vmap " + tag)
        h1, m1 = sgm.sgm_graph_stats(ctx)
        assert m1 - m0 == 2 and h1 - h0 == 4
    finally:
        sgm.sgm_set_graphs(ctx, False)
