"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message and exit status 2 (this library has no multi-GPU path)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_aggregation_bytes_follow_the_schedule():
    # 8 directions reading the cost volume: 2 bytes per evaluation; with the
    # horizontal pair on Census windows those two write their byte and read
    # one 16-byte code record per pixel instead of D cost bytes
    sys.path.insert(0, ROOT)
    import bench
    from paper_1807_06271_amd.sgm import Params
    p = Params(width=1920, height=1080, max_disp=256)
    cells = 1920 * 1080 * 256
    vol = {"h_lanes": 64, "h_costs": "volume"}
    codes = {"h_lanes": 64, "h_costs": "codes"}
    assert bench.agg_alg_bytes(p, 8, vol) == 8 * 8 * 2 * cells == 2 * 8 * p.disp_evals()
    assert bench.agg_alg_bytes(p, 8, codes) == 8 * (6 * 2 * cells + 2 * (cells + 16 * 1920 * 1080))
    assert bench.agg_kernel_name(codes).endswith("unsigned char, 8, false, 2>")
    assert bench.agg_kernel_name({"h_lanes": 32, "h_costs": "volume"}) == \
        "agg_kernel<16, 8, 32, 0, unsigned char, 8, false, 0>"


def test_roofline_kernel_follows_the_two_pass_schedule():
    # on the two-pass schedule the longest kernel is the per-direction launch
    # of L->R, R->L, TR->BL and BL->TR: the diagonals read their costs and
    # write their path costs (2 B per cell), the horizontal ones write theirs
    # and read one 16-byte code record per pixel (or the costs); its grid is
    # the library's: one wave per scanline of 64 lanes horizontally, per four
    # 16-lane diagonal scanlines, four waves per 256-thread block
    sys.path.insert(0, ROOT)
    import bench
    from paper_1807_06271_amd.sgm import Params
    p = Params(width=1920, height=1080, max_disp=256)
    cells = 1920 * 1080 * 256
    name, stage, alg, evals, _, grid = bench.dominant_kernel(p, 8, {"h_lanes": 64, "h_costs": "codes",
                                                                    "two_pass": "wide"})
    assert name == "agg_kernel<16, 4, 64, 0, unsigned char, 8, false, 2>" and stage == "aggregate"
    assert alg == 8 * (2 * 2 * cells + 2 * (cells + 16 * 1920 * 1080)) and evals == 8 * 4 * cells
    assert grid == 1873920  # 8 x (2 x 1080 + 2 x 750) waves in blocks of 4
    name, stage, alg, evals, _, grid = bench.dominant_kernel(p, 8, {"h_lanes": 64, "h_costs": "volume",
                                                                    "two_pass": "off"})
    assert stage == "aggregate" and alg == 2 * evals == 2 * 8 * p.disp_evals()
    assert grid == 3133440  # 8 x (2 x 1080 + 2 x 480 + 4 x 750) waves in blocks of 4