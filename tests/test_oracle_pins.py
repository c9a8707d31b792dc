"""Pins of the CPU oracle against facts fixed by the paper's definitions and by
mathematics, independent of the oracle's own code (no GPU needed).

Each test names the passage it follows.  Golden fixtures under tests/golden/
hold hand-derived values with their derivations.
"""
import json
import os

import numpy as np
import pytest
import scipy.ndimage

import bruteforce as bf
from gen import synthetic
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DIRS = O.DIRS


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- Census (3.1.2)

def test_census_worked_example():
    g = load_golden("census_3x3.json")
    codes = O.census(np.array(g["image"], np.uint8), *g["window"])
    for key, want in g["codes_xy"].items():
        x, y = map(int, key.split(","))
        assert int(codes[y, x]) == want, key


def test_census_constant_image_is_zero():
    for cw, ch in [(5, 5), (9, 7), (3, 3)]:
        img = np.full((13, 17), 77, np.uint8)
        assert not O.census(img, cw, ch).any()


@pytest.mark.parametrize("cw,ch", [(5, 5), (9, 7), (7, 9), (3, 5)])
def test_census_one_dark_pixel_sets_one_bit_per_neighbour(cw, ch):
    # A single darker pixel q in a constant image: every p whose window holds q
    # gets exactly one set bit, at the raster position of q - p in the window
    # (first neighbour = most significant of the N_b used bits); q itself and
    # every other pixel get 0.
    H, W = 25, 29
    qy, qx = 12, 14
    img = np.full((H, W), 100, np.uint8)
    img[qy, qx] = 3
    codes = O.census(img, cw, ch)
    rx, ry = cw // 2, ch // 2
    nb = cw * ch - 1
    for y in range(H):
        for x in range(W):
            dx, dy = qx - x, qy - y
            if (dx, dy) != (0, 0) and abs(dx) <= rx and abs(dy) <= ry:
                idx = (dy + ry) * cw + (dx + rx)
                if idx > ry * cw + rx:
                    idx -= 1
                assert int(codes[y, x]) == 1 << (nb - 1 - idx), (x, y)
            else:
                assert int(codes[y, x]) == 0, (x, y)


def test_census_uses_strict_less_than_and_clamped_borders():
    # a 1-pixel-wide image: every neighbour clamps onto the column itself
    img = np.array([[5], [9], [1]], np.uint8)
    codes = O.census(img, 3, 3)
    # (0,0) centre 5: rows 0,0,1 -> values 5,5,5 / 5,5 / 9,9,9 -> 0
    assert int(codes[0, 0]) == 0
    # (0,2) centre 1: nothing below 1 -> 0
    assert int(codes[2, 0]) == 0
    # (0,1) centre 9: 5,5,5 / 9,9 / 1,1,1 -> 1,1,1,0,0,1,1,1
    assert int(codes[1, 0]) == 0b11100111


# ----------------------------------------------------------- Cost, equation (1)

def test_cost_is_popcount_of_xor_and_nbits_left_of_image():
    rng = np.random.default_rng(5)
    H, W, D, nb = 3, 11, 6, 24
    cl = rng.integers(0, 1 << nb, size=(H, W), dtype=np.uint64)
    cr = rng.integers(0, 1 << nb, size=(H, W), dtype=np.uint64)
    c = O.cost(cl, cr, D, nb)
    for y in range(H):
        for x in range(W):
            for d in range(D):
                want = bf.popcount(int(cl[y, x]) ^ int(cr[y, x - d])) if x >= d else nb
                assert int(c[y, x, d]) == want


@pytest.mark.parametrize("nb", [24, 31, 33, 48, 62, 64])
def test_cost_popcount_over_the_full_code_width(nb):
    # Equation (1) with the Hamming distance of N_b-bit codes: the 9x7 window
    # of the workloads gives 62-bit codes, so every bit position up to N_b - 1
    # must count (a popcount of the low 32 bits alone would pass 24-bit codes).
    # Codes are uniform over all N_b bits; Python's bin().count is the
    # reference.
    rng = np.random.default_rng(nb)
    H, W, D = 4, 13, 7
    raw = np.frombuffer(rng.bytes(8 * H * W * 2), np.uint64).reshape(2, H, W)
    mask = np.uint64((1 << nb) - 1) if nb < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    cl, cr = raw[0] & mask, raw[1] & mask
    # codes with every bit set, and pairs that differ only above bit 31
    cl[0, 0] = mask
    cr[0, 0] = 0
    if nb > 32:
        cl[1, 3] = np.uint64(1 << (nb - 1)) | np.uint64(5)
        cr[1, 3] = np.uint64(5)
    c = O.cost(cl, cr, D, nb)
    assert int(c[0, 0, 0]) == nb
    if nb > 32:
        assert int(c[1, 3, 0]) == 1
    hi = 0
    for y in range(H):
        for x in range(W):
            for d in range(D):
                want = bf.popcount(int(cl[y, x]) ^ int(cr[y, x - d])) if x >= d else nb
                assert int(c[y, x, d]) == want
                if x >= d:
                    hi += bf.popcount((int(cl[y, x]) ^ int(cr[y, x - d])) >> 32)
    if nb > 32:
        assert hi > 0  # the high word took part


def test_cost_constant_images():
    # identical constant images: C = 0 where the right pixel exists, else N_b
    img = np.full((6, 20), 50, np.uint8)
    cl, cr = O.census(img, 9, 7), O.census(img, 9, 7)
    c = O.cost(cl, cr, 8, 62)
    for x in range(20):
        for d in range(8):
            assert (c[:, x, d] == (0 if d <= x else 62)).all()


def test_cost_zero_at_true_shift():
    # right = left shifted by d0 along rows: C(p, d0) = 0 wherever both Census
    # windows lie inside the image and x - d0 - rx >= 0
    rng = np.random.default_rng(7)
    H, W, d0, cw, ch = 20, 64, 5, 9, 7
    left = synthetic.random_image(rng, H, W + d0)
    right = left[:, d0:]
    left = left[:, :W]
    # right(x) = left(x + d0): the match of left x is right x - d0
    c = O.cost(O.census(left, cw, ch), O.census(right, cw, ch), 8, cw * ch - 1)
    rx, ry = cw // 2, ch // 2
    sub = c[ry:H - ry, d0 + rx:W - rx, d0]
    assert not sub.any()
    # and some other disparity is not free (random texture)
    assert c[ry:H - ry, d0 + rx:W - rx, d0 + 1].mean() > 10


# ------------------------------------------- Aggregation, equation (2), 3.1.3

def test_aggregation_worked_example():
    g = load_golden("scanline_3px.json")
    c = np.array(g["cost"], np.uint16)
    assert (O.aggregate(c, O.L2R, g["p1"], g["p2"]) == np.array(g["l2r"])).all()
    assert (O.aggregate(c, O.R2L, g["p1"], g["p2"]) == np.array(g["r2l"])).all()
    s = O.aggregate(c, O.L2R | O.R2L, g["p1"], g["p2"])
    assert (s == np.array(g["aggr_l2r_r2l"])).all()


def _scanline(dirbit, n):
    """Image shape and the pixel sequence of the longest scanline of a
    direction on an n-pixel image (1 x n, n x 1 or n x n)."""
    dx, dy = DIRS[dirbit]
    if dy == 0:
        H, W = 1, n
    elif dx == 0:
        H, W = n, 1
    else:
        H, W = n, n
    x0 = 0 if dx >= 0 else W - 1
    y0 = 0 if dy >= 0 else H - 1
    return H, W, [(x0 + i * dx, y0 + i * dy) for i in range(n)]


def test_aggregation_matches_enumeration_on_tiny_scanlines():
    rng = np.random.default_rng(11)
    for trial in range(120):
        dirbit = trial % 8
        n = int(rng.integers(1, 5))
        D = int(rng.integers(1, 5))
        p1 = int(rng.integers(0, 6))
        p2 = int(rng.integers(p1, 12))
        H, W, pix = _scanline(dirbit, n)
        c = synthetic.random_cost(rng, H, W, D, 9)
        L = O.aggregate(c, 1 << dirbit, p1, p2)
        want = bf.normalised_path_costs([list(map(int, c[y, x])) for x, y in pix], p1, p2)
        got = [list(map(int, L[y, x])) for x, y in pix]
        assert got == want, (trial, dirbit, n, D, p1, p2)


@pytest.mark.parametrize("dirbit", range(8))
def test_aggregation_recurrence_bounds(dirbit):
    # C(p,d) <= L_r(p,d) <= C(p,d) + P2 (the penalised minimum lies between
    # the predecessor's minimum m and m + P2, and m is subtracted).
    rng = np.random.default_rng(100 + dirbit)
    c = synthetic.random_cost(rng, 9, 13, 7, 24)
    p1, p2 = 3, 17
    L = O.aggregate(c, 1 << dirbit, p1, p2).astype(np.int64)
    assert (L >= c).all() and (L <= c.astype(np.int64) + p2).all()
    # at the predecessor's best disparity d* the penalised minimum is exactly
    # m, so min_d (L(p,d) - C(p,d)) == 0 for every pixel with a predecessor.
    dx, dy = DIRS[dirbit]
    H, W = c.shape[:2]
    for y in range(H):
        for x in range(W):
            if 0 <= x - dx < W and 0 <= y - dy < H:
                assert (L[y, x] - c[y, x]).min() == 0


def test_aggregation_zero_penalties_is_sum_of_costs():
    rng = np.random.default_rng(3)
    c = synthetic.random_cost(rng, 7, 9, 5, 24)
    for mask in [O.L2R, 0x0F, 0xFF, O.TL2BR | O.BL2TR]:
        s = O.aggregate(c, mask, 0, 0)
        assert (s == c.astype(np.int64) * bin(mask).count("1")).all()


def test_aggregation_infinite_penalties_is_prefix_sum():
    # With P1 = P2 larger than any path's accumulated cost, no disparity change
    # is ever taken, so L(p_n, d) = sum_{i<=n} C_i(d) - min_k sum_{i<n} C_i(k).
    rng = np.random.default_rng(4)
    n, D = 6, 5
    c = synthetic.random_cost(rng, 1, n, D, 9)
    L = O.aggregate(c, O.L2R, 10000, 10000).astype(np.int64)
    pre = np.cumsum(c[0].astype(np.int64), axis=0)
    for i in range(n):
        want = pre[i] - (pre[i - 1].min() if i else 0)
        assert (L[0, i] == want).all()


def _flip(v, fx, fy, tr=False):
    if fx:
        v = v[:, ::-1]
    if fy:
        v = v[::-1]
    if tr:
        v = v.transpose(1, 0, 2)
    return np.ascontiguousarray(v)


def test_aggregation_direction_conventions_by_symmetry():
    # Mirroring the cost volume maps one direction onto another; this pins the
    # direction table and the diagonal start rules.
    rng = np.random.default_rng(9)
    c = synthetic.random_cost(rng, 8, 11, 6, 24)
    p1, p2 = 4, 15

    def agg(v, bit):
        return O.aggregate(np.ascontiguousarray(v), bit, p1, p2)

    l2r = agg(c, O.L2R)
    tl = agg(c, O.TL2BR)
    assert (agg(c, O.R2L) == _flip(agg(_flip(c, 1, 0), O.L2R), 1, 0)).all()
    assert (agg(c, O.T2B) == _flip(agg(_flip(c, 0, 0, True), O.L2R), 0, 0, True)).all()
    assert (agg(c, O.B2T) == _flip(agg(_flip(c, 0, 1), O.T2B), 0, 1)).all()
    assert (agg(c, O.BR2TL) == _flip(agg(_flip(c, 1, 1), O.TL2BR), 1, 1)).all()
    assert (agg(c, O.TR2BL) == _flip(agg(_flip(c, 1, 0), O.TL2BR), 1, 0)).all()
    assert (agg(c, O.BL2TR) == _flip(agg(_flip(c, 0, 1), O.TL2BR), 0, 1)).all()
    # the main diagonal is its own transpose
    assert (tl == _flip(agg(_flip(c, 0, 0, True), O.TL2BR), 0, 0, True)).all()
    # horizontal paths: every row is an independent scanline
    for y in range(c.shape[0]):
        assert (l2r[y] == agg(c[y:y + 1], O.L2R)[0]).all()
    # the first column starts every L2R path: L = C there
    assert (l2r[:, 0] == c[:, 0]).all()
    # diagonal start pixels (top row and left column) take the cost unchanged
    assert (tl[0] == c[0]).all() and (tl[:, 0] == c[:, 0]).all()


def test_aggregation_sum_over_paths():
    rng = np.random.default_rng(12)
    c = synthetic.random_cost(rng, 6, 7, 5, 24)
    per = [O.aggregate(c, 1 << b, 2, 9).astype(np.int64) for b in range(8)]
    assert (O.aggregate(c, 0xFF, 2, 9) == sum(per)).all()
    assert (O.aggregate(c, 0x0F, 2, 9) == sum(per[:4])).all()


def test_aggregation_reports_overflow():
    c = np.full((2, 3, 2), 60000, np.uint16)
    with pytest.raises(O.OracleError):
        O.aggregate(c, 0x03, 1, 2)


# ------------------------------------------------------------ WTA (3.1.3)

def test_wta_is_first_argmin():
    rng = np.random.default_rng(1)
    s = synthetic.random_cost(rng, 5, 9, 7, 4)  # small range: many ties
    assert (O.wta(s) == np.argmin(s, axis=-1)).all()


# ------------------------------------------- right view and LR check (3.1.4)

def test_right_disparity_and_lr_worked_example():
    g = load_golden("scanline_3px.json")
    s = np.array(g["aggr_l2r_r2l"], np.uint16)
    assert (O.wta(s) == np.array(g["wta"])).all()
    dr = O.right_disparity(s)
    assert (dr == np.array(g["right"])).all()
    assert (O.lr_check(O.wta(s), dr, 1, 255) == np.array(g["lr_maxdiff1"])).all()
    assert (O.lr_check(O.wta(s), dr, 0, 255) == np.array(g["lr_maxdiff0_invalid255"])).all()


def test_right_disparity_is_argmin_of_resampled_volume():
    # D_R(x) = argmin_d S(x + d, d): build the right-view volume by re-indexing
    # with NumPy and take numpy.argmin (first occurrence), with cells whose
    # left pixel falls outside the image set to +inf.
    rng = np.random.default_rng(2)
    for H, W, D in [(3, 10, 4), (2, 5, 8), (4, 17, 6)]:
        s = synthetic.random_cost(rng, H, W, D, 5)
        big = np.full((H, W, D), np.iinfo(np.int64).max, np.int64)
        for d in range(D):
            if d < W:
                big[:, : W - d, d] = s[:, d:, d]
        assert (O.right_disparity(s) == np.argmin(big, axis=-1)).all()
        assert (O.right_disparity(s).astype(np.int64) == np.array(bf.right_disparity_loop(s.tolist()))).all()


def test_lr_check_hand_built_cases():
    inv = 255
    # row of 6 pixels
    dl = np.array([[0, 2, 3, 1, 4, 2]], np.uint16)
    dr = np.array([[0, 1, 4, 0, 3, 3]], np.uint16)
    out = O.lr_check(dl, dr, 1, inv)
    # x=0: dl 0 -> xr 0, dr 0: keep.          x=1: dl 2 -> xr -1 < 0: invalid
    # x=2: dl 3 -> xr -1: invalid.            x=3: dl 1 -> xr 2, dr 4, diff 3: invalid
    # x=4: dl 4 -> xr 0, dr 0, diff 4: invalid x=5: dl 2 -> xr 3, dr 0, diff 2: invalid
    assert out.tolist() == [[0, inv, inv, inv, inv, inv]]
    dl = np.array([[0, 1, 1, 2, 3, 3]], np.uint16)
    dr = np.array([[1, 0, 2, 2, 1, 5]], np.uint16)
    # x=1: xr 0 dr 1 diff 0 keep; x=2: xr 1 dr 0 diff 1 keep (off by one kept);
    # x=3: xr 1 dr 0 diff 2 invalid (off by two); x=4: xr 1 dr 0 diff 3 invalid;
    # x=5: xr 2 dr 2 diff 1 keep
    assert O.lr_check(dl, dr, 1, inv).tolist() == [[0, 1, 1, inv, inv, 3]]
    assert O.lr_check(dl, dr, 0, inv).tolist() == [[inv, 1, inv, inv, inv, inv]]
    # x - D_L < 0 is invalid even when D_R at the clamped column would agree:
    # x=0: dl 0, D_R(0) = 1, diff 1: keep; x=1: dl 2 -> xr -1 (D_R(0) = 1
    # would be within 1 of 2).
    assert O.lr_check(np.array([[0, 2]], np.uint16), np.array([[1, 0]], np.uint16), 1, inv).tolist() \
        == [[0, inv]]


def test_selection_chain_worked_example():
    # WTA -> right-view disparity -> LR check -> 3x3 median -> U/V maps, in
    # the order of sections 3.1.3 to 3.2, on a hand-worked 3 x 5 volume in
    # which the check invalidates pixels, and where a median of D_L or U/V of
    # the pre-median map would give other values (see the fixture).
    g = load_golden("chain_3x5.json")
    H, W, D = g["height"], g["width"], g["max_disp"]
    s = np.full((H, W, D), 10, np.uint16)
    for y in range(H):
        for x in range(W):
            s[y, x, g["disp_l_defining_s"][y][x]] = 0
    out = O.select(s, D, True, g["lr_max_diff"], g["median"], g["invalid"])
    assert out["disp_l"].tolist() == g["disp_l_defining_s"]
    assert out["disp_r"].tolist() == g["disp_r"]
    assert out["disp_lr"].tolist() == g["disp_lr"]
    assert out["disp"].tolist() == g["disp"]
    assert out["umap"].tolist() == g["umap"]
    assert out["vmap"].tolist() == g["vmap"]


def test_whole_path_stages_chain_in_the_paper_order():
    # Every stage of the whole path consumes the previous stage's output
    # (sections 3.1.2 to 3.2), checked with library routines: the WTA map is
    # numpy.argmin of S, the final map is scipy's 3x3 median of the
    # LR-checked map, and U/V are numpy.bincount of the final map.  The input
    # is chosen so that each wrong order would show: the check invalidates
    # pixels, the median changes pixels, and the median of D_L differs from
    # the median of the checked map.
    left, right, _ = synthetic.make_pair("kitti", 31, 96, 40, 32)
    out = O.sgm(left, right, 32, 9, 7, 0xFF, 10, 120, True, 1, 3)
    dl, dlr, disp = out["disp_l"], out["disp_lr"], out["disp"]
    assert (dl == np.argmin(out["aggr"], axis=-1)).all()
    big = np.full(out["aggr"].shape, np.iinfo(np.int64).max, np.int64)
    for d in range(32):
        big[:, : 96 - d, d] = out["aggr"][:, d:, d]
    assert (out["disp_r"] == np.argmin(big, axis=-1)).all()
    assert (disp == scipy.ndimage.median_filter(dlr, size=3, mode="nearest")).all()
    for x in range(96):
        col = disp[:, x]
        assert (out["umap"][:, x] == np.bincount(col[col < 32], minlength=32)).all()
    for y in range(40):
        row = disp[y]
        assert (out["vmap"][y] == np.bincount(row[row < 32], minlength=32)).all()
    # kept pixels keep D_L; invalidated ones carry the invalid value
    assert ((dlr == dl) | (dlr == 255)).all()
    assert (dlr == 255).sum() > 20
    assert (disp != dlr).sum() > 20
    assert (scipy.ndimage.median_filter(dl, size=3, mode="nearest") != disp).any()


# ------------------------------------------------------------ median (3.1.5)

@pytest.mark.parametrize("k", [3, 5])
def test_median_matches_scipy(k):
    rng = np.random.default_rng(k)
    for H, W in [(1, 1), (1, 7), (6, 1), (9, 13), (16, 31)]:
        img = rng.integers(0, 6, size=(H, W)).astype(np.uint16)
        img[rng.random((H, W)) < 0.1] = 255
        want = scipy.ndimage.median_filter(img, size=k, mode="nearest")
        assert (O.median(img, k) == want).all()


# -------------------------------------------------------------- U/V maps (3.2)

def test_uv_maps_are_histograms():
    rng = np.random.default_rng(6)
    H, W, D = 17, 23, 9
    disp = rng.integers(0, D, size=(H, W)).astype(np.uint16)
    disp[rng.random((H, W)) < 0.2] = 255
    u, v = O.uv_maps(disp, D)
    assert u.shape == (D, W) and v.shape == (H, D)
    for x in range(W):
        col = disp[:, x]
        assert (u[:, x] == np.bincount(col[col < D], minlength=D)).all()
    for y in range(H):
        row = disp[y]
        assert (v[y] == np.bincount(row[row < D], minlength=D)).all()
    valid = int((disp < D).sum())
    assert int(u.sum()) == valid == int(v.sum())


# ----------------------------------------------------------------- end to end

def test_constant_images_give_zero_disparity_everywhere():
    img = np.full((20, 30), 128, np.uint8)
    out = O.sgm(img, img, 16, 5, 5, 0xFF, 10, 120, True, 1, 3)
    assert not out["disp_l"].any() and not out["disp"].any()
    assert (out["umap"][0] == 20).all() and not out["umap"][1:].any()
    assert (out["vmap"][:, 0] == 30).all() and not out["vmap"][:, 1:].any()


@pytest.mark.parametrize("d0", [0, 3, 9])
def test_fronto_parallel_shift_is_recovered(d0):
    rng = np.random.default_rng(20 + d0)
    H, W, D = 40, 96, 16
    base = np.rint(synthetic.fractal_texture(rng, H, W + d0)).clip(0, 255).astype(np.uint8)
    left, right = base[:, :W], base[:, d0:W + d0]
    out = O.sgm(left, right, D, 9, 7, 0xFF, 10, 120, True, 1, 3)
    inner = out["disp_l"][4:-4, D + 5:-5]
    assert (inner == d0).mean() >= 0.99


def test_synthetic_scene_sanity_statistics():
    # the paper's accuracy measures (density; share of pixels within 3 px of
    # the ground truth) on a seeded synthetic scene, as a sanity statistic
    left, right, gt = synthetic.make_pair("small", 1000)
    out = O.sgm(left, right, 64, 5, 5, 0x0F, 10, 120, True, 1, 3)
    disp = out["disp"].astype(np.int64)
    valid = disp < 64
    density = valid.mean()
    has_gt = gt >= 0
    both = valid & has_gt
    correct = (np.abs(disp[both] - gt[both]) < 3).mean()
    assert density > 0.6 and correct > 0.8, (density, correct)


# ------------------------------------------------------- SAD cost (3.1.2)

def test_sad_worked_example():
    g = load_golden("sad_1x4.json")
    c = O.sad_cost(np.array(g["left"], np.uint8), np.array(g["right"], np.uint8), *g["window"], g["max_disp"])
    assert c.tolist() == g["cost"]


def test_sad_matches_brute_force_loops():
    rng = np.random.default_rng(31)
    for (H, W, D, ww, wh) in [(3, 7, 4, 3, 3), (5, 6, 8, 5, 5), (4, 9, 3, 1, 3)]:
        L = synthetic.random_image(rng, H, W)
        R = synthetic.random_image(rng, H, W)
        c = O.sad_cost(L, R, ww, wh, D)
        rx, ry = ww // 2, wh // 2
        for y in range(H):
            for x in range(W):
                for d in range(D):
                    if x < d:
                        want = ww * wh * 255
                    else:
                        want = 0
                        for dy in range(-ry, ry + 1):
                            for dx in range(-rx, rx + 1):
                                yy = min(max(y + dy, 0), H - 1)
                                a = int(L[yy, min(max(x + dx, 0), W - 1)])
                                b = int(R[yy, min(max(x - d + dx, 0), W - 1)])
                                want += abs(a - b)
                    assert int(c[y, x, d]) == want


def test_sad_zero_at_true_shift_and_on_constant_images():
    rng = np.random.default_rng(8)
    H, W, d0 = 12, 40, 4
    base = synthetic.random_image(rng, H, W + d0)
    left, right = base[:, :W], base[:, d0:W + d0]
    c = O.sad_cost(left, right, 5, 5, 8)
    assert not c[:, d0 + 2:W - 2, d0].any()
    flat = np.full((6, 10), 9, np.uint8)
    c = O.sad_cost(flat, flat, 5, 5, 4)
    for x in range(10):
        for d in range(4):
            assert (c[:, x, d] == (0 if d <= x else 25 * 255)).all()


def test_sad_pipeline_on_fronto_parallel_shift():
    # the paper's SAD setting (5x5, P1 = 200, P2 = 800) recovers a plain shift
    rng = np.random.default_rng(21)
    H, W, D, d0 = 40, 96, 16, 6
    base = np.rint(synthetic.fractal_texture(rng, H, W + d0)).clip(0, 255).astype(np.uint8)
    out = O.sgm(base[:, :W], base[:, d0:W + d0], D, 5, 5, 0x55, 200, 800, True, 1, 5, cost_kind=1)
    assert (out["disp_l"][4:-4, D + 4:-4] == d0).mean() >= 0.99


# --------------------------------------------------- rectification (3.1.1)

def test_rectify_identity_flip_and_out_of_range():
    rng = np.random.default_rng(40)
    src = synthetic.random_image(rng, 7, 11)
    ys, xs = np.mgrid[0:7, 0:11]
    assert (O.rectify(src, xs.astype(np.uint16), ys.astype(np.uint16)) == src).all()
    flip = O.rectify(src, (10 - xs).astype(np.uint16), ys.astype(np.uint16))
    assert (flip == src[:, ::-1]).all()
    mx = xs.astype(np.uint16).copy()
    mx[2, 3] = 11      # one column beyond the raw image
    my = ys.astype(np.uint16).copy()
    my[4, 5] = 65535   # "no source pixel"
    out = O.rectify(src, mx, my)
    assert out[2, 3] == 0 and out[4, 5] == 0
    mask = np.ones_like(src, bool)
    mask[2, 3] = mask[4, 5] = False
    assert (out[mask] == src[mask]).all()


def test_rectify_is_a_gather():
    # against NumPy fancy indexing on a raw image of another size
    rng = np.random.default_rng(41)
    src = synthetic.random_image(rng, 40, 50)
    mx, my = synthetic.rectification_maps(33, 21, 50, 40, seed=3)
    want = np.zeros((21, 33), np.uint8)
    ok = (mx < 50) & (my < 40)
    want[ok] = src[my[ok].astype(int), mx[ok].astype(int)]
    assert (O.rectify(src, mx, my) == want).all()
    assert ok.mean() > 0.8


# ------------------------------------------- U/V map filtering (section 3.2)

def test_uv_filter_threshold_is_inclusive():
    m = np.array([[0, 4, 5, 6], [65535, 5, 1, 0]], np.uint16)
    assert O.uv_filter(m, 5, 0, 0).tolist() == [[0, 0, 255, 255], [255, 255, 0, 0]]


def test_uv_filter_dilation_matches_scipy():
    from scipy import ndimage
    rng = np.random.default_rng(50)
    m = rng.integers(0, 40, size=(23, 31)).astype(np.uint16)
    b = m >= 36
    for r in range(4):
        want = ndimage.binary_dilation(b, structure=np.ones((2 * r + 1, 2 * r + 1), bool), border_value=0)
        assert (O.uv_filter(m, 36, r, 0) == want.astype(np.uint8) * 255).all(), r


def test_uv_filter_gaussian_matches_scipy():
    # binomial weights from scipy.special.comb, replicated borders from
    # ndimage's "nearest" mode, exact float64 sums, rounding half up
    from scipy import ndimage, special
    rng = np.random.default_rng(51)
    m = rng.integers(0, 10, size=(19, 26)).astype(np.uint16)
    b = (m >= 7).astype(np.float64) * 255
    for g in range(1, 4):
        w = special.comb(2 * g, np.arange(2 * g + 1), exact=False)
        s = ndimage.correlate(b, np.outer(w, w), mode="nearest")
        want = np.floor((s + 2.0 ** (4 * g - 1)) / 2.0 ** (4 * g)).astype(np.uint8)
        assert (O.uv_filter(m, 7, 0, g) == want).all(), g


def test_uv_filter_impulse_response_is_the_binomial_outer_product():
    import math
    m = np.zeros((11, 13), np.uint16)
    m[5, 6] = 9
    out = O.uv_filter(m, 1, 0, 2)
    want = np.zeros((11, 13), np.uint8)
    for i in range(-2, 3):
        for j in range(-2, 3):
            want[5 + i, 6 + j] = (255 * math.comb(4, 2 + i) * math.comb(4, 2 + j) + 128) // 256
    assert (out == want).all()
    assert out[5, 6] == 36 and out[5, 4] == 6 and out[3, 4] == 1   # 255*36/256, 255*6/256, 255/256


def test_uv_filter_dilation_then_blur_and_region_of_interest():
    m = np.zeros((9, 9), np.uint16)
    m[4, 4] = 3
    # dilation by 1 makes a 3x3 block; a [1,2,1] blur of it has a flat 255 centre
    out = O.uv_filter(m, 3, 1, 1)
    assert out[4, 4] == 255 and out[3, 3] == (255 * (4 + 2 + 2 + 1) + 8) // 16
    assert out[0, 0] == 0 and out[4, 1] == 0
    full = O.uv_filter(np.full((6, 8), 10, np.uint16), 5, 2, 3)
    assert (full == 255).all()
    roi = O.uv_filter(np.full((6, 8), 10, np.uint16), 5, 2, 3, roi=(1, 3, 2, 5))
    want = np.zeros((6, 8), np.uint8)
    want[1:3, 2:5] = 255
    assert (roi == want).all()
