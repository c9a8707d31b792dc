"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is a copy of the oracle's C source with one plausible mistake (a
wrong comparison, a dropped term, a swapped index or direction, a wrong tie
rule).  It is compiled on the CPU, loaded in place of the real oracle, and the
pin tests of test_oracle_pins are run against it: at least one must fail.
"""
import os
import subprocess

import pytest

import test_oracle_pins as pins
from oracle import oracle as O

MUTANTS = [
    ("census <= instead of <", "(uint64_t)(v < centre ? 1 : 0)", "(uint64_t)(v <= centre ? 1 : 0)"),
    ("census > instead of <", "(uint64_t)(v < centre ? 1 : 0)", "(uint64_t)(v > centre ? 1 : 0)"),
    ("census column-major order",
     "for (int dy = -ry; dy <= ry; ++dy) {\n                for (int dx = -rx; dx <= rx; ++dx) {",
     "for (int dx = -rx; dx <= rx; ++dx) {\n                for (int dy = -ry; dy <= ry; ++dy) {"),
    ("cost: valid range off by one", "if (x - d >= 0)\n", "if (x - d > 0)\n"),
    ("cost: zero instead of N_b left of image", "c = nbits;", "c = 0;"),
    ("P2 used for one-step change", "lp[d - 1] + p1 < best) best = lp[d - 1] + p1",
     "lp[d - 1] + p2 < best) best = lp[d - 1] + p2"),
    ("predecessor minimum not subtracted", "l[d] = (int32_t)c[d] + best - m;", "l[d] = (int32_t)c[d] + best;"),
    ("P1 instead of P2 for large jumps", "if (m + p2 < best) best = m + p2;", "if (m + p1 < best) best = m + p1;"),
    ("d+1 neighbour dropped", "if (d + 1 < d_max && lp[d + 1] + p1 < best)", "if (0 && lp[d + 1] + p1 < best)"),
    ("predecessor on the wrong side", "int px_ = (x) - dx, py_ = (y) - dy;", "int px_ = (x) + dx, py_ = (y) - dy;"),
    ("path start not equal to cost", "for (int d = 0; d < d_max; ++d) l[d] = c[d];",
     "for (int d = 0; d < d_max; ++d) l[d] = 0;"),
    ("diagonal direction table swapped", "{+1, -1, 0, 0, +1, -1, -1, +1}", "{+1, -1, 0, 0, +1, -1, +1, -1}"),
    ("WTA picks the last tie", "if (s[d] < s[best]) best = d;", "if (s[d] <= s[best]) best = d;"),
    ("right disparity picks the last tie", "if (v < bestv) { bestv = v; best = d; }",
     "if (v <= bestv) { bestv = v; best = d; }"),
    ("LR strict difference", "if (diff <= max_diff) v = (uint16_t)dl;", "if (diff < max_diff) v = (uint16_t)dl;"),
    ("LR accepts left-of-image", "if (xr >= 0) {", "if (xr >= 0 || 1) { if (xr < 0) xr = 0;"),
    ("median picks the wrong rank", "out[(int64_t)y * w + x] = win[n / 2];",
     "out[(int64_t)y * w + x] = win[n / 2 + (n > 1)];"),
    ("V-map skips d = 0", "v[(int64_t)y * d_max + d] += 1;", "v[(int64_t)y * d_max + d] += (d > 0);"),
    ("popcount of the low 32 bits only", "while (v) { v &= v - 1; ++n; }",
     "v &= 0xFFFFFFFFu; while (v) { v &= v - 1; ++n; }"),
]

PIN_CALLS = [
    (pins.test_census_worked_example, {}),
    (pins.test_census_constant_image_is_zero, {}),
    (pins.test_census_one_dark_pixel_sets_one_bit_per_neighbour, {"cw": 5, "ch": 5}),
    (pins.test_census_uses_strict_less_than_and_clamped_borders, {}),
    (pins.test_cost_is_popcount_of_xor_and_nbits_left_of_image, {}),
    (pins.test_cost_popcount_over_the_full_code_width, {"nb": 62}),
    (pins.test_cost_constant_images, {}),
    (pins.test_cost_zero_at_true_shift, {}),
    (pins.test_aggregation_worked_example, {}),
    (pins.test_aggregation_matches_enumeration_on_tiny_scanlines, {}),
    (pins.test_aggregation_zero_penalties_is_sum_of_costs, {}),
    (pins.test_aggregation_infinite_penalties_is_prefix_sum, {}),
    (pins.test_aggregation_direction_conventions_by_symmetry, {}),
    (pins.test_wta_is_first_argmin, {}),
    (pins.test_right_disparity_and_lr_worked_example, {}),
    (pins.test_right_disparity_is_argmin_of_resampled_volume, {}),
    (pins.test_lr_check_hand_built_cases, {}),
    (pins.test_median_matches_scipy, {"k": 3}),
    (pins.test_uv_maps_are_histograms, {}),
    (pins.test_selection_chain_worked_example, {}),
    (pins.test_whole_path_stages_chain_in_the_paper_order, {}),
    (pins.test_constant_images_give_zero_disparity_everywhere, {}),
]


@pytest.fixture(scope="module")
def restore_oracle():
    yield
    O.load()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, restore_oracle, name, old, new):
    src = open(O.SRC).read()
    assert src.count(old) >= 1, "mutation site not found: " + name
    mutated = src.replace(old, new)
    c_path = tmp_path / "mutant.c"
    so_path = tmp_path / "libmutant.so"
    c_path.write_text(mutated)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-o", str(so_path), str(c_path)])
    O.load(str(so_path))
    caught = []
    try:
        for fn, kw in PIN_CALLS:
            try:
                fn(**kw)
            except (AssertionError, O.OracleError):
                caught.append(fn.__name__)
    finally:
        O.load()
    assert caught, "no pin caught the planted mistake: " + name


SAD_MUTANTS = [
    ("SAD clamps the right view with the left coordinate",
     "int b = right[(int64_t)yy * pitch + clampi(x - d + dx, 0, w - 1)];",
     "int b = right[(int64_t)yy * pitch + clampi(x + dx, 0, w - 1) - d * (x + dx >= d)];"),
    ("SAD zero left of the image", "c = ww * wh * 255;", "c = 0;"),
    ("SAD signed difference", "c += a > b ? a - b : b - a;", "c += a - b;"),
]


@pytest.mark.parametrize("name,old,new", SAD_MUTANTS, ids=[m[0] for m in SAD_MUTANTS])
def test_sad_pins_catch_planted_mistake(tmp_path, restore_oracle, name, old, new):
    src = open(O.SRC).read()
    assert src.count(old) == 1, name
    c_path = tmp_path / "mutant.c"
    so_path = tmp_path / "libmutant.so"
    c_path.write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-o", str(so_path), str(c_path)])
    O.load(str(so_path))
    caught = []
    try:
        for fn in (pins.test_sad_worked_example, pins.test_sad_matches_brute_force_loops,
                   pins.test_sad_zero_at_true_shift_and_on_constant_images):
            try:
                fn()
            except (AssertionError, O.OracleError):
                caught.append(fn.__name__)
    finally:
        O.load()
    assert caught, "no pin caught: " + name


RECTIFY_MUTANTS = [
    ("rectify swaps the two maps", "int sx = map_x[(int64_t)y * w + x], sy = map_y[(int64_t)y * w + x];",
     "int sx = map_y[(int64_t)y * w + x], sy = map_x[(int64_t)y * w + x];"),
    ("rectify reads one column beyond the image", "(sx < src_w && sy < src_h)", "(sx <= src_w && sy < src_h)"),
    ("rectify fills with the first pixel", "+ sx] : 0;", "+ sx] : src[0];"),
]


@pytest.mark.parametrize("name,old,new", RECTIFY_MUTANTS, ids=[m[0] for m in RECTIFY_MUTANTS])
def test_rectify_pins_catch_planted_mistake(tmp_path, restore_oracle, name, old, new):
    src = open(O.SRC).read()
    assert src.count(old) == 1, name
    c_path = tmp_path / "mutant.c"
    so_path = tmp_path / "libmutant.so"
    c_path.write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-o", str(so_path), str(c_path)])
    O.load(str(so_path))
    caught = []
    try:
        for fn in (pins.test_rectify_identity_flip_and_out_of_range, pins.test_rectify_is_a_gather):
            try:
                fn()
            except (AssertionError, O.OracleError):
                caught.append(fn.__name__)
    finally:
        O.load()
    assert caught, "no pin caught: " + name


UV_FILTER_MUTANTS = [
    ("threshold strict", "b[i] = map[i] >= thr ? 255 : 0;", "b[i] = map[i] > thr ? 255 : 0;"),
    ("dilation one short on one side", "for (int dy = -dil_r; dy <= dil_r; ++dy)", "for (int dy = -dil_r; dy < dil_r; ++dy)"),
    ("blur truncates", "(acc + ((int64_t)1 << (shift - 1))) >> shift", "acc >> shift"),
    ("blur box weights", "binom(2 * blur_r, blur_r + i) * binom(2 * blur_r, blur_r + j)",
     "binom(2 * blur_r, blur_r) * binom(2 * blur_r, blur_r)"),
    ("blur border wraps to zero", "int yy = clampi(y + i, 0, rows - 1), xx = clampi(x + j, 0, cols - 1);",
     "int yy = clampi(y + i, 0, rows - 1), xx = clampi(x + j, 0, cols - 1);\n"
     "                    if (y + i < 0 || y + i >= rows) continue;"),
    ("ROI end inclusive", "y < roi_r1 && x >= roi_c0", "y <= roi_r1 && x >= roi_c0"),
]


@pytest.mark.parametrize("name,old,new", UV_FILTER_MUTANTS, ids=[m[0] for m in UV_FILTER_MUTANTS])
def test_uv_filter_pins_catch_planted_mistake(tmp_path, restore_oracle, name, old, new):
    src = open(O.SRC).read()
    assert src.count(old) == 1, name
    c_path = tmp_path / "mutant.c"
    so_path = tmp_path / "libmutant.so"
    c_path.write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-o", str(so_path), str(c_path)])
    O.load(str(so_path))
    caught = []
    try:
        for fn in (pins.test_uv_filter_threshold_is_inclusive, pins.test_uv_filter_dilation_matches_scipy,
                   pins.test_uv_filter_gaussian_matches_scipy,
                   pins.test_uv_filter_impulse_response_is_the_binomial_outer_product,
                   pins.test_uv_filter_dilation_then_blur_and_region_of_interest):
            try:
                fn()
            except (AssertionError, O.OracleError):
                caught.append(fn.__name__)
    finally:
        O.load()
    assert caught, "no pin caught: " + name


# Mistakes in the composition of the whole path (oracle.py): the order of
# the stages after aggregation (sections 3.1.3 to 3.2) and what each stage
# consumes.  The mutated module is loaded under another name and put in place
# of the oracle module that the pins call; it shares the C library.
PY_MUTANTS = [
    ("median of D_L instead of the checked map", "disp = median(dlr, median_k) if median_k else dlr",
     "disp = median(dl, median_k) if median_k else dlr"),
    ("U/V maps of the map before the median", "u, v = uv_maps(disp, d_max)", "u, v = uv_maps(dlr, d_max)"),
    ("U/V maps of D_L", "u, v = uv_maps(disp, d_max)", "u, v = uv_maps(dl, d_max)"),
    ("LR check skipped", "dlr = lr_check(dl, dr, lr_max_diff, invalid)", "dlr = dl"),
    ("WTA of the cost volume instead of S", "out.update(select(s, d_max,", "out.update(select(c, d_max,"),
    ("right-view disparity from the cost volume", "dr = right_disparity(s)", "dr = right_disparity(s[:, :, ::-1])"),
]

PY_PIN_CALLS = [
    pins.test_selection_chain_worked_example,
    pins.test_whole_path_stages_chain_in_the_paper_order,
    pins.test_constant_images_give_zero_disparity_everywhere,
    pins.test_fronto_parallel_shift_is_recovered,
    pins.test_synthetic_scene_sanity_statistics,
]


@pytest.mark.parametrize("name,old,new", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_pins_catch_planted_composition_mistake(name, old, new, monkeypatch):
    import importlib.util
    import sys
    path = os.path.join(os.path.dirname(O.SRC), "oracle.py")
    src = open(path).read()
    assert src.count(old) == 1, "mutation site not found: " + name
    spec = importlib.util.spec_from_loader("oracle_mutant", loader=None)
    mod = importlib.util.module_from_spec(spec)
    mod.__file__ = path
    sys.modules["oracle_mutant"] = mod
    try:
        exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
        mod._lib, mod._lib_path = O.lib(), O._lib_path
        monkeypatch.setattr(pins, "O", mod)
        caught = []
        for fn in PY_PIN_CALLS:
            kw = {"d0": 3} if fn is pins.test_fronto_parallel_shift_is_recovered else {}
            try:
                fn(**kw)
            except (AssertionError, mod.OracleError):
                caught.append(fn.__name__)
    finally:
        del sys.modules["oracle_mutant"]
    assert caught, "no pin caught the planted mistake: " + name
