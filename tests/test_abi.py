"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/sgm.h declares, and rejects bad parameters before any GPU
work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def sgm():
    from paper_1807_06271_amd import sgm as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_1807_06271_amd import build
        build.build()
    return mod


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["sgm_census", "sgm_cost", "sgm_aggregate", "sgm_disparity", "uv_maps", "sgm_submit",
              "sgm_poll", "sgm_create", "sgm_destroy", "sgm_last_error", "sgm_validate"]:
        assert n in names


def test_library_exports_every_declared_symbol(sgm):
    lib = ctypes.CDLL(sgm.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(sgm.EXPORTS)


def test_params_struct_layout_matches_header(sgm):
    # 5 int32, uint32, 2 uint16, 3 int32, 2 uint16 = 44 bytes, no hidden padding
    assert ctypes.sizeof(sgm.sgm_params) == 44
    assert sgm.sgm_params.p1.offset == 24 and sgm.sgm_params.lr_check.offset == 28
    assert sgm.sgm_params.invalid.offset == 40 and sgm.sgm_params.cost.offset == 42
    assert ctypes.sizeof(sgm.sgm_frame) == 8 * 3 + 48 + 8 * 3


def test_remap_struct_layout_matches_header(sgm):
    # 4 pointers, 2 int64 pitches, 4 int32 sizes = 64 bytes
    assert ctypes.sizeof(sgm.sgm_remap) == 64
    assert sgm.sgm_remap.src_pitch.offset == 32 and sgm.sgm_remap.src_w.offset == 48
    assert sgm.sgm_remap.h.offset == 60


def test_uv_filter_job_layout_matches_header(sgm):
    # 2 pointers, 2 int32, 4 uint16, 4 int32 = 48 bytes
    assert ctypes.sizeof(sgm.uv_filter_job) == 48
    assert sgm.uv_filter_job.threshold.offset == 24 and sgm.uv_filter_job.roi_r0.offset == 32


def test_rectify_rejects_null_context_without_a_gpu(sgm):
    assert sgm.lib().sgm_rectify(None, None, 0, None) == sgm.SGM_EINVAL
    assert sgm.lib().uv_filter(None, None, 0, None) == sgm.SGM_EINVAL


def good(sgm, **kw):
    p = sgm.Params(width=64, height=48, max_disp=64)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("field,value", [
    ("width", 0), ("height", 0), ("width", 16385), ("max_disp", 0), ("max_disp", 257),
    ("census_w", 4), ("census_h", 0), ("census_w", 11), ("path_mask", 0), ("path_mask", 0x100),
    ("p1", 130), ("p2", 9000), ("lr_check", 2), ("lr_max_diff", -1), ("median", 7), ("invalid", 10),
    ("cost", 2),
])
def test_validation_rejects(sgm, field, value):
    with pytest.raises(sgm.SgmError) as e:
        sgm.sgm_validate(good(sgm, **{field: value}))
    assert e.value.status == sgm.SGM_EINVAL


@pytest.mark.parametrize("kw", [
    {}, {"census_w": 5, "census_h": 5, "path_mask": 0x0F, "median": 0, "lr_check": 0},
    {"max_disp": 256, "invalid": 65535}, {"census_w": 65, "census_h": 1}, {"width": 1, "height": 1},
    {"max_disp": 60, "census_w": 5, "census_h": 5, "p1": 8, "p2": 32, "median": 5, "path_mask": 0x55},
    {"p1": 200, "p2": 8000, "path_mask": 0x01},
    {"cost": 1, "census_w": 5, "census_h": 5, "p1": 200, "p2": 800},   # the paper's SAD setting
])
def test_validation_accepts(sgm, kw):
    sgm.sgm_validate(good(sgm, **kw))


def test_sad_overflow_rule_uses_window_times_255(sgm):
    # 8 * (25 * 255 + p2) <= 65535  <=>  p2 <= 1816
    sgm.sgm_validate(good(sgm, cost=1, census_w=5, census_h=5, p1=200, p2=1816))
    with pytest.raises(sgm.SgmError):
        sgm.sgm_validate(good(sgm, cost=1, census_w=5, census_h=5, p1=200, p2=1817))
    with pytest.raises(sgm.SgmError):  # 17 x 17 * 255 > 65535
        sgm.sgm_validate(good(sgm, cost=1, census_w=17, census_h=17, p1=0, p2=0, path_mask=1))


def test_overflow_rule_is_paths_times_nbits_plus_p2(sgm):
    # 8 * (62 + p2) <= 65535  <=>  p2 <= 8129
    sgm.sgm_validate(good(sgm, p2=8129))
    with pytest.raises(sgm.SgmError):
        sgm.sgm_validate(good(sgm, p2=8130))
