"""NumPy front end of the plain C oracle (``sgm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  It builds
``liboracle_sgm.so`` with gcc on first use (or via :func:`build`) and wraps
each definition of the semi-global-matching path of Ruf et al. (arXiv
1807.06271, section 3.1 and 3.2) as a function on NumPy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sgm_oracle.c")
LIB = os.path.join(HERE, "liboracle_sgm.so")

# path mask bits, in the order of the oracle's direction table
L2R, R2L, T2B, B2T, TL2BR, BR2TL, TR2BL, BL2TR = (1 << i for i in range(8))
ALL8 = 0xFF
# r = (dx, dy) per bit
DIRS = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (-1, 1), (1, -1)]

_lib = None
_lib_path = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (OpenMP across scanlines)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                               "-Wall", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def load(path: str | None = None):
    """Load (and return) the oracle library; ``path`` selects another build of
    the same source, e.g. a deliberately mutated copy in a test."""
    global _lib, _lib_path
    if path is None:
        path = build()
    L = ctypes.CDLL(path)
    _declare(L)
    _lib, _lib_path = L, path
    return L


def lib():
    return _lib if _lib is not None else load()


def _declare(L):
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u16p = ctypes.POINTER(ctypes.c_uint16)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i = ctypes.c_int
    L.oracle_census.argtypes = [u8p, i, i, ctypes.c_int64, i, i, u64p]
    L.oracle_cost.argtypes = [u64p, u64p, i, i, i, i, u16p]
    L.oracle_rectify.argtypes = [u8p, i, i, ctypes.c_int64, u16p, u16p, i, i, u8p]
    L.oracle_sad_cost.argtypes = [u8p, u8p, i, i, ctypes.c_int64, i, i, i, u16p]
    L.oracle_aggregate.argtypes = [u16p, i, i, i, ctypes.c_uint32, i, i, u16p]
    L.oracle_wta.argtypes = [u16p, i, i, i, u16p]
    L.oracle_wta.restype = None
    L.oracle_right_disparity.argtypes = [u16p, i, i, i, u16p]
    L.oracle_right_disparity.restype = None
    L.oracle_lr_check.argtypes = [u16p, u16p, i, i, i, ctypes.c_uint16, u16p]
    L.oracle_lr_check.restype = None
    L.oracle_median.argtypes = [u16p, i, i, i, u16p]
    L.oracle_uv_maps.argtypes = [u16p, i, i, i, u16p, u16p]
    L.oracle_uv_filter.argtypes = [u16p, i, i, i, i, i, i, i, i, i, u8p]
    L.oracle_set_threads.argtypes = [i]
    L.oracle_set_threads.restype = None
    L.oracle_threads.argtypes = []
    L.oracle_threads.restype = ctypes.c_int


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        raise OracleError("%s failed with code %d (1 = 16-bit overflow, 2 = bad args)" % (what, rc))


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def threads() -> int:
    return int(lib().oracle_threads())


def census(img: np.ndarray, cw: int, ch: int) -> np.ndarray:
    img = np.ascontiguousarray(img, np.uint8)
    h, w = img.shape
    out = np.zeros((h, w), np.uint64)
    _check(lib().oracle_census(_p(img, ctypes.c_uint8), w, h, w, cw, ch, _p(out, ctypes.c_uint64)),
           "census")
    return out


def cost(cl: np.ndarray, cr: np.ndarray, d_max: int, nbits: int) -> np.ndarray:
    cl = np.ascontiguousarray(cl, np.uint64)
    cr = np.ascontiguousarray(cr, np.uint64)
    h, w = cl.shape
    out = np.zeros((h, w, d_max), np.uint16)
    _check(lib().oracle_cost(_p(cl, ctypes.c_uint64), _p(cr, ctypes.c_uint64), w, h, d_max, nbits,
                             _p(out, ctypes.c_uint16)), "cost")
    return out


def rectify(src: np.ndarray, map_x: np.ndarray, map_y: np.ndarray) -> np.ndarray:
    src = np.ascontiguousarray(src, np.uint8)
    map_x = np.ascontiguousarray(map_x, np.uint16)
    map_y = np.ascontiguousarray(map_y, np.uint16)
    sh, sw = src.shape
    h, w = map_x.shape
    out = np.zeros((h, w), np.uint8)
    _check(lib().oracle_rectify(_p(src, ctypes.c_uint8), sw, sh, sw, _p(map_x, ctypes.c_uint16),
                                _p(map_y, ctypes.c_uint16), w, h, _p(out, ctypes.c_uint8)), "rectify")
    return out


def sad_cost(left: np.ndarray, right: np.ndarray, ww: int, wh: int, d_max: int) -> np.ndarray:
    left = np.ascontiguousarray(left, np.uint8)
    right = np.ascontiguousarray(right, np.uint8)
    h, w = left.shape
    out = np.zeros((h, w, d_max), np.uint16)
    _check(lib().oracle_sad_cost(_p(left, ctypes.c_uint8), _p(right, ctypes.c_uint8), w, h, w, ww, wh, d_max,
                                 _p(out, ctypes.c_uint16)), "sad_cost")
    return out


def aggregate(c: np.ndarray, mask: int, p1: int, p2: int) -> np.ndarray:
    c = np.ascontiguousarray(c, np.uint16)
    h, w, d = c.shape
    out = np.zeros((h, w, d), np.uint16)
    _check(lib().oracle_aggregate(_p(c, ctypes.c_uint16), w, h, d, mask, p1, p2,
                                  _p(out, ctypes.c_uint16)), "aggregate")
    return out


def wta(s: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(s, np.uint16)
    h, w, d = s.shape
    out = np.zeros((h, w), np.uint16)
    lib().oracle_wta(_p(s, ctypes.c_uint16), w, h, d, _p(out, ctypes.c_uint16))
    return out


def right_disparity(s: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(s, np.uint16)
    h, w, d = s.shape
    out = np.zeros((h, w), np.uint16)
    lib().oracle_right_disparity(_p(s, ctypes.c_uint16), w, h, d, _p(out, ctypes.c_uint16))
    return out


def lr_check(dl: np.ndarray, dr: np.ndarray, max_diff: int, invalid: int) -> np.ndarray:
    dl = np.ascontiguousarray(dl, np.uint16)
    dr = np.ascontiguousarray(dr, np.uint16)
    h, w = dl.shape
    out = np.zeros((h, w), np.uint16)
    lib().oracle_lr_check(_p(dl, ctypes.c_uint16), _p(dr, ctypes.c_uint16), w, h, max_diff,
                          invalid, _p(out, ctypes.c_uint16))
    return out


def median(img: np.ndarray, k: int) -> np.ndarray:
    img = np.ascontiguousarray(img, np.uint16)
    h, w = img.shape
    out = np.zeros((h, w), np.uint16)
    _check(lib().oracle_median(_p(img, ctypes.c_uint16), w, h, k, _p(out, ctypes.c_uint16)),
           "median")
    return out


def uv_maps(disp: np.ndarray, d_max: int):
    disp = np.ascontiguousarray(disp, np.uint16)
    h, w = disp.shape
    u = np.zeros((d_max, w), np.uint16)
    v = np.zeros((h, d_max), np.uint16)
    _check(lib().oracle_uv_maps(_p(disp, ctypes.c_uint16), w, h, d_max, _p(u, ctypes.c_uint16),
                                _p(v, ctypes.c_uint16)), "uv_maps")
    return u, v


def uv_filter(m: np.ndarray, thr: int, dil_r: int, blur_r: int, roi=None) -> np.ndarray:
    """Threshold, dilation, binomial Gaussian and region of interest of one
    U- or V-map (uint16 [rows][cols]) -> uint8 [rows][cols].  roi = (r0, r1,
    c0, c1), default the whole map."""
    m = np.ascontiguousarray(m, np.uint16)
    rows, cols = m.shape
    r0, r1, c0, c1 = roi if roi is not None else (0, rows, 0, cols)
    out = np.zeros((rows, cols), np.uint8)
    _check(lib().oracle_uv_filter(_p(m, ctypes.c_uint16), rows, cols, thr, dil_r, blur_r, r0, r1, c0, c1,
                                  _p(out, ctypes.c_uint8)), "uv_filter")
    return out


def default_invalid(d_max: int) -> int:
    return 255 if d_max <= 255 else 65535


def select(s, d_max, lr_check_on=True, lr_max_diff=1, median_k=3, invalid=None):
    """Disparity selection from the aggregated volume S [H][W][D], in the
    paper's order: winner-takes-all (section 3.1.3), right-view disparity and
    left-right check (section 3.1.4), k x k median of the checked map
    (section 3.1.5), U-/V-maps of the final map (section 3.2).  Returns a dict
    of every intermediate map."""
    invalid = default_invalid(d_max) if invalid is None else invalid
    dl = wta(s)
    out = {"disp_l": dl}
    if lr_check_on:
        dr = right_disparity(s)
        dlr = lr_check(dl, dr, lr_max_diff, invalid)
        out["disp_r"] = dr
    else:
        dlr = dl
    out["disp_lr"] = dlr
    disp = median(dlr, median_k) if median_k else dlr
    u, v = uv_maps(disp, d_max)
    out.update(disp=disp, umap=u, vmap=v)
    return out


def sgm(left, right, d_max, census_w, census_h, mask, p1, p2, lr_check_on=True,
        lr_max_diff=1, median_k=3, invalid=None, cost_kind=0):
    """The whole path: census -> cost -> aggregate -> WTA -> (right disparity,
    LR check) -> median -> U/V maps, or with cost_kind = 1 the SAD cost over
    the census_w x census_h window instead of census + Hamming.  Returns a
    dict of every stage output."""
    if cost_kind == 1:
        c = sad_cost(left, right, census_w, census_h, d_max)
        out = {"cost": c}
    else:
        nbits = census_w * census_h - 1
        cl = census(left, census_w, census_h)
        cr = census(right, census_w, census_h)
        c = cost(cl, cr, d_max, nbits)
        out = {"census_l": cl, "census_r": cr, "cost": c}
    s = aggregate(c, mask, p1, p2)
    out["aggr"] = s
    out.update(select(s, d_max, lr_check_on, lr_max_diff, median_k, invalid))
    return out
