"""Python binding of libsgm.so (include/sgm.h): argument marshalling only.

Every entry point keeps the C name and takes torch CUDA tensors (device
memory) plus an optional torch stream; all computation runs in the library's
HIP kernels.  There is no fallback: if libsgm.so is missing or the GPU is not
usable, the calls raise.

    from paper_1807_06271_amd import sgm
    ctx = sgm.Context()
    p = sgm.Params(width=1242, height=375, max_disp=128)
    sgm.sgm_census(ctx, p, left, census_l)
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import torch  # loaded first so that libsgm.so shares torch's HIP runtime

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsgm.so")

SGM_OK, SGM_EINVAL, SGM_ENOMEM, SGM_EHIP, SGM_EBUSY, SGM_ENOTFOUND = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "SGM_OK", -1: "SGM_EINVAL", -2: "SGM_ENOMEM", -3: "SGM_EHIP", -4: "SGM_EBUSY",
                -5: "SGM_ENOTFOUND"}

PATH_L2R, PATH_R2L, PATH_T2B, PATH_B2T = 1, 2, 4, 8
PATH_TL2BR, PATH_BR2TL, PATH_TR2BL, PATH_BL2TR = 16, 32, 64, 128
PATHS_PAPER4 = PATH_L2R | PATH_TL2BR | PATH_T2B | PATH_TR2BL
PATHS_HV4 = PATH_L2R | PATH_R2L | PATH_T2B | PATH_B2T
PATHS_ALL8 = 0xFF
COST_CENSUS, COST_SAD = 0, 1
HCOSTS_DEFAULT, HCOSTS_VOLUME, HCOSTS_CODES = 0, 1, 2
TWOPASS_DEFAULT, TWOPASS_OFF, TWOPASS_WIDE, TWOPASS_NARROW = 0, 1, 2, 3

EXPORTS = ["sgm_validate", "sgm_create", "sgm_destroy", "sgm_last_error", "sgm_census", "sgm_cost",
           "sgm_cost_sad",
           "sgm_aggregate",
           "sgm_disparity", "uv_maps", "sgm_submit", "sgm_poll", "sgm_wait", "sgm_memory", "sgm_profile",
           "sgm_profile_read", "sgm_set_streams", "sgm_set_schedule", "sgm_get_schedule",
           "sgm_autotune", "sgm_set_graphs", "sgm_graph_stats", "sgm_rectify",
           "sgm_submit_rectify", "uv_filter", "sgm_submit_after",
           "sgm_disparity_noalloc", "sgm_set_split", "sgm_set_stripe_wait"]
STAGES = ["census", "aggregate", "disparity", "median", "uv", "rectify"]


class SgmError(RuntimeError):
    def __init__(self, status: int, what: str, message: str):
        super().__init__("%s: %s (%s)" % (what, message, STATUS_NAMES.get(status, status)))
        self.status = status


class sgm_params(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("max_disp", ctypes.c_int32),
                ("census_w", ctypes.c_int32), ("census_h", ctypes.c_int32),
                ("path_mask", ctypes.c_uint32), ("p1", ctypes.c_uint16), ("p2", ctypes.c_uint16),
                ("lr_check", ctypes.c_int32), ("lr_max_diff", ctypes.c_int32),
                ("median", ctypes.c_int32), ("invalid", ctypes.c_uint16),
                ("cost", ctypes.c_uint16)]


class sgm_schedule(ctypes.Structure):
    _fields_ = [("h_lanes", ctypes.c_int32), ("sweep", ctypes.c_int32), ("disp_threads", ctypes.c_int32),
                ("h_costs", ctypes.c_int32), ("two_pass", ctypes.c_int32)]


class sgm_remap(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("map_x", ctypes.c_void_p), ("map_y", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("src_pitch", ctypes.c_int64), ("out_pitch", ctypes.c_int64),
                ("src_w", ctypes.c_int32), ("src_h", ctypes.c_int32), ("w", ctypes.c_int32),
                ("h", ctypes.c_int32)]


class uv_filter_job(ctypes.Structure):
    _fields_ = [("map", ctypes.c_void_p), ("out", ctypes.c_void_p), ("rows", ctypes.c_int32),
                ("cols", ctypes.c_int32), ("threshold", ctypes.c_uint16), ("dilate_r", ctypes.c_uint16),
                ("blur_r", ctypes.c_uint16), ("reserved", ctypes.c_uint16), ("roi_r0", ctypes.c_int32),
                ("roi_r1", ctypes.c_int32), ("roi_c0", ctypes.c_int32), ("roi_c1", ctypes.c_int32)]


class sgm_frame(ctypes.Structure):
    _fields_ = [("left", ctypes.c_void_p), ("right", ctypes.c_void_p), ("pitch", ctypes.c_int64),
                ("p", sgm_params), ("disp", ctypes.c_void_p), ("umap", ctypes.c_void_p),
                ("vmap", ctypes.c_void_p)]


@dataclasses.dataclass
class Params:
    """Frame parameters (mirrors sgm_params)."""
    width: int
    height: int
    max_disp: int
    census_w: int = 9
    census_h: int = 7
    path_mask: int = PATHS_ALL8
    p1: int = 10
    p2: int = 120
    lr_check: int = 1
    lr_max_diff: int = 1
    median: int = 3
    invalid: int | None = None
    cost: int = COST_CENSUS  # or COST_SAD (census_w x census_h support region)

    @property
    def nbits(self) -> int:
        return self.census_w * self.census_h - 1

    @property
    def cmax(self) -> int:
        """Largest matching cost: N_b (Census) or window * 255 (SAD)."""
        return self.census_w * self.census_h * 255 if self.cost == COST_SAD else self.nbits

    @property
    def paths(self) -> int:
        return bin(self.path_mask).count("1")

    def inv(self) -> int:
        return (255 if self.max_disp <= 255 else 65535) if self.invalid is None else self.invalid

    def c(self) -> sgm_params:
        return sgm_params(self.width, self.height, self.max_disp, self.census_w, self.census_h,
                          self.path_mask, self.p1, self.p2, self.lr_check, self.lr_max_diff,
                          self.median, self.inv(), self.cost)

    def disp_evals(self) -> int:
        """W*H*D*paths: the unit of the throughput metric."""
        return self.width * self.height * self.max_disp * self.paths


_lib = None


def lib():
    """Load libsgm.so once (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsgm.so is not built; run `python -m paper_1807_06271_amd.build` "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, P = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER
        L.sgm_validate.argtypes = [P(sgm_params)]
        L.sgm_create.argtypes = [P(vp), i32, ctypes.c_size_t]
        L.sgm_destroy.argtypes = [vp]
        L.sgm_last_error.argtypes = []
        L.sgm_last_error.restype = ctypes.c_char_p
        L.sgm_census.argtypes = [vp, P(sgm_params), vp, ctypes.c_int64, vp, vp]
        L.sgm_rectify.argtypes = [vp, P(sgm_remap), i32, vp]
        L.uv_filter.argtypes = [vp, P(uv_filter_job), i32, vp]
        L.sgm_submit_rectify.argtypes = [vp, P(sgm_frame), P(sgm_remap), i32, P(ctypes.c_uint64)]
        L.sgm_cost.argtypes = [vp, P(sgm_params), vp, vp, vp, vp]
        L.sgm_cost_sad.argtypes = [vp, P(sgm_params), vp, vp, ctypes.c_int64, vp, vp]
        L.sgm_aggregate.argtypes = [vp, P(sgm_params), vp, vp, vp]
        L.sgm_disparity.argtypes = [vp, P(sgm_params), vp, vp, vp]
        L.sgm_disparity_noalloc.argtypes = [vp, P(sgm_params), vp, vp, vp]
        L.uv_maps.argtypes = [vp, P(sgm_params), vp, vp, vp, vp]
        L.sgm_submit.argtypes = [vp, P(sgm_frame), i32, P(ctypes.c_uint64)]
        L.sgm_submit_after.argtypes = [vp, P(sgm_frame), i32, P(vp), i32, P(ctypes.c_uint64)]
        L.sgm_poll.argtypes = [vp, ctypes.c_uint64, P(i32)]
        L.sgm_wait.argtypes = [vp, ctypes.c_uint64]
        L.sgm_memory.argtypes = [vp, P(ctypes.c_size_t), P(ctypes.c_size_t)]
        L.sgm_profile.argtypes = [vp, i32]
        L.sgm_set_streams.argtypes = [vp, i32]
        L.sgm_set_split.argtypes = [vp, i32]
        L.sgm_set_graphs.argtypes = [vp, i32]
        L.sgm_graph_stats.argtypes = [vp, P(ctypes.c_uint64), P(ctypes.c_uint64)]
        L.sgm_set_schedule.argtypes = [vp, P(sgm_params), P(sgm_schedule)]
        L.sgm_get_schedule.argtypes = [vp, P(sgm_params), P(sgm_schedule)]
        L.sgm_autotune.argtypes = [vp, P(sgm_frame), i32, i32, P(sgm_schedule), P(ctypes.c_float), i32]
        L.sgm_profile_read.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_uint64), i32]
        for name in EXPORTS:
            if name != "sgm_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str) -> int:
    if rc != SGM_OK:
        raise SgmError(rc, what, lib().sgm_last_error().decode(errors="replace"))
    return rc


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _need(t, shape, dtype, name):
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype:
        raise ValueError("%s must be %s %s, got %s %s" % (name, dtype, tuple(shape), t.dtype, tuple(t.shape)))


def sgm_validate(p: Params) -> None:
    """Raise SgmError(SGM_EINVAL) if the parameters are not accepted (no GPU used)."""
    _check(lib().sgm_validate(ctypes.byref(p.c())), "sgm_validate")


class Context:
    """An sgm_ctx on one device; frees it on close() / exit / GC."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().sgm_create(ctypes.byref(self._h), device, hbm_budget_bytes), "sgm_create")
        self.device = device

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("context is closed")
        return self._h

    def close(self):
        if self._h:
            h, self._h = self._h, ctypes.c_void_p()
            _check(lib().sgm_destroy(h), "sgm_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _rows(t, name, dtype):
    if t.dtype != dtype or t.dim() != 2 or t.stride(1) != 1 or not t.is_cuda:
        raise ValueError("%s must be a CUDA %s [rows][pitch] tensor with contiguous rows" % (name, dtype))


def remap_job(src, map_x, map_y, out) -> sgm_remap:
    """One sgm_remap from tensors: src uint8 [src_h][src_w] (row pitch from its
    stride), map_x/map_y contiguous uint16 [h][w], out uint8 [h][w] (pitch from
    its stride).  The struct holds raw device pointers: keep the tensors alive
    until the work is done."""
    _rows(src, "src", torch.uint8)
    _rows(out, "out", torch.uint8)
    _need(map_x, tuple(out.shape), torch.uint16, "map_x")
    _need(map_y, tuple(out.shape), torch.uint16, "map_y")
    h, w = out.shape
    return sgm_remap(src.data_ptr(), _ptr(map_x), _ptr(map_y), out.data_ptr(), src.stride(0), out.stride(0),
                     src.shape[1], src.shape[0], w, h)


def sgm_rectify(ctx: Context, jobs, stream=None):
    """Rectify every (src, map_x, map_y, out) of `jobs` (tuples or sgm_remap)."""
    rj = [j if isinstance(j, sgm_remap) else remap_job(*j) for j in jobs]
    arr = (sgm_remap * max(len(rj), 1))(*rj)
    _check(lib().sgm_rectify(ctx.handle, arr, len(rj), _stream(stream)), "sgm_rectify")


def filter_job(m, out, threshold: int, dilate_r: int = 1, blur_r: int = 2, roi=None) -> uv_filter_job:
    """One uv_filter_job: m uint16 [rows][cols] (a U- or V-map), out uint8
    [rows][cols]; roi = (r0, r1, c0, c1), default the whole map.  The struct
    holds raw device pointers: keep m and out alive until the work is done."""
    _need(out, tuple(m.shape), torch.uint8, "out")
    if m.dtype != torch.uint16 or m.dim() != 2:
        raise ValueError("map must be uint16 [rows][cols]")
    rows, cols = m.shape
    r0, r1, c0, c1 = roi if roi is not None else (0, rows, 0, cols)
    return uv_filter_job(_ptr(m), _ptr(out), rows, cols, threshold, dilate_r, blur_r, 0, r0, r1, c0, c1)


def uv_filter(ctx: Context, jobs, stream=None):
    """Threshold, dilate, blur and crop every map of `jobs` (uv_filter_job or
    (map, out, threshold, dilate_r, blur_r[, roi]) tuples) in one launch."""
    fj = [j if isinstance(j, uv_filter_job) else filter_job(*j) for j in jobs]
    arr = (uv_filter_job * max(len(fj), 1))(*fj)
    _check(lib().uv_filter(ctx.handle, arr, len(fj), _stream(stream)), "uv_filter")


def sgm_census(ctx: Context, p: Params, img, census, stream=None):
    _need(census, (p.height, p.width), torch.uint64, "census")
    if img.dtype != torch.uint8 or img.dim() != 2 or img.shape[0] != p.height or img.shape[1] < p.width:
        raise ValueError("img must be uint8 [H][pitch >= W]")
    pitch = img.stride(0)
    if img.stride(1) != 1:
        raise ValueError("img rows must be contiguous")
    _check(lib().sgm_census(ctx.handle, ctypes.byref(p.c()), img.data_ptr(), pitch, _ptr(census),
                            _stream(stream)), "sgm_census")


def sgm_cost(ctx: Context, p: Params, cl, cr, cost, stream=None):
    for t, n in ((cl, "cl"), (cr, "cr")):
        _need(t, (p.height, p.width), torch.uint64, n)
    _need(cost, (p.height, p.width, p.max_disp), torch.uint16, "cost")
    _check(lib().sgm_cost(ctx.handle, ctypes.byref(p.c()), _ptr(cl), _ptr(cr), _ptr(cost),
                          _stream(stream)), "sgm_cost")


def sgm_cost_sad(ctx: Context, p: Params, left, right, cost, stream=None):
    for t, n in ((left, "left"), (right, "right")):
        if t.dtype != torch.uint8 or t.dim() != 2 or t.shape[0] != p.height or t.shape[1] < p.width \
                or t.stride(1) != 1:
            raise ValueError("%s must be uint8 [H][pitch >= W] with contiguous rows" % n)
    if left.stride(0) != right.stride(0):
        raise ValueError("left and right must share one pitch")
    _need(cost, (p.height, p.width, p.max_disp), torch.uint16, "cost")
    _check(lib().sgm_cost_sad(ctx.handle, ctypes.byref(p.c()), left.data_ptr(), right.data_ptr(), left.stride(0),
                              _ptr(cost), _stream(stream)), "sgm_cost_sad")


def sgm_aggregate(ctx: Context, p: Params, cost, aggr, stream=None):
    for t, n in ((cost, "cost"), (aggr, "aggr")):
        _need(t, (p.height, p.width, p.max_disp), torch.uint16, n)
    _check(lib().sgm_aggregate(ctx.handle, ctypes.byref(p.c()), _ptr(cost), _ptr(aggr), _stream(stream)),
           "sgm_aggregate")


def sgm_disparity(ctx: Context, p: Params, aggr, disp, stream=None):
    _need(aggr, (p.height, p.width, p.max_disp), torch.uint16, "aggr")
    _need(disp, (p.height, p.width), torch.uint16, "disp")
    _check(lib().sgm_disparity(ctx.handle, ctypes.byref(p.c()), _ptr(aggr), _ptr(disp), _stream(stream)),
           "sgm_disparity")


def sgm_disparity_noalloc(ctx: Context, p: Params, aggr, disp, stream=None):
    """sgm_disparity with the library's fixed scratch: no device allocation."""
    _need(aggr, (p.height, p.width, p.max_disp), torch.uint16, "aggr")
    _need(disp, (p.height, p.width), torch.uint16, "disp")
    _check(lib().sgm_disparity_noalloc(ctx.handle, ctypes.byref(p.c()), _ptr(aggr), _ptr(disp),
                                       _stream(stream)), "sgm_disparity_noalloc")


def uv_maps(ctx: Context, p: Params, disp, umap, vmap, stream=None):
    _need(disp, (p.height, p.width), torch.uint16, "disp")
    _need(umap, (p.max_disp, p.width), torch.uint16, "umap")
    _need(vmap, (p.height, p.max_disp), torch.uint16, "vmap")
    _check(lib().uv_maps(ctx.handle, ctypes.byref(p.c()), _ptr(disp), _ptr(umap), _ptr(vmap),
                         _stream(stream)), "uv_maps")


@dataclasses.dataclass
class Frame:
    """One frame for sgm_submit: inputs and (preallocated) outputs."""
    p: Params
    left: torch.Tensor
    right: torch.Tensor
    disp: torch.Tensor
    umap: torch.Tensor | None = None
    vmap: torch.Tensor | None = None

    @staticmethod
    def alloc(p: Params, left, right, uv: bool = True) -> "Frame":
        dev = left.device
        disp = torch.empty((p.height, p.width), dtype=torch.uint16, device=dev)
        u = torch.empty((p.max_disp, p.width), dtype=torch.uint16, device=dev) if uv else None
        v = torch.empty((p.height, p.max_disp), dtype=torch.uint16, device=dev) if uv else None
        return Frame(p, left, right, disp, u, v)

    def c(self) -> sgm_frame:
        for t, n in ((self.left, "left"), (self.right, "right")):
            if t.dtype != torch.uint8 or t.dim() != 2 or t.shape[0] != self.p.height \
                    or t.shape[1] < self.p.width or t.stride(1) != 1:
                raise ValueError("%s must be uint8 [H][pitch >= W] with contiguous rows" % n)
        if self.left.stride(0) != self.right.stride(0):
            raise ValueError("left and right must share one pitch")
        _need(self.disp, (self.p.height, self.p.width), torch.uint16, "disp")
        if (self.umap is None) != (self.vmap is None):
            raise ValueError("give both umap and vmap or neither")
        if self.umap is not None:
            _need(self.umap, (self.p.max_disp, self.p.width), torch.uint16, "umap")
            _need(self.vmap, (self.p.height, self.p.max_disp), torch.uint16, "vmap")
        return sgm_frame(self.left.data_ptr(), self.right.data_ptr(), self.left.stride(0), self.p.c(),
                         _ptr(self.disp), _ptr(self.umap), _ptr(self.vmap))


def sgm_submit(ctx: Context, frames) -> int:
    """Enqueue a batch; returns its ticket.  Raises SgmError with status
    SGM_EBUSY when the batch does not fit next to the batches in flight."""
    arr = (sgm_frame * len(frames))(*[f.c() for f in frames])
    t = ctypes.c_uint64()
    _check(lib().sgm_submit(ctx.handle, arr, len(frames), ctypes.byref(t)), "sgm_submit")
    return t.value


def sgm_submit_rectify(ctx: Context, frames, remaps) -> int:
    """sgm_submit with rectification first: remaps[2i] / remaps[2i+1]
    ((src, map_x, map_y) tuples, or sgm_remap) fill frame i's left / right
    buffers from raw images on the batch's stream.  Returns the ticket."""
    if len(remaps) != 2 * len(frames):
        raise ValueError("need two remaps (left, right) per frame")
    rj = []
    for i, r in enumerate(remaps):
        if not isinstance(r, sgm_remap):
            f = frames[i // 2]
            view = f.right if i & 1 else f.left
            r = remap_job(r[0], r[1], r[2], view[:, :f.p.width])
        rj.append(r)
    arr = (sgm_frame * len(frames))(*[f.c() for f in frames])
    rarr = (sgm_remap * len(rj))(*rj)
    t = ctypes.c_uint64()
    _check(lib().sgm_submit_rectify(ctx.handle, arr, rarr, len(frames), ctypes.byref(t)), "sgm_submit_rectify")
    return t.value


def _events(after):
    """ctypes array of raw HIP event handles of torch.cuda.Event objects."""
    ev = [e.cuda_event if hasattr(e, "cuda_event") else int(e) for e in after]
    return (ctypes.c_void_p * len(ev))(*ev), len(ev)


def sgm_submit_after(ctx: Context, frames, after) -> int:
    """sgm_submit whose batch waits on the GPU for the events `after`
    (torch.cuda.Event, recorded) before its first launch."""
    arr = (sgm_frame * len(frames))(*[f if isinstance(f, sgm_frame) else f.c() for f in frames])
    ev, n = _events(after)
    t = ctypes.c_uint64()
    _check(lib().sgm_submit_after(ctx.handle, arr, len(frames), ev, n, ctypes.byref(t)), "sgm_submit_after")
    return t.value


def try_submit(ctx: Context, frames, after=()) -> int | None:
    """Like sgm_submit (sgm_submit_after when events are given in `after`),
    but returns None instead of raising on SGM_EBUSY.  `frames` may hold
    Frame objects or their already marshalled sgm_frame structs (Frame.c()),
    which a caller that resubmits the same buffers can keep."""
    arr = (sgm_frame * len(frames))(*[f if isinstance(f, sgm_frame) else f.c() for f in frames])
    t = ctypes.c_uint64()
    if after:
        ev, n = _events(after)
        rc = lib().sgm_submit_after(ctx.handle, arr, len(frames), ev, n, ctypes.byref(t))
    else:
        rc = lib().sgm_submit(ctx.handle, arr, len(frames), ctypes.byref(t))
    if rc == SGM_EBUSY:
        return None
    _check(rc, "sgm_submit")
    return t.value


def sgm_poll(ctx: Context, ticket: int) -> bool:
    done = ctypes.c_int()
    _check(lib().sgm_poll(ctx.handle, ticket, ctypes.byref(done)), "sgm_poll")
    return bool(done.value)


def sgm_wait(ctx: Context, ticket: int) -> None:
    _check(lib().sgm_wait(ctx.handle, ticket), "sgm_wait")


def sgm_memory(ctx: Context):
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().sgm_memory(ctx.handle, ctypes.byref(a), ctypes.byref(b)), "sgm_memory")
    return a.value, b.value


def sgm_set_schedule(ctx: Context, p: Params | None, h_lanes: int, sweep: bool = False,
                     disp_threads: int = 0, h_costs: int = HCOSTS_DEFAULT,
                     two_pass: int = TWOPASS_DEFAULT) -> None:
    """Schedule for frames of p's shape (p=None: the default): lanes per
    horizontal scanline, whether eligible frames use the single-pass sweep,
    the disparity-selection block size (0: by block count), where the
    horizontal scanlines take their costs from (HCOSTS_*), and whether the
    vertical and diagonal paths run as two stripe passes (TWOPASS_*)."""
    sc = sgm_schedule(h_lanes, int(bool(sweep)), int(disp_threads), int(h_costs), int(two_pass))
    _check(lib().sgm_set_schedule(ctx.handle, ctypes.byref(p.c()) if p is not None else None,
                                  ctypes.byref(sc)), "sgm_set_schedule")


def sgm_get_schedule(ctx: Context, p: Params) -> int:
    """Lanes per horizontal scanline that sgm_submit would use for p's shape."""
    return schedule_of(ctx, p)[0]


def schedule_of(ctx: Context, p: Params):
    """(h_lanes, sweep, disp_threads, h_costs, two_pass) that sgm_submit
    would use for frames like p."""
    sc = sgm_schedule()
    _check(lib().sgm_get_schedule(ctx.handle, ctypes.byref(p.c()), ctypes.byref(sc)), "sgm_get_schedule")
    return sc.h_lanes, bool(sc.sweep), sc.disp_threads, sc.h_costs, sc.two_pass


AUTOTUNE_CANDIDATES = ("h_lanes=16", "h_lanes=32", "h_lanes=64", "h_costs=codes", "two_pass=wide",
                       "two_pass=narrow", "disp_threads=256", "disp_threads=512", "disp_threads=1024", "sweep")
TWOPASS_NAMES = {TWOPASS_OFF: "off", TWOPASS_WIDE: "wide", TWOPASS_NARROW: "narrow"}


def sgm_autotune(ctx: Context, sample, reps: int = 5):
    """Time the candidate schedules on `sample` (a Frame, or a list of
    Frames of one shape submitted as one batch) (lanes per horizontal
    scanline; horizontal costs from Census codes where that applies; the
    two-pass stripes where they apply; the disparity block size; the sweep
    where it applies) and keep the fastest for its shape.  Returns
    (schedule, {candidate: ms per submit}) with schedule = {"h_lanes",
    "sweep", "disp_threads", "h_costs", "two_pass"}."""
    frames = list(sample) if isinstance(sample, (list, tuple)) else [sample]
    arr = (sgm_frame * len(frames))(*[f.c() for f in frames])
    best = sgm_schedule()
    n = len(AUTOTUNE_CANDIDATES)
    ms = (ctypes.c_float * n)()
    _check(lib().sgm_autotune(ctx.handle, arr, len(frames), reps, ctypes.byref(best), ms, n), "sgm_autotune")
    sched = {"h_lanes": best.h_lanes, "sweep": bool(best.sweep), "disp_threads": best.disp_threads,
             "h_costs": "codes" if best.h_costs == HCOSTS_CODES else "volume",
             "two_pass": TWOPASS_NAMES.get(best.two_pass, "off")}
    return sched, {name: ms[i] for i, name in enumerate(AUTOTUNE_CANDIDATES) if ms[i] >= 0}


def sgm_set_graphs(ctx: Context, on: bool) -> None:
    _check(lib().sgm_set_graphs(ctx.handle, int(bool(on))), "sgm_set_graphs")


def sgm_graph_stats(ctx: Context):
    """(hits, misses) of the batch graph cache."""
    h, m = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().sgm_graph_stats(ctx.handle, ctypes.byref(h), ctypes.byref(m)), "sgm_graph_stats")
    return h.value, m.value


def sgm_set_streams(ctx: Context, n: int) -> None:
    _check(lib().sgm_set_streams(ctx.handle, int(n)), "sgm_set_streams")


def sgm_set_stripe_wait(ctx: Context, max_polls: int = 0, withhold_edges: bool = False) -> None:
    """Bound the two-pass stripes' waits for a neighbour's edge (0: the
    default) and optionally withhold the edges (tests of the failure path)."""
    _check(lib().sgm_set_stripe_wait(ctx.handle, int(max_polls), int(bool(withhold_edges))), "sgm_set_stripe_wait")


def sgm_set_split(ctx: Context, n: int) -> None:
    """Spread each batch's frames over up to n of the context's streams."""
    _check(lib().sgm_set_split(ctx.handle, int(n)), "sgm_set_split")


def sgm_profile(ctx: Context, enable: bool) -> None:
    _check(lib().sgm_profile(ctx.handle, int(bool(enable))), "sgm_profile")


def sgm_profile_read(ctx: Context, reset: bool = False) -> dict:
    """{stage: (summed ms, launches)} for batches found done since the last reset."""
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_uint64 * len(STAGES))()
    _check(lib().sgm_profile_read(ctx.handle, ms, n, int(bool(reset))), "sgm_profile_read")
    return {name: (ms[i], n[i]) for i, name in enumerate(STAGES)}


def run_stages(ctx: Context, p: Params, left, right, stream=None, keep=False):
    """The per-frame path through the five stage calls.  Returns the final
    disparity map, U-map and V-map (and, with keep=True, every intermediate)."""
    dev = left.device
    H, W, D = p.height, p.width, p.max_disp
    cl = torch.empty((H, W), dtype=torch.uint64, device=dev)
    cr = torch.empty((H, W), dtype=torch.uint64, device=dev)
    cost = torch.empty((H, W, D), dtype=torch.uint16, device=dev)
    aggr = torch.empty((H, W, D), dtype=torch.uint16, device=dev)
    disp = torch.empty((H, W), dtype=torch.uint16, device=dev)
    u = torch.empty((D, W), dtype=torch.uint16, device=dev)
    v = torch.empty((H, D), dtype=torch.uint16, device=dev)
    if p.cost == COST_SAD:
        sgm_cost_sad(ctx, p, left, right, cost, stream)
    else:
        sgm_census(ctx, p, left, cl, stream)
        sgm_census(ctx, p, right, cr, stream)
        sgm_cost(ctx, p, cl, cr, cost, stream)
    sgm_aggregate(ctx, p, cost, aggr, stream)
    sgm_disparity(ctx, p, aggr, disp, stream)
    uv_maps(ctx, p, disp, u, v, stream)
    out = {"disp": disp, "umap": u, "vmap": v}
    if keep:
        out.update(census_l=cl, census_r=cr, cost=cost, aggr=aggr)
    return out
