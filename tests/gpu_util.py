"""Shared helpers of the GPU tests."""
import sys

import numpy as np
import pytest


def announce(*parts):
    """Name the case about to run on the GPU (flushed, so a fault still
    leaves the name in the log)."""
    print("[gpu-case]", *parts, file=sys.stderr, flush=True)


def gpu_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return torch


def to_dev(torch, a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_np(t):
    return t.cpu().numpy()


def assert_equal(got: np.ndarray, want: np.ndarray, what: str):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        idx = tuple(bad[0])
        raise AssertionError("%s: %d of %d elements differ; first at %s: got %s want %s"
                             % (what, len(bad), got.size, idx, got[idx], want[idx]))
