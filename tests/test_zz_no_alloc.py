"""GPU test of m2s_dot_noalloc, the entry point that allocates nothing (its
reduction scratch is a fixed device array of the library): through the C
ABI, two calls in a row -- the second with a smaller input -- each give the
bits of m2s_dot on the same vectors (same kernel and reduction order), and
agree with an independent numpy dot to rounding."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2204_13304_amd import _lib as L
from tests.gpu_util import banner, dev

pytestmark = pytest.mark.gpu


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dot(fn, x, y, n=None):
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    st = fn(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
            C.c_int64(x.numel() if n is None else n),
            C.c_void_p(out.data_ptr()), _stream())
    assert st == L.M2S_OK, st
    torch.cuda.synchronize()
    return out.item()


def test_dot_noalloc_matches_dot_two_calls():
    lib = L.load()
    assert torch.cuda.is_available()
    rng = np.random.default_rng(81)
    for n in (3_000_001, 777):      # second call: a smaller input
        banner(f"dot_noalloc n={n}")
        xh, yh = rng.standard_normal(n), rng.standard_normal(n)
        x, y = dev(xh), dev(yh)
        got = _dot(lib.m2s_dot_noalloc, x, y)
        ref = _dot(lib.m2s_dot, x, y)
        assert got == ref, (n, got, ref)
        exact = float(np.dot(xh, yh))
        scale = float(np.dot(np.abs(xh), np.abs(yh)))
        assert abs(got - exact) <= 1e-13 * scale
    # zero length: the sum of nothing
    e = torch.ones(4, dtype=torch.float64, device="cuda")
    assert _dot(lib.m2s_dot_noalloc, e, e, n=0) == 0.0
    # argument errors are reported before anything is launched
    assert lib.m2s_dot_noalloc(None, None, 1, None, None) == 1
