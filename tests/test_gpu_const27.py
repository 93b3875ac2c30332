"""GPU parity of the CONST27 SpMV and the exact lexicographic SymGS
wavefront against the CPU oracle (relative 1e-13 in FP64), bitwise
agreement of the wavefront with the one-thread sequential kernel, the
residual identity of a forward sweep, and the FP32 path."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_13304_amd import inputs
from tests import assemble
from tests.gpu_util import banner, dev, host, rel_inf

pytestmark = pytest.mark.gpu

SHAPES = [(16, 16, 16), (9, 26, 13), (40, 17, 33), (1, 1, 1), (2, 3, 70),
          (70, 3, 2), (5, 1, 8), (24, 24, 24)]


@pytest.fixture(scope="module")
def m():
    import paper_2204_13304_amd as pkg
    assert torch.cuda.is_available()
    return pkg


@pytest.mark.parametrize("shape", SHAPES)
def test_spmv_parity(m, shape):
    banner(f"spmv27 {shape}")
    A = m.const27(shape)
    x = inputs.standard_normal(0, shape)
    y = host(m.spmv(A, dev(x)))
    assert rel_inf(y, oracle.spmv27(x)) <= 1e-13
    ones = np.ones(shape)
    assert np.array_equal(host(m.spmv(A, dev(ones))), oracle.spmv27(ones))


# shapes around the SpMV tiling: 64 x 16 (x, y) tiles of layers of planes
# (64 x 32 in FP32), ragged in x and y, one or two planes, several layers
SPMV_SHAPES = [(3, 33, 130), (2, 17, 65), (64, 16, 64), (33, 48, 200),
               (7, 95, 129)]


@pytest.mark.parametrize("shape", SPMV_SHAPES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_spmv_tiling_edges(m, shape, dtype):
    banner(f"spmv27 tiling {shape} {dtype}")
    A = m.const27(shape, dtype=dtype)
    x = inputs.standard_normal(6, shape)
    y = host(m.spmv(A, dev(x, dtype)))
    ref = oracle.spmv27(x.astype(np.float32).astype(np.float64)
                        if dtype == torch.float32 else x)
    assert rel_inf(y, ref) <= (1e-13 if dtype == torch.float64 else 2e-6)


def test_pcg_on_a_wide_plane(m):
    # a 1 x 1040 x 2048 grid has more SpMV tiles than the fused p.Ap's
    # reduction partials hold, so the SpMV and the dot run as two kernels
    shape = (1, 1040, 2048)
    banner(f"pcg wide plane {shape}")
    A = m.const27(shape)
    b = inputs.standard_normal(7, shape)
    x, info = m.pcg_solve(A, dev(b), None, "none", max_iter=4, rtol=0.0)
    ref = oracle.pcg(b, precond="none", max_iter=4)
    assert info["iters"] == ref["iters"] == 4
    assert rel_inf(host(x), ref["x"]) <= 1e-12


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("direction", ["fwd", "bwd", "sym"])
def test_symgs_parity_and_bitwise(m, shape, direction):
    banner(f"symgs27 {direction} {shape}")
    A = m.const27(shape)
    r = inputs.standard_normal(1, shape)
    x0 = inputs.standard_normal(2, shape)
    ref = oracle.symgs27(r, x0, direction)
    xg = dev(x0)
    m.symgs(A, dev(r), xg, direction)
    out = host(xg)
    assert rel_inf(out, ref) <= 1e-13
    xs = dev(x0)
    m.symgs_sequential(A, dev(r), xs, direction)
    assert np.array_equal(out, host(xs)), "wavefront != sequential"


@pytest.mark.parametrize("nw", ["1", "2", "4"])
def test_symgs_tile_height_bitwise(m, nw, monkeypatch):
    # every tile height (4 planes per wavefront, 1, 2 or 4 wavefronts) gives
    # the identical result: only the schedule changes, never the arithmetic
    monkeypatch.setenv("M2S_C27_WAVES", nw)
    shape = (21, 19, 23)
    banner(f"symgs27 wavefronts per tile {nw}")
    A = m.const27(shape)
    r = inputs.standard_normal(3, shape)
    x0 = inputs.standard_normal(4, shape)
    xg = dev(x0)
    m.symgs(A, dev(r), xg, "sym")
    xs = dev(x0)
    m.symgs_sequential(A, dev(r), xs, "sym")
    assert np.array_equal(host(xg), host(xs))


@pytest.mark.parametrize("direction", ["fwd", "bwd"])
def test_symgs_many_tiles_and_few_tiles_bitwise(m, direction):
    # more tiles than workgroups (the sweep polls 4 steps ahead) on a thin
    # grid, and few tiles (2 steps ahead): both bitwise equal to the
    # sequential kernel and within 1e-13 of the oracle
    for shape in ((200, 200, 5), (24, 24, 24)):
        banner(f"symgs27 tile count {shape} {direction}")
        A = m.const27(shape)
        r = inputs.standard_normal(12, shape)
        x0 = inputs.standard_normal(13, shape)
        xg = dev(x0)
        m.symgs(A, dev(r), xg, direction)
        xs = dev(x0)
        m.symgs_sequential(A, dev(r), xs, direction)
        out = host(xg)
        assert np.array_equal(out, host(xs))
        assert rel_inf(out, oracle.symgs27(r, x0, direction)) <= 1e-13
    assert m.plan_sweep(m.const27((200, 200, 5)))["nslabs"] > 256
    assert m.plan_sweep(m.const27((24, 24, 24)))["nslabs"] <= 256


def test_residual_identity(m):
    # (D + L) x_new + U x_old = r for a forward sweep, evaluated on the CPU
    shape = (12, 20, 18)
    A = m.const27(shape)
    r = inputs.standard_normal(5, shape)
    x0 = inputs.standard_normal(6, shape)
    x1 = dev(np.zeros(shape))
    m.symgs_oop(A, dev(r), dev(x0), x1, "fwd")
    x1 = host(x1)
    # the GPU output goes through the independently assembled matrix, not
    # through the oracle
    Lp, Dp, Up = assemble.split_ldu(assemble.const27(shape[2], shape[1],
                                                     shape[0]))
    lhs = (Dp + Lp) @ x1.ravel() + Up @ x0.ravel()
    assert np.max(np.abs(lhs - r.ravel())) <= 1e-12


def test_zero_start_sweep(m):
    shape = (16, 16, 16)
    A = m.const27(shape)
    r = inputs.standard_normal(7, shape)
    out = dev(np.full(shape, np.nan))
    m.symgs_oop(A, dev(r), None, out, "fwd")
    ref = oracle.symgs27(r, np.zeros(shape), "fwd")
    assert rel_inf(host(out), ref) <= 1e-13


def test_float32_path(m):
    shape = (20, 18, 22)
    A = m.const27(shape, dtype=torch.float32)
    r = inputs.standard_normal(8, shape)
    x0 = inputs.standard_normal(9, shape)
    xg = dev(x0, torch.float32)
    m.symgs(A, dev(r, torch.float32), xg, "sym")
    out = host(xg)
    ref32 = oracle.symgs27(r.astype(np.float32), x0.astype(np.float32),
                           "sym", dtype=np.float32)
    ref64 = oracle.symgs27(r, x0, "sym")
    assert rel_inf(out, ref32) <= 2e-6
    assert rel_inf(out, ref64) <= 2e-6
    y = host(m.spmv(A, dev(x0, torch.float32)))
    assert rel_inf(y, oracle.spmv27(x0)) <= 2e-6


@pytest.mark.parametrize("n", [104, 256])
def test_full_size_symgs(m, n):
    # the configuration the benchmark times, compared point by point
    shape = (n, n, n)
    banner(f"symgs27 full size {shape}")
    A = m.const27(shape)
    r = inputs.standard_normal(10, shape)
    x0 = inputs.standard_normal(11, shape)
    xg = dev(x0)
    m.symgs(A, dev(r), xg, "sym")
    out = host(xg)
    ref = oracle.symgs27(r, x0, "sym")
    assert rel_inf(out, ref) <= 1e-13
    y = host(m.spmv(A, dev(x0)))
    assert rel_inf(y, oracle.spmv27(x0)) <= 1e-13


def test_full_size_symgs_512_forward(m):
    # the larger-than-MALL probe size (1.07 GB per vector), compared point
    # by point; the deepest buffer offsets the sweep kernels form
    shape = (512, 512, 512)
    banner(f"symgs27 full size {shape} fwd")
    A = m.const27(shape)
    r = inputs.standard_normal(12, shape)
    x0 = inputs.standard_normal(13, shape)
    out = torch.empty(shape, dtype=torch.float64, device="cuda")
    m.symgs_oop(A, dev(r), dev(x0), out, "fwd")
    got = host(out)
    del out
    assert rel_inf(got, oracle.symgs27(r, x0, "fwd")) <= 1e-13


def test_tile_wait_timeout_is_reported_and_recovered(m, monkeypatch):
    # a spin limit of one poll makes a tile give up waiting for a producer
    # tile's boundary records: every role of every workgroup leaves its step
    # loop together, the latch reports the time-out, and the workspace works
    # afterwards
    shape = (24, 40, 12)
    banner("symgs27 forced tile wait time-out")
    A = m.const27(shape)
    ws = m.Workspace(A)
    r = inputs.standard_normal(66, shape)
    x0 = inputs.standard_normal(67, shape)
    monkeypatch.setenv("M2S_SPIN_LIMIT", "1")
    m.symgs(A, dev(r), dev(x0), "fwd", ws)
    with pytest.raises(RuntimeError, match="M2S_ERR_TIMEOUT"):
        ws.check()
    monkeypatch.delenv("M2S_SPIN_LIMIT")
    xg = dev(x0)
    m.symgs(A, dev(r), xg, "sym", ws)
    ws.check()
    assert rel_inf(host(xg), oracle.symgs27(r, x0, "sym")) <= 1e-13
