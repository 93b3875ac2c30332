"""GPU parity of the BLOCK7x5 SpMV and the block SSOR half-sweeps (NPB-LU
shaped, omega = 1.2) against the oracle, bitwise agreement of the tiled
wavefront kernel with the one-thread lexicographic kernel, and the
162^3 x 5 configuration point by point."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_13304_amd import inputs
from tests.gpu_util import banner, dev, host, rel_inf

pytestmark = pytest.mark.gpu

SHAPES = [(6, 7, 8), (13, 5, 9), (1, 1, 1), (2, 9, 3), (17, 17, 17)]


@pytest.fixture(scope="module")
def m():
    import paper_2204_13304_amd as pkg
    assert torch.cuda.is_available()
    return pkg


@pytest.mark.parametrize("shape", SHAPES)
def test_spmv_block7(m, shape):
    B = inputs.block7_blocks(4)
    A = m.block7(shape, B)
    x = inputs.standard_normal(1, shape + (5,))
    y = host(m.spmv(A, dev(x)))
    assert rel_inf(y, oracle.spmv_block7(x, B)) <= 1e-13


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("direction", ["fwd", "bwd", "sym"])
def test_ssor_parity(m, shape, direction):
    banner(f"ssor {direction} {shape}")
    B = inputs.block7_blocks(4)
    A = m.block7(shape, B)
    b = inputs.standard_normal(2, shape + (5,))
    x0 = inputs.standard_normal(3, shape + (5,))
    xg = dev(x0)
    m.ssor_sweep(A, dev(b), xg, 1.2, direction)
    ref = oracle.ssor_block7(b, x0, B, 1.2, direction)
    assert rel_inf(host(xg), ref) <= 1e-13


@pytest.mark.parametrize("shape", [(11, 9, 10), (21, 37, 19), (4, 16, 33)])
@pytest.mark.parametrize("direction", ["fwd", "bwd", "sym"])
def test_ssor_tiles_bitwise_vs_sequential(m, shape, direction):
    """Several tiles along j and k with ragged tails: parity with the oracle
    and bitwise equality with the sequential kernel."""
    banner(f"ssor tiles {direction} {shape}")
    B = inputs.block7_blocks(4)
    A = m.block7(shape, B)
    b = inputs.standard_normal(4, shape + (5,))
    x0 = inputs.standard_normal(5, shape + (5,))
    xg, xs = dev(x0), dev(x0)
    m.ssor_sweep(A, dev(b), xg, 1.2, direction)
    m.ssor_sweep_sequential(A, dev(b), xs, 1.2, direction)
    out = host(xg)
    assert rel_inf(out, oracle.ssor_block7(b, x0, B, 1.2, direction)) <= 1e-13
    assert np.array_equal(out, host(xs))


def test_ssor_omega_change_same_workspace(m):
    """The relaxation factor is built into the device constants; a new
    omega on the same workspace must take effect."""
    shape = (9, 18, 7)
    B = inputs.block7_blocks(4)
    A = m.block7(shape, B)
    ws = m.Workspace(A)
    b = inputs.standard_normal(6, shape + (5,))
    x0 = inputs.standard_normal(7, shape + (5,))
    for w in (1.2, 0.7, 1.2):
        xg = dev(x0)
        m.ssor_sweep(A, dev(b), xg, w, "sym", ws)
        ref = oracle.ssor_block7(b, x0, B, w, "sym")
        assert rel_inf(host(xg), ref) <= 1e-13


def test_ssor_iterations_converge(m):
    # 20 SSOR iterations from x0 = 0 on b = A*1 approach x = 1
    shape = (12, 12, 12)
    B = inputs.block7_blocks(4)
    A = m.block7(shape, B)
    bh = oracle.spmv_block7(np.ones(shape + (5,)), B)
    b = dev(bh)
    x = torch.zeros_like(b)
    for _ in range(20):
        m.ssor_sweep(A, b, x, 1.2, "sym")
    ref = np.zeros(shape + (5,))
    for _ in range(20):
        ref = oracle.ssor_block7(bh, ref, B, 1.2, "sym")
    assert rel_inf(host(x), ref) <= 1e-12
    assert np.max(np.abs(host(x) - 1)) < 1e-6


def test_full_size_ssor_162(m):
    # the NPB-LU-shaped configuration: one SSOR iteration at 162^3 x 5
    shape = (162, 162, 162)
    banner("ssor 162^3 x 5")
    B = inputs.block7_blocks(4)
    A = m.block7(shape, B)
    ones = np.ones(shape + (5,))
    b = oracle.spmv_block7(ones, B)
    xg = torch.zeros(shape + (5,), dtype=torch.float64, device="cuda")
    m.ssor_sweep(A, dev(b), xg, 1.2, "sym")
    ref = oracle.ssor_block7(b, np.zeros_like(b), B, 1.2, "sym")
    assert rel_inf(host(xg), ref) <= 1e-13


def test_full_size_ssor_162_random_start(m):
    # two SSOR iterations at 162^3 x 5 from a random x0, so that the forward
    # half-sweep reads non-zero old values across every tile boundary
    shape = (162, 162, 162)
    banner("ssor 162^3 x 5, random x0, 2 iterations")
    B = inputs.block7_blocks(4)
    A = m.block7(shape, B)
    b = oracle.spmv_block7(np.ones(shape + (5,)), B)
    x0 = inputs.standard_normal(73, shape + (5,))
    xg = dev(x0)
    ref = x0
    for _ in range(2):
        m.ssor_sweep(A, dev(b), xg, 1.2, "sym")
        ref = oracle.ssor_block7(b, ref, B, 1.2, "sym")
    assert rel_inf(host(xg), ref) <= 1e-13


def test_ssor_rejects_bad_omega(m):
    A = m.block7((4, 4, 4), inputs.block7_blocks(4))
    x = torch.zeros((4, 4, 4, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError):
        m.ssor_sweep(A, x.clone(), x, 2.5, "sym")


def test_tile_wait_timeout_is_reported_and_recovered(m, monkeypatch):
    # as for the 27-point tiles: a forced time-out is latched and reported,
    # and the workspace is usable afterwards
    shape = (12, 40, 8)
    banner("ssor forced tile wait time-out")
    B = inputs.block7_blocks(4)
    A = m.block7(shape, B)
    ws = m.Workspace(A)
    b = inputs.standard_normal(71, shape + (5,))
    x0 = inputs.standard_normal(72, shape + (5,))
    monkeypatch.setenv("M2S_SPIN_LIMIT", "1")
    m.ssor_sweep(A, dev(b), dev(x0), 1.2, "fwd", ws)
    with pytest.raises(RuntimeError, match="M2S_ERR_TIMEOUT"):
        ws.check()
    monkeypatch.delenv("M2S_SPIN_LIMIT")
    xg = dev(x0)
    m.ssor_sweep(A, dev(b), xg, 1.2, "sym", ws)
    ws.check()
    assert rel_inf(host(xg), oracle.ssor_block7(b, x0, B, 1.2, "sym")) <= 1e-13
