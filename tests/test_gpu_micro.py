"""GPU parity of the microbenchmark kernels (Sec. 7.2.1: Jacobi iterations
of the 2-D 9-point operator, temporally blocked) and of the pentadiagonal
line solves (Sec. 7.1, SP-shaped), against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_13304_amd import inputs
from tests.gpu_util import banner, dev, host, rel_inf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import paper_2204_13304_amd as pkg
    assert torch.cuda.is_available()
    return pkg


@pytest.mark.parametrize("shape", [(45, 70), (64, 64), (1, 1), (200, 130),
                                   (257, 3)])
@pytest.mark.parametrize("iters", [1, 5, 16])
def test_jacobi9_parity_and_block_independence(m, shape, iters):
    banner(f"jacobi9 {shape} iters {iters}")
    b = inputs.standard_normal(30, shape)
    x0 = inputs.standard_normal(31, shape)
    ref = oracle.jacobi9(b, x0, iters)
    outs = []
    for tb in (1, 2, 4, 8):
        x = dev(x0)
        m.jacobi9(dev(b), x, iters, tblock=tb)
        outs.append(host(x))
        assert rel_inf(outs[-1], ref) <= 1e-13
    for o in outs[1:]:
        # the fused iterations recompute the halo with the same arithmetic
        assert np.array_equal(o, outs[0])


def test_jacobi9_full_size_sampled(m):
    """4096^2, 64 iterations: a point after T iterations depends only on
    its (2T+1)^2 neighbourhood, so the oracle runs on that window (clipped
    to the grid, where the Dirichlet boundary is the true one)."""
    n, T = 4096, 64
    banner(f"jacobi9 {n}^2 x {T}")
    b = inputs.standard_normal(32, (n, n))
    x0 = np.zeros((n, n))
    x = dev(x0)
    m.jacobi9(dev(b), x, T, tblock=8)
    out = host(x)
    for (py, px) in [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1),
                     (2000, 1), (17, 3001), (2048, 2048), (4000, 100)]:
        y0, y1 = max(0, py - T), min(n, py + T + 1)
        x0_, x1_ = max(0, px - T), min(n, px + T + 1)
        win = oracle.jacobi9(b[y0:y1, x0_:x1_], x0[y0:y1, x0_:x1_], T)
        ref = win[py - y0, px - x0_]
        assert abs(out[py, px] - ref) <= 1e-13 * max(1.0, abs(ref))


def test_jacobi9_rejects_bad_arguments(m):
    b = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(RuntimeError):
        m.jacobi9(b, x, 3, tblock=3)
    with pytest.raises(RuntimeError):
        m.jacobi9(b, x, 3, tmp=x)


def _penta(shape, seed):
    rng = np.random.default_rng(seed)
    coef = rng.uniform(-1.0, 1.0, (5,) + shape)
    coef[2] += 6.0
    return coef, rng.standard_normal(shape)


@pytest.mark.parametrize("axis", ["x", "y", "z"])
@pytest.mark.parametrize("shape", [(7, 9, 11), (1, 1, 1), (3, 65, 2),
                                   (33, 4, 70)])
def test_penta_lines_parity(m, axis, shape):
    banner(f"penta {axis} {shape}")
    coef, r = _penta(shape, 40)
    x = m.penta_lines(dev(coef), dev(r), axis)
    ref = oracle.penta_lines(coef, r, axis)
    assert rel_inf(host(x), ref) <= 1e-13


def test_penta_lines_full_size_162(m):
    shape = (162, 162, 162)
    banner("penta 162^3")
    coef, r = _penta(shape, 41)
    cg, rg = dev(coef), dev(r)
    for axis in ("x", "y", "z"):
        x = m.penta_lines(cg, rg, axis)
        assert rel_inf(host(x), oracle.penta_lines(coef, r, axis)) <= 1e-13


def test_penta_lines_rejects_aliasing(m):
    coef = torch.zeros((5, 4, 4, 4), dtype=torch.float64, device="cuda")
    r = torch.zeros((4, 4, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError):
        m.penta_lines(coef, r, "x", x=coef[0])
