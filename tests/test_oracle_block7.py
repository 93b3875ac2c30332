"""Pins of the oracle's BLOCK7x5 SpMV and block SSOR half-sweeps (the
NPB-LU-shaped kernel; SSOR as one of the paper's Seidel-style routines,
Sec. 1 and Sec. 4.3.3) against a Kronecker-assembled block matrix and the
closed forms of SOR and SSOR."""
import numpy as np
import pytest

import oracle
from tests import assemble
from paper_2204_13304_amd import inputs

SHAPES = [(2, 3, 4), (3, 3, 3), (1, 2, 5)]


def _blocks(seed=4):
    return inputs.block7_blocks(seed)


@pytest.mark.parametrize("shape", SHAPES)
def test_spmv_vs_assembled(shape):
    nz, ny, nx = shape
    B = _blocks()
    A = assemble.block7(nx, ny, nz, B)
    x = inputs.standard_normal(1, shape + (5,))
    y = oracle.spmv_block7(x, B)
    ref = A @ x.ravel()
    assert np.max(np.abs(y.ravel() - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_lu5_matches_numpy():
    B = _blocks()
    lu, piv = oracle.lu5(B[0])
    s = inputs.standard_normal(2, 5)
    # reconstruct P A = L U
    L = np.tril(lu, -1) + np.eye(5)
    U = np.triu(lu)
    PA = B[0].copy()
    for c in range(5):
        PA[[c, piv[c]]] = PA[[piv[c], c]]
    assert np.allclose(L @ U, PA, atol=1e-14)
    assert np.allclose(np.linalg.solve(B[0], s),
                       np.linalg.solve(U, np.linalg.solve(L, s[
                           _perm(piv)])), atol=1e-14)


def _perm(piv):
    p = np.arange(5)
    for c in range(5):
        p[[c, piv[c]]] = p[[piv[c], c]]
    return p


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("omega", [1.0, 1.2])
def test_forward_sor_closed_form(shape, omega):
    # (D + w L) x_new = w b - (w U + (w - 1) D) x_old
    nz, ny, nx = shape
    B = _blocks()
    A = assemble.block7(nx, ny, nz, B)
    L, D, U = (m.toarray() for m in assemble.split_block_ldu(A))
    b = inputs.standard_normal(3, shape + (5,))
    x0 = inputs.standard_normal(4, shape + (5,))
    x1 = oracle.ssor_block7(b, x0, B, omega, "fwd")
    ref = np.linalg.solve(D + omega * L, omega * b.ravel() -
                          (omega * U + (omega - 1) * D) @ x0.ravel())
    assert np.max(np.abs(x1.ravel() - ref)) <= 1e-13 * np.max(np.abs(ref))
    xb = oracle.ssor_block7(b, x0, B, omega, "bwd")
    ref = np.linalg.solve(D + omega * U, omega * b.ravel() -
                          (omega * L + (omega - 1) * D) @ x0.ravel())
    assert np.max(np.abs(xb.ravel() - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", SHAPES)
def test_ssor_iteration_closed_form(shape):
    # one SSOR iteration = x + M^{-1}(b - A x),
    # M = (D + wL) D^{-1} (D + wU) / (w (2 - w))
    nz, ny, nx = shape
    w = 1.2
    B = _blocks()
    A = assemble.block7(nx, ny, nz, B)
    L, D, U = (m.toarray() for m in assemble.split_block_ldu(A))
    Ad = A.toarray()
    b = inputs.standard_normal(5, shape + (5,))
    x0 = inputs.standard_normal(6, shape + (5,))
    x1 = oracle.ssor_block7(b, x0, B, w, "sym")
    M = (D + w * L) @ np.linalg.solve(D, D + w * U) / (w * (2 - w))
    ref = x0.ravel() + np.linalg.solve(M, b.ravel() - Ad @ x0.ravel())
    assert np.max(np.abs(x1.ravel() - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_ssor_converges_to_ones():
    shape = (4, 4, 4)
    B = _blocks()
    nz, ny, nx = shape
    A = assemble.block7(nx, ny, nz, B)
    b = (A @ np.ones(A.shape[0])).reshape(shape + (5,))
    x = np.zeros_like(b)
    for _ in range(30):
        x = oracle.ssor_block7(b, x, B, 1.2, "sym")
    assert np.max(np.abs(x - 1)) < 1e-10


def test_scalar_reduction_to_gauss_seidel():
    # w = 1 with blocks c_d * I decouples into 5 scalar 7-point
    # Gauss-Seidel problems; with unit-coefficient faces the VAR7 sweep
    # is the same scalar problem.
    shape = (3, 4, 5)
    nz, ny, nx = shape
    B = np.zeros((7, 5, 5))
    B[0] = 6 * np.eye(5)
    for d in range(1, 7):
        B[d] = -np.eye(5)
    kx, ky, kz = (np.ones((nz, ny, nx + 1)), np.ones((nz, ny + 1, nx)),
                  np.ones((nz + 1, ny, nx)))
    b = inputs.standard_normal(7, shape + (5,))
    x0 = inputs.standard_normal(8, shape + (5,))
    xs = oracle.ssor_block7(b, x0, B, 1.0, "fwd")
    for c in range(5):
        ref = oracle.symgs_var7(b[..., c], x0[..., c], kx, ky, kz, "fwd")
        assert np.max(np.abs(xs[..., c] - ref)) <= 1e-14
