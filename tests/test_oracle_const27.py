"""Pins of the CPU oracle's CONST27 SpMV and Gauss-Seidel sweeps against
things other than itself: closed forms, an explicitly assembled sparse
matrix, triangular solves and symmetry (HPCG operator, Sec. 7.1; SymGS as
the textbook lexicographic routine, Sec. 4.3.3)."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from tests import assemble
from paper_2204_13304_amd import inputs

SHAPES = [(3, 4, 5), (5, 6, 7), (6, 6, 6), (1, 3, 4), (2, 1, 9)]


def test_closed_form_b_equals_A_ones():
    # b = A*1: 26 minus the number of in-grid neighbours -> interior 0,
    # face 9, edge 15, corner 19 (Dirichlet truncation of the 26/-1 row).
    n = 6
    b = oracle.spmv27(np.ones((n, n, n)))
    interior = b[1:-1, 1:-1, 1:-1]
    assert np.all(interior == 0)
    assert b[0, 0, 0] == 19 and b[-1, -1, -1] == 19 and b[0, -1, 0] == 19
    assert b[0, 0, 2] == 15 and b[2, 0, 0] == 15 and b[0, 3, -1] == 15
    assert b[0, 2, 3] == 9 and b[2, 3, -1] == 9 and b[-1, 2, 2] == 9


@pytest.mark.parametrize("shape", SHAPES)
def test_spmv_vs_assembled(shape):
    nz, ny, nx = shape
    A = assemble.const27(nx, ny, nz)
    x = inputs.standard_normal(11, shape)
    y = oracle.spmv27(x)
    yref = (A @ x.ravel()).reshape(shape)
    assert np.max(np.abs(y - yref)) <= 1e-13 * max(1, np.max(np.abs(yref)))


def test_spmv_symmetry():
    shape = (6, 5, 7)
    x = inputs.standard_normal(1, shape)
    y = inputs.standard_normal(2, shape)
    a = np.dot(x.ravel(), oracle.spmv27(y).ravel())
    b = np.dot(y.ravel(), oracle.spmv27(x).ravel())
    assert abs(a - b) <= 1e-13 * abs(a)


@pytest.mark.parametrize("shape", SHAPES)
def test_triangle_parts(shape):
    nz, ny, nx = shape
    A = assemble.const27(nx, ny, nz)
    L, D, U = assemble.split_ldu(A)
    x = inputs.standard_normal(3, shape).ravel()
    lo = oracle.spmv27_part(x.reshape(shape), -1).ravel()
    up = oracle.spmv27_part(x.reshape(shape), +1).ravel()
    assert np.allclose(lo, L @ x, atol=1e-13)
    assert np.allclose(up, U @ x, atol=1e-13)


@pytest.mark.parametrize("shape", SHAPES)
def test_symgs_fwd_is_lower_triangular_solve(shape):
    # forward sweep: (D + L) x_new = r - U x_old
    nz, ny, nx = shape
    A = assemble.const27(nx, ny, nz).toarray()
    r = inputs.standard_normal(4, shape)
    x0 = inputs.standard_normal(5, shape)
    x1 = oracle.symgs27(r, x0, "fwd")
    DL, U = np.tril(A), np.triu(A, 1)
    ref = sla.solve_triangular(DL, r.ravel() - U @ x0.ravel(), lower=True)
    assert np.max(np.abs(x1.ravel() - ref)) <= 1e-13 * np.max(np.abs(ref))
    # residual identity (D+L) x_new + U x_old = r: catches any order error
    res = DL @ x1.ravel() + U @ x0.ravel() - r.ravel()
    assert np.max(np.abs(res)) <= 1e-12


@pytest.mark.parametrize("shape", SHAPES)
def test_symgs_bwd_is_upper_triangular_solve(shape):
    nz, ny, nx = shape
    A = assemble.const27(nx, ny, nz).toarray()
    r = inputs.standard_normal(6, shape)
    x0 = inputs.standard_normal(7, shape)
    x1 = oracle.symgs27(r, x0, "bwd")
    DU, L = np.triu(A), np.tril(A, -1)
    ref = sla.solve_triangular(DU, r.ravel() - L @ x0.ravel(), lower=False)
    assert np.max(np.abs(x1.ravel() - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_symgs_from_zero_is_symmetric_operator():
    # S r = SymGS(r, 0) = (D+U)^{-1} D (D+L)^{-1} r, a symmetric operator.
    shape = (5, 4, 6)
    r1 = inputs.standard_normal(8, shape)
    r2 = inputs.standard_normal(9, shape)
    z = np.zeros(shape)
    s1 = oracle.symgs27(r1, z, "sym")
    s2 = oracle.symgs27(r2, z, "sym")
    a, b = np.dot(r2.ravel(), s1.ravel()), np.dot(r1.ravel(), s2.ravel())
    assert abs(a - b) <= 1e-13 * abs(a)
    nz, ny, nx = shape
    A = assemble.const27(nx, ny, nz).toarray()
    Dm = np.diag(np.diag(A))
    S = np.linalg.solve(np.triu(A), Dm @ np.linalg.solve(np.tril(A), r1.ravel()))
    assert np.max(np.abs(S - s1.ravel())) <= 1e-13 * np.max(np.abs(S))


def test_float32_instantiation_tracks_float64():
    shape = (8, 8, 8)
    r = inputs.standard_normal(10, shape)
    x0 = np.zeros(shape)
    x64 = oracle.symgs27(r, x0, "sym")
    x32 = oracle.symgs27(r.astype(np.float32), x0.astype(np.float32), "sym",
                         dtype=np.float32)
    rel = np.max(np.abs(x32 - x64)) / np.max(np.abs(x64))
    assert 0 < rel < 1e-5


def test_degenerate_single_point():
    # 1x1x1 grid: the sweep is x = r / 26, SpMV is 26 x.
    r = np.array([[[13.0]]])
    assert oracle.symgs27(r, np.zeros_like(r), "fwd")[0, 0, 0] == 0.5
    assert oracle.spmv27(r)[0, 0, 0] == 26 * 13.0


def _dense_sweep_adjoint(A, g, direction):
    """(gr, gx) of <g, S(r, x)> from the dense triangles of an assembled A:
    forward S = (D+L)^{-1}(r - U x), backward S = (D+U)^{-1}(r - L x), sym =
    backward after forward; transposed solves written out with
    solve_triangular(trans=1), no symmetry assumed."""
    DL, DU = np.tril(A), np.triu(A)
    U, L = np.triu(A, 1), np.tril(A, -1)
    if direction == "fwd":
        gr = sla.solve_triangular(DL, g, lower=True, trans=1)
        return gr, -U.T @ gr
    if direction == "bwd":
        gr = sla.solve_triangular(DU, g, lower=False, trans=1)
        return gr, -L.T @ gr
    grb, gmid = _dense_sweep_adjoint(A, g, "bwd")
    grf, gx = _dense_sweep_adjoint(A, gmid, "fwd")
    return grb + grf, gx


@pytest.mark.parametrize("shape", [(3, 4, 5), (6, 6, 6), (1, 2, 7)])
@pytest.mark.parametrize("direction", ["fwd", "bwd", "sym"])
def test_sweep_adjoint_vs_dense_transposed_solves(shape, direction):
    nz, ny, nx = shape
    A = assemble.const27(nx, ny, nz).toarray()
    g = inputs.standard_normal(7, shape)
    gr, gx = oracle.symgs_adjoint(g, direction)
    rr, rx = _dense_sweep_adjoint(A, g.ravel(), direction)
    assert np.max(np.abs(gr.ravel() - rr)) <= 1e-13 * np.max(np.abs(rr))
    assert np.max(np.abs(gx.ravel() - rx)) <= 1e-13 * np.max(np.abs(rx))
    # and the defining identity <g, S(r, x)> = <gr, r> + <gx, x> (S affine
    # in (r, x) with S(0, 0) = 0)
    r = inputs.standard_normal(8, shape)
    x = inputs.standard_normal(9, shape)
    lhs = np.dot(g.ravel(), oracle.symgs27(r, x, direction).ravel())
    rhs = np.dot(gr.ravel(), r.ravel()) + np.dot(gx.ravel(), x.ravel())
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
