"""Pins of the oracle's microbenchmark routines (Sec. 7.2.1: Jacobi
iterations of a 2-D 9-point stencil, the 27-point ILU(0) and the
factored-diagonal D-ILU) and of its
pentadiagonal and 5x5 block-tridiagonal line solves (the SP- and
BT-shaped systems of Sec. 7.1), against
closed forms, fixed points, defining properties and library routines
(scipy.sparse, scipy.linalg.solve_banded) -- never against a retyping of
the oracle's own loops."""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle


def _tri_ones(n):
    return sp.diags([np.ones(n - 1), np.ones(n), np.ones(n - 1)], [-1, 0, 1])


def _A9(ny, nx, diag=8.0, off=-1.0):
    """2-D 9-point operator as a sparse matrix: the neighbour sum of the
    3x3 box minus the centre is (T_y kron T_x - I)."""
    T = sp.kron(_tri_ones(ny), _tri_ones(nx)).tocsr()
    return (diag * sp.identity(nx * ny) + off * (T - sp.identity(nx * ny))).tocsr()


def _A27(nz, ny, nx, diag=26.0, off=-1.0):
    T = sp.kron(sp.kron(_tri_ones(nz), _tri_ones(ny)), _tri_ones(nx)).tocsr()
    n = nx * ny * nz
    return (diag * sp.identity(n) + off * (T - sp.identity(n))).tocsr()


# ------------------------------------------------------------- Jacobi
def test_jacobi9_one_step_from_zero():
    b = np.random.default_rng(0).standard_normal((9, 13))
    x = oracle.jacobi9(b, np.zeros_like(b), 1)
    assert np.array_equal(x, b / 8.0)


def test_jacobi9_fixed_point():
    ny, nx = 11, 17
    b = (_A9(ny, nx) @ np.ones(nx * ny)).reshape(ny, nx)
    x = oracle.jacobi9(b, np.ones((ny, nx)), 5)
    assert np.max(np.abs(x - 1)) <= 1e-15


@pytest.mark.parametrize("shape", [(7, 9), (1, 12), (16, 5)])
def test_jacobi9_against_sparse_matrix(shape):
    ny, nx = shape
    rng = np.random.default_rng(1)
    b = rng.standard_normal(shape)
    x0 = rng.standard_normal(shape)
    A = _A9(ny, nx)
    D = A.diagonal()
    x = x0.ravel().copy()
    for _ in range(6):
        x = x + (b.ravel() - A @ x) / D
    got = oracle.jacobi9(b, x0, 6)
    assert np.max(np.abs(got.ravel() - x)) <= 1e-13 * max(1, np.abs(x).max())


def test_jacobi9_converges_to_solution():
    ny, nx = 12, 12
    b = (_A9(ny, nx) @ np.ones(nx * ny)).reshape(ny, nx)
    e50 = np.abs(oracle.jacobi9(b, np.zeros_like(b), 50) - 1).max()
    e200 = np.abs(oracle.jacobi9(b, np.zeros_like(b), 200) - 1).max()
    assert e200 < e50 < 1


# ---------------------------------------------------------------- ILU
@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 6, 3), (4, 4, 4)])
def test_dilu27_diagonal_of_factor_matches_operator(shape):
    nz, ny, nx = shape
    A = _A27(nz, ny, nx)
    d = oracle.dilu27_factor(shape).ravel()
    L, U, D = sp.tril(A, -1), sp.triu(A, 1), sp.diags(d)
    M = ((D + L) @ sp.diags(1.0 / d) @ (D + U)).toarray()
    assert np.max(np.abs(np.diag(M) - 26.0)) <= 1e-13
    # off the diagonal M = A + L D^-1 U
    Mo = A.toarray() + (L @ sp.diags(1.0 / d) @ U).toarray()
    np.fill_diagonal(Mo, 0.0)
    M0 = M.copy()
    np.fill_diagonal(M0, 0.0)
    assert np.max(np.abs(M0 - Mo)) <= 1e-14


@pytest.mark.parametrize("shape", [(3, 4, 5), (5, 3, 2)])
def test_dilu27_solve_inverts_factor(shape):
    nz, ny, nx = shape
    A = _A27(nz, ny, nx)
    d = oracle.dilu27_factor(shape)
    r = np.random.default_rng(2).standard_normal(shape)
    z = oracle.dilu27_solve(d, r).ravel()
    dv = d.ravel()
    L, U, D = sp.tril(A, -1), sp.triu(A, 1), sp.diags(dv)
    Mz = (D + L) @ ((D + U) @ z / dv)
    assert np.max(np.abs(Mz - r.ravel())) <= 1e-13


def test_dilu27_is_exact_on_a_line():
    # one grid line: the 27-point operator is tridiagonal and its ILU the
    # exact LU factorisation
    shape = (1, 1, 23)
    A = _A27(*shape)
    d = oracle.dilu27_factor(shape)
    r = np.random.default_rng(3).standard_normal(shape)
    z = oracle.dilu27_solve(d, r).ravel()
    ref = spla.spsolve(A.tocsc(), r.ravel())
    assert np.max(np.abs(z - ref)) <= 1e-14 * np.abs(ref).max()


# -------------------------------------------------- pentadiagonal lines
def _ilu0_matrices(Lf, Uf):
    """Assemble the unit lower L and the upper U from the ILU(0) factor
    arrays (offsets in lexicographic (dk, dj, di) order)."""
    nz, ny, nx = Lf.shape[:3]
    n = nx * ny * nz
    L = np.eye(n)
    U = np.zeros((n, n))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = (k * ny + j) * nx + i
                U[p, p] = Uf[k, j, i, 0]
                for m in range(27):
                    dk, dj, di = m // 9 - 1, (m // 3) % 3 - 1, m % 3 - 1
                    kk, jj, ii = k + dk, j + dj, i + di
                    if not (0 <= kk < nz and 0 <= jj < ny and 0 <= ii < nx):
                        continue
                    q = (kk * ny + jj) * nx + ii
                    if m < 13:
                        L[p, q] = Lf[k, j, i, m]
                    elif m > 13:
                        U[p, q] = Uf[k, j, i, 1 + m - 14]
    return L, U


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 6, 3), (4, 4, 4),
                                   (5, 5, 5), (1, 4, 7)])
def test_ilu0_27_reproduces_operator_on_its_pattern(shape):
    # the defining property of ILU(0): L unit lower and U upper with the
    # pattern of A, and (L U)_pq = a_pq on that pattern (the fill outside it
    # dropped)
    nz, ny, nx = shape
    A = _A27(nz, ny, nx).toarray()
    Lf, Uf = oracle.ilu0_27_factor(shape)
    L, U = _ilu0_matrices(Lf, Uf)
    pat = A != 0
    assert np.all(np.tril(L, -1)[~pat] == 0) and np.all(np.triu(U, 1)[~pat] == 0)
    LU = L @ U
    assert np.max(np.abs(LU[pat] - A[pat])) <= 1e-13
    # fill outside the pattern exists (it is not the complete LU)
    if min(shape) >= 3:
        assert np.max(np.abs(LU[~pat])) > 1e-3


def test_ilu0_27_differs_from_the_factored_diagonal_variant():
    # the factored-diagonal variant (D-ILU) keeps A's off-diagonals, so its
    # M = (D + L) D^{-1} (D + U) misses the off-diagonal pattern entries that
    # ILU(0) reproduces
    shape = (4, 4, 4)
    A = _A27(*shape)
    d = oracle.dilu27_factor(shape).ravel()
    L, U, D = sp.tril(A, -1), sp.triu(A, 1), sp.diags(d)
    M = ((D + L) @ sp.diags(1.0 / d) @ (D + U)).toarray()
    pat = A.toarray() != 0
    assert np.max(np.abs(M[pat] - A.toarray()[pat])) > 1e-3


@pytest.mark.parametrize("shape", [(3, 4, 5), (4, 4, 4)])
def test_ilu0_27_factors_are_symmetric(shape):
    # A is symmetric, so L = U^T diag(U)^{-1}: l_pq = u_qp / u_qq (the form
    # the GPU factor stores, 14 values per point)
    Lf, Uf = oracle.ilu0_27_factor(shape)
    L, U = _ilu0_matrices(Lf, Uf)
    Ls = np.tril(U.T / np.diag(U)[None, :], -1) + np.eye(L.shape[0])
    assert np.max(np.abs(L - Ls)) <= 1e-14


@pytest.mark.parametrize("shape", [(3, 4, 5), (5, 3, 2), (6, 6, 6)])
def test_ilu0_27_solve_inverts_LU(shape):
    Lf, Uf = oracle.ilu0_27_factor(shape)
    L, U = _ilu0_matrices(Lf, Uf)
    r = np.random.default_rng(7).standard_normal(shape)
    z = oracle.ilu0_27_solve(Lf, Uf, r).ravel()
    res = L @ (U @ z) - r.ravel()
    assert np.max(np.abs(res)) <= 1e-13 * np.abs(r).max()


@pytest.mark.parametrize("shape", [(2, 2, 2), (1, 1, 17), (1, 2, 2)])
def test_ilu0_27_is_exact_when_nothing_is_dropped(shape):
    # on a 2x2x2 grid every point neighbours every other (A is dense), and
    # on one line A is tridiagonal: no fill-in is dropped, so ILU(0) is the
    # complete LU and the solve is A^{-1} r
    A = _A27(*shape).toarray()
    Lf, Uf = oracle.ilu0_27_factor(shape)
    r = np.random.default_rng(8).standard_normal(shape)
    z = oracle.ilu0_27_solve(Lf, Uf, r).ravel()
    ref = scipy.linalg.solve(A, r.ravel())
    assert np.max(np.abs(z - ref)) <= 1e-14 * np.abs(ref).max() * 10


def _penta(shape, seed):
    rng = np.random.default_rng(seed)
    coef = rng.uniform(-1.0, 1.0, (5,) + shape)
    coef[2] += 6.0  # diagonally dominant
    return coef, rng.standard_normal(shape)


@pytest.mark.parametrize("axis", ["x", "y", "z"])
@pytest.mark.parametrize("shape", [(4, 5, 6), (1, 1, 9), (7, 3, 2)])
def test_penta_lines_against_solve_banded(axis, shape):
    coef, r = _penta(shape, 4)
    x = oracle.penta_lines(coef, r, axis)
    ax = {"x": 2, "y": 1, "z": 0}[axis]
    c = np.moveaxis(coef, ax + 1, -1)
    rr = np.moveaxis(r, ax, -1)
    xx = np.moveaxis(x, ax, -1)
    n = rr.shape[-1]
    for idx in np.ndindex(rr.shape[:-1]):
        a, b, cc, d, e = (c[(k,) + idx] for k in range(5))
        ab = np.zeros((5, n))
        # solve_banded: ab[u + i - j, j] = A[i, j], u = 2
        ab[0, 2:] = e[:-2]
        ab[1, 1:] = d[:-1]
        ab[2, :] = cc
        ab[3, :-1] = b[1:]
        ab[4, :-2] = a[2:]
        ref = scipy.linalg.solve_banded((2, 2), ab, rr[idx])
        assert np.max(np.abs(xx[idx] - ref)) <= 1e-13 * max(1, np.abs(ref).max())


def test_penta_lines_residual():
    shape = (3, 4, 11)
    coef, r = _penta(shape, 5)
    x = oracle.penta_lines(coef, r, "x")
    a, b, c, d, e = coef
    res = c * x
    res[..., 1:] += b[..., 1:] * x[..., :-1]
    res[..., 2:] += a[..., 2:] * x[..., :-2]
    res[..., :-1] += d[..., :-1] * x[..., 1:]
    res[..., :-2] += e[..., :-2] * x[..., 2:]
    assert np.max(np.abs(res - r)) <= 1e-13


# ------------------------------------------ block-tridiagonal (5x5) lines
def _bt_matrix(coef, axis):
    """The block-tridiagonal operator of every line of `axis` as one sparse
    matrix over the grid's 5-vectors (C order of (nz, ny, nx, 5))."""
    nz, ny, nx = coef.shape[1:4]
    ax = {"x": 2, "y": 1, "z": 0}[axis]
    length = (nz, ny, nx)[ax]
    step = (nx * ny, nx, 1)[ax]
    idx = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    pos = np.indices((nz, ny, nx))[ax]
    rows, cols, vals = [], [], []
    for blk, off in ((0, -1), (1, 0), (2, 1)):
        ok = (pos + off >= 0) & (pos + off < length)
        p = idx[ok]
        q = p + off * step
        v = coef[blk][ok]  # (m, 5, 5)
        for a in range(5):
            for b in range(5):
                rows.append(5 * p + a)
                cols.append(5 * q + b)
                vals.append(v[:, a, b])
    n5 = 5 * nx * ny * nz
    return sp.csr_matrix((np.concatenate(vals),
                          (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n5, n5))


@pytest.mark.parametrize("axis", ["x", "y", "z"])
@pytest.mark.parametrize("shape", [(3, 4, 5), (1, 1, 7), (6, 1, 1),
                                   (2, 5, 3)])
def test_bt_lines_against_spsolve(axis, shape):
    from paper_2204_13304_amd import inputs
    coef, r = inputs.bt_problem(60, shape)
    x = oracle.bt_lines(coef, r, axis)
    ref = spla.spsolve(_bt_matrix(coef, axis).tocsc(), r.ravel())
    assert np.max(np.abs(x.ravel() - ref)) <= 1e-13 * np.abs(ref).max()


def test_bt_lines_uncoupled_is_pointwise_solve():
    # with A = C = 0 every point is its own 5x5 system B_p x_p = r_p
    from paper_2204_13304_amd import inputs
    coef, r = inputs.bt_problem(61, (3, 4, 6))
    coef[0] = 0.0
    coef[2] = 0.0
    ref = np.linalg.solve(coef[1], r[..., None])[..., 0]
    for axis in ("x", "y", "z"):
        x = oracle.bt_lines(coef, r, axis)
        assert np.max(np.abs(x - ref)) <= 1e-14 * np.abs(ref).max()


def test_bt_lines_residual_and_singular_pivot():
    from paper_2204_13304_amd import inputs
    coef, r = inputs.bt_problem(62, (2, 3, 9))
    x = oracle.bt_lines(coef, r, "x")
    A, B, C = coef
    res = np.einsum("...ab,...b->...a", B, x)
    res[..., 1:, :] += np.einsum("...ab,...b->...a", A[..., 1:, :, :],
                                 x[..., :-1, :])
    res[..., :-1, :] += np.einsum("...ab,...b->...a", C[..., :-1, :, :],
                                  x[..., 1:, :])
    assert np.max(np.abs(res - r)) <= 1e-13 * np.abs(r).max()
    coef[1, 0, 0, 0] = 0.0  # a zero first pivot block: reported, not hidden
    coef[0, 0, 0, 0] = 0.0
    with pytest.raises(ValueError, match="singular"):
        oracle.bt_lines(coef, r, "x")
