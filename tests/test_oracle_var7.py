"""Pins of the oracle's VAR7 operator (D^T K D from the paper's D and P
matrices, Sec. 4.1), its sweeps, the coarse-coefficient reading and the
face-coefficient gradient (checked against finite differences)."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from tests import assemble
from paper_2204_13304_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SHAPES = [(3, 4, 5), (4, 4, 4), (2, 5, 3), (1, 1, 6)]


def _problem(shape, seed=21):
    return inputs.var7_problem(seed, shape)


def test_paper_matrices_fixture():
    # D_(n) and P = [0; I; 0] as printed in Sec. 4.1, and the 1-D VAR7
    # operator with unit faces equal to (D P)^T (D P) = tridiag(-1, 2, -1).
    with open(os.path.join(GOLD, "paper_sec4_1_matrices.json")) as fh:
        g = json.load(fh)
    D4 = assemble.diff_matrix(4).toarray()
    assert np.array_equal(D4, np.array(g["D_4"], float))
    P2 = assemble.pad_matrix(2).toarray()
    assert np.array_equal(P2, np.array(g["P_2"], float))
    n = g["laplace_1d_n"]
    kx = np.ones((1, 1, n + 1))
    ky = np.zeros((1, 2, n))
    kz = np.zeros((2, 1, n))
    A = np.column_stack([
        oracle.spmv_var7(np.eye(n)[c].reshape(1, 1, n), kx, ky, kz).ravel()
        for c in range(n)])
    assert np.array_equal(A, np.array(g["laplace_1d"], float))


@pytest.mark.parametrize("shape", SHAPES)
def test_spmv_vs_DtKD(shape):
    pr = _problem(shape)
    A = assemble.var7(pr["kx"], pr["ky"], pr["kz"])
    x = inputs.standard_normal(3, shape)
    y = oracle.spmv_var7(x, pr["kx"], pr["ky"], pr["kz"])
    ref = A @ x.ravel()
    assert np.max(np.abs(y.ravel() - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_spd():
    shape = (3, 4, 5)
    pr = _problem(shape)
    A = assemble.var7(pr["kx"], pr["ky"], pr["kz"]).toarray()
    assert np.allclose(A, A.T, atol=0)
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("shape", SHAPES)
def test_sweeps_are_triangular_solves(shape):
    pr = _problem(shape)
    kx, ky, kz = pr["kx"], pr["ky"], pr["kz"]
    A = assemble.var7(kx, ky, kz).toarray()
    r = inputs.standard_normal(4, shape)
    x0 = inputs.standard_normal(5, shape)
    xf = oracle.symgs_var7(r, x0, kx, ky, kz, "fwd")
    ref = sla.solve_triangular(np.tril(A), r.ravel() - np.triu(A, 1) @
                               x0.ravel(), lower=True)
    assert np.max(np.abs(xf.ravel() - ref)) <= 1e-13 * np.max(np.abs(ref))
    xb = oracle.symgs_var7(r, x0, kx, ky, kz, "bwd")
    ref = sla.solve_triangular(np.triu(A), r.ravel() - np.tril(A, -1) @
                               x0.ravel(), lower=False)
    assert np.max(np.abs(xb.ravel() - ref)) <= 1e-13 * np.max(np.abs(ref))
    lo = oracle.spmv_var7_part(x0, kx, ky, kz, -1).ravel()
    assert np.allclose(lo, np.tril(A, -1) @ x0.ravel(), rtol=0, atol=1e-13)
    up = oracle.spmv_var7_part(x0, kx, ky, kz, +1).ravel()
    assert np.allclose(up, np.triu(A, 1) @ x0.ravel(), rtol=0, atol=1e-13)
    assert np.allclose(lo + up + np.diag(A) * x0.ravel(), A @ x0.ravel(),
                       rtol=0, atol=1e-12)


def _schur_conductances(k):
    """Face conductances of the exact coarse operator on a 1-D line: the
    fine operator D^T K D (Sec. 4.1, assembled through the paper's D and P
    matrices) with faces k[0..n], the odd points eliminated (Schur
    complement onto the even points, which injection keeps).  Returns the
    n/2 + 1 conductances: the coupling between consecutive coarse points,
    and at each end the row sum, i.e. the coupling to the Dirichlet ghost."""
    n = len(k) - 1
    D = assemble.padded_diff(n).toarray()
    A = D.T @ np.diag(k) @ D
    ev, od = np.arange(0, n, 2), np.arange(1, n, 2)
    S = (A[np.ix_(ev, ev)] - A[np.ix_(ev, od)] @
         np.linalg.solve(A[np.ix_(od, od)], A[np.ix_(od, ev)]))
    m = len(ev)
    if m == 1:  # one coarse point touches both ghosts: only the total
        return S[0, 0]
    c = np.empty(m + 1)
    c[0] = S[0].sum()
    c[1:m] = -np.diag(S, 1)
    c[m] = S[m - 1].sum()
    return c


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n", [2, 8, 14])
def test_coarsen_is_half_the_exact_1d_elimination(axis, n):
    # Reading (the paper is silent): every coarse face gets one constant
    # multiple (1/2) of the conductance that exact elimination of the fine
    # points between coarse points gives on a line.  A planted factor on
    # one face, e.g. the first, breaks the constant ratio.
    ext = [2, 2, 2]
    ext[axis] = n
    shape = (ext[2], ext[1], ext[0])
    pr = _problem(shape, seed=40 + n + axis)
    kc = oracle.var7_coarsen(pr["kx"], pr["ky"], pr["kz"])[axis]
    # the fine line through the coincident points (2J, 2K) = (0, 0) and the
    # coarse faces on it
    if axis == 0:
        line, cline = pr["kx"][0, 0, :], kc[0, 0, :]
    elif axis == 1:
        line, cline = pr["ky"][0, :, 0], kc[0, :, 0]
    else:
        line, cline = pr["kz"][:, 0, 0], kc[:, 0, 0]
    exact = _schur_conductances(line)
    if n == 2:
        # one coarse point: its two faces together against the total
        assert np.isclose(cline.sum() / exact, 0.5, rtol=1e-13, atol=0)
        return
    ratio = cline / exact
    assert np.allclose(ratio, 0.5, rtol=1e-13, atol=0), ratio


def test_coarsen_unit_faces_and_spd():
    # unit faces: the first face of each axis spans one fine face (1/2), the
    # others two in series (1/2 * 1/2); the coarse operator stays SPD
    one = lambda s: np.ones(s)  # noqa: E731
    kxc, kyc, kzc = oracle.var7_coarsen(one((4, 4, 5)), one((4, 5, 4)),
                                        one((5, 4, 4)))
    assert np.all(kxc[:, :, 0] == 0.5) and np.all(kxc[:, :, 1:] == 0.25)
    assert np.all(kyc[:, 0, :] == 0.5) and np.all(kyc[:, 1:, :] == 0.25)
    assert np.all(kzc[0] == 0.5) and np.all(kzc[1:] == 0.25)
    pr = _problem((8, 6, 4), seed=3)
    c = oracle.var7_coarsen(pr["kx"], pr["ky"], pr["kz"])
    assert c[0].shape == (4, 3, 3) and c[1].shape == (4, 4, 2) and \
        c[2].shape == (5, 3, 2)
    Ac = assemble.var7(*c).toarray()
    assert np.allclose(Ac, Ac.T, atol=0)
    assert np.linalg.eigvalsh(Ac).min() > 0
    # transverse position: coarse (I, J, K) = (1, 2, 1) takes the fine row
    # (2J, 2K) = (4, 2)
    kx = pr["kx"]
    a, b = kx[2, 4, 1], kx[2, 4, 2]
    assert np.isclose(c[0][1, 2, 1], a * b / (2 * (a + b)), rtol=1e-15)


def _loss_and_grads_dense(kx, ky, kz, f, ut):
    A = assemble.var7(kx, ky, kz).toarray()
    u = np.linalg.solve(A, f.ravel())
    lam = np.linalg.solve(A.T, u - ut.ravel())
    return A, u, lam, 0.5 * np.sum((u - ut.ravel()) ** 2)


def test_face_gradient_vs_finite_differences():
    shape = (3, 3, 3)
    pr = _problem(shape, seed=55)
    kx, ky, kz, f, ut = (pr[k] for k in ("kx", "ky", "kz", "f", "u_t"))
    _, u, lam, L0 = _loss_and_grads_dense(kx, ky, kz, f, ut)
    gx, gy, gz = oracle.var7_face_grad(u.reshape(shape), lam.reshape(shape))
    h = 1e-6
    rng = np.random.default_rng(0)
    for arr, g in ((kx, gx), (ky, gy), (kz, gz)):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            ap, am = arr.copy(), arr.copy()
            ap[idx] += h
            am[idx] -= h
            ks = {"kx": kx, "ky": ky, "kz": kz}
            name = [n for n, v in ks.items() if v is arr][0]
            ks_p, ks_m = dict(ks), dict(ks)
            ks_p[name], ks_m[name] = ap, am
            Lp = _loss_and_grads_dense(ks_p["kx"], ks_p["ky"], ks_p["kz"],
                                       f, ut)[3]
            Lm = _loss_and_grads_dense(ks_m["kx"], ks_m["ky"], ks_m["kz"],
                                       f, ut)[3]
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd,
                                                                  g[idx])
    # dL/df = lambda
    i = 13
    fp, fm = f.copy(), f.copy()
    fp.ravel()[i] += h
    fm.ravel()[i] -= h
    fd = (_loss_and_grads_dense(kx, ky, kz, fp, ut)[3] -
          _loss_and_grads_dense(kx, ky, kz, fm, ut)[3]) / (2 * h)
    assert abs(fd - lam[i]) <= 1e-6 * max(1, abs(fd))


@pytest.mark.parametrize("shape", [(3, 4, 5), (6, 6, 6), (1, 1, 6)])
@pytest.mark.parametrize("direction", ["fwd", "bwd", "sym"])
def test_sweep_adjoint_vs_dense_transposed_solves(shape, direction):
    from tests.test_oracle_const27 import _dense_sweep_adjoint
    pr = _problem(shape, seed=31)
    f = (pr["kx"], pr["ky"], pr["kz"])
    A = assemble.var7(*f).toarray()
    g = inputs.standard_normal(7, shape)
    gr, gx = oracle.symgs_adjoint(g, direction, kind="var7", faces=f)
    rr, rx = _dense_sweep_adjoint(A, g.ravel(), direction)
    assert np.max(np.abs(gr.ravel() - rr)) <= 1e-13 * np.max(np.abs(rr))
    assert np.max(np.abs(gx.ravel() - rx)) <= 1e-13 * np.max(np.abs(rx))


def test_sweep_adjoint_dot_products():
    # forward sweep S(r, x) = (D+L)^{-1}(r - U x).  Its adjoint is a
    # backward sweep from zero on g, and -L applied to that for x.
    shape = (3, 4, 5)
    pr = _problem(shape)
    kx, ky, kz = pr["kx"], pr["ky"], pr["kz"]
    r = inputs.standard_normal(1, shape)
    x = inputs.standard_normal(2, shape)
    g = inputs.standard_normal(3, shape)
    s = oracle.symgs_var7(r, x, kx, ky, kz, "fwd")
    y = oracle.symgs_var7(g, np.zeros(shape), kx, ky, kz, "bwd")
    gx = -oracle.spmv_var7_part(y, kx, ky, kz, -1)
    lhs = np.dot(g.ravel(), s.ravel())
    rhs = np.dot(y.ravel(), r.ravel()) + np.dot(gx.ravel(), x.ravel())
    assert abs(lhs - rhs) <= 1e-13 * max(1, abs(lhs))
