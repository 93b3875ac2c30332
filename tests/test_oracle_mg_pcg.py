"""Pins of the oracle's multigrid V-cycle and HPCG-form PCG (Sec. 7.1):
linearity, symmetry and positivity of the V-cycle, injection transfer
operators as transposes, convergence to the known solution x = 1, and
agreement with scipy's CG driven by the same preconditioner."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from tests import assemble
from paper_2204_13304_amd import inputs


def test_injection_transfer_are_transposes():
    fine = (8, 6, 4)
    r = inputs.standard_normal(1, fine)
    zc = inputs.standard_normal(2, (4, 3, 2))
    rc = oracle.restrict_inject(r, np.zeros(fine))
    pz = oracle.prolong_inject(zc, np.zeros(fine))
    assert np.isclose(np.dot(rc.ravel(), zc.ravel()),
                      np.dot(r.ravel(), pz.ravel()), rtol=1e-14)
    assert np.array_equal(rc, r[::2, ::2, ::2])


@pytest.mark.parametrize("kind", ["const27", "var7"])
def test_vcycle_linear_symmetric_positive(kind):
    shape = (8, 8, 8)
    faces = None
    if kind == "var7":
        pr = inputs.var7_problem(7, shape)
        faces = (pr["kx"], pr["ky"], pr["kz"])
    mg = oracle.MG(kind, shape, 3, faces=faces)
    x = inputs.standard_normal(3, shape)
    y = inputs.standard_normal(4, shape)
    Bx, By = mg.vcycle(x), mg.vcycle(y)
    Bxy = mg.vcycle(2 * x - 3 * y)
    assert np.max(np.abs(Bxy - (2 * Bx - 3 * By))) <= 1e-13 * np.max(
        np.abs(Bxy))
    a, b = np.dot(y.ravel(), Bx.ravel()), np.dot(x.ravel(), By.ravel())
    assert abs(a - b) <= 1e-13 * max(abs(a), 1e-300)
    assert np.dot(x.ravel(), Bx.ravel()) > 0


def test_single_level_is_one_symgs_from_zero():
    shape = (6, 5, 4)
    r = inputs.standard_normal(5, shape)
    z = oracle.MG("const27", shape, 1).vcycle(r)
    assert np.array_equal(z, oracle.symgs27(r, np.zeros(shape), "sym"))


def test_vcycle_two_levels_by_hand():
    # z = S(r); z += P S_c(R (r - A z)); z = SymGS(r, z)
    shape = (4, 4, 4)
    r = inputs.standard_normal(6, shape)
    z = oracle.symgs27(r, np.zeros(shape), "sym")
    rc = (r - oracle.spmv27(z))[::2, ::2, ::2]
    zc = oracle.symgs27(rc, np.zeros(rc.shape), "sym")
    z[::2, ::2, ::2] += zc
    z = oracle.symgs27(r, z, "sym")
    zz = oracle.MG("const27", shape, 2).vcycle(r)
    assert np.max(np.abs(z - zz)) <= 1e-15 * np.max(np.abs(z))


def test_pcg_symgs_converges_to_ones_small_config():
    # 16^3, b = A*1, x0 = 0, 50 SymGS-preconditioned iterations
    shape = (16, 16, 16)
    b = oracle.spmv27(np.ones(shape))
    out = oracle.pcg(b, precond="symgs", max_iter=50, tol=0.0)
    assert out["status"] == 0 and out["iters"] == 50
    assert np.max(np.abs(out["x"] - 1)) <= 1e-12
    out9 = oracle.pcg(b, precond="symgs", max_iter=200, tol=1e-9)
    assert out9["status"] == 0 and out9["true_relres"] <= 1e-9
    assert 10 <= out9["iters"] <= 40


@pytest.mark.parametrize("precond", ["none", "symgs", "mg"])
def test_pcg_matches_scipy_cg(precond):
    shape = (8, 8, 8)
    nz, ny, nx = shape
    A = assemble.const27(nx, ny, nz)
    b = oracle.spmv27(np.ones(shape)) + inputs.rhs_perturbation(2, shape)
    if precond == "none":
        M = None
    elif precond == "symgs":
        M = spla.LinearOperator(A.shape, matvec=lambda v: oracle.symgs27(
            v.reshape(shape), np.zeros(shape), "sym").ravel())
    else:
        mg = oracle.MG("const27", shape, 3)
        M = spla.LinearOperator(A.shape, matvec=lambda v: mg.vcycle(
            v.reshape(shape)).ravel())
    tol = 1e-9
    count = [0]
    xs, info = spla.cg(A, b.ravel(), rtol=tol, atol=0.0, maxiter=500, M=M,
                       callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert info == 0
    out = oracle.pcg(b, precond=precond, levels=3, max_iter=500, tol=tol)
    assert out["status"] == 0
    assert abs(out["iters"] - count[0]) <= 1
    assert np.max(np.abs(out["x"].ravel() - xs)) <= 1e-7


def test_pcg_mg_var7_converges():
    shape = (16, 16, 16)
    pr = inputs.var7_problem(55, shape)
    faces = (pr["kx"], pr["ky"], pr["kz"])
    out = oracle.pcg(pr["f"], kind="var7", faces=faces, precond="mg",
                     levels=3, max_iter=200, tol=1e-10)
    assert out["status"] == 0 and out["true_relres"] <= 1e-10
    A = assemble.var7(*faces)
    res = pr["f"].ravel() - A @ out["x"].ravel()
    assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(pr["f"])


def test_pcg_mixed_precision_reaches_1e9():
    shape = (16, 16, 16)
    b = oracle.spmv27(np.ones(shape)) + inputs.rhs_perturbation(3, shape)
    o64 = oracle.pcg(b, precond="mg", levels=3, max_iter=200, tol=1e-9)
    o32 = oracle.pcg(b, precond="mg_f32", levels=3, max_iter=200, tol=1e-9,
                     replace_every=50)
    assert o64["status"] == 0 and o32["status"] == 0
    assert o32["true_relres"] <= 1e-9
    assert abs(o32["iters"] - o64["iters"]) <= 3
    assert np.max(np.abs(o32["x"] - o64["x"])) <= 1e-7


def test_pcg_breakdown_detection():
    shape = (4, 4, 4)
    b = np.ones(shape)
    # indefinite operator: diag -26 makes A negative definite -> p.Ap < 0
    out = oracle.pcg(b, precond="none", diag=-26.0, max_iter=10, tol=1e-9)
    assert out["status"] == 2
    bn = b.copy()
    bn[1, 1, 1] = np.nan
    assert oracle.pcg(bn, precond="none", max_iter=10, tol=1e-9)[
        "status"] == 2


def test_pcg_zero_rhs():
    out = oracle.pcg(np.zeros((4, 4, 4)), precond="symgs", max_iter=5,
                     tol=1e-9)
    assert out["status"] == 0 and out["iters"] == 0
    assert np.all(out["x"] == 0)
