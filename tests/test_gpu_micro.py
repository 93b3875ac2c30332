"""GPU parity of the microbenchmark kernels (Sec. 7.2.1: Jacobi iterations
of the 2-D 9-point operator, temporally blocked) and of the pentadiagonal
and 5x5 block-tridiagonal line solves (Sec. 7.1, SP- and BT-shaped),
against the oracle."""
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


# (300, 270): tiles whose whole region lies inside the grid at every fusion
# depth (the kernel's path without the boundary select) beside boundary ones
@pytest.mark.parametrize("shape", [(45, 70), (64, 64), (1, 1), (200, 130),
                                   (257, 3), (300, 270)])
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
                                   (33, 4, 70), (5, 3, 400), (300, 2, 3)])
def test_penta_lines_parity(m, axis, shape):
    # ragged and single-point lines, and long ones (400 along x, 300 along
    # z): many 16-point chunks with a ragged last one
    banner(f"penta {axis} {shape}")
    coef, r = _penta(shape, 40)
    x = m.penta_lines(dev(coef), dev(r), axis)
    ref = oracle.penta_lines(coef, r, axis)
    assert rel_inf(host(x), ref) <= 1e-13


@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_penta_lines_split_variants_bitwise(m, axis, monkeypatch):
    # 1, 2 or 4 lanes per line in the chunk transfers change only which
    # lane moves which value: every variant gives the same bits
    shape = (19, 37, 45)
    banner(f"penta {axis} transfer splits")
    coef, r = _penta(shape, 44)
    outs = []
    for split in ("1", "2", "4"):
        monkeypatch.setenv("M2S_PL_SPLIT", split)
        outs.append(host(m.penta_lines(dev(coef), dev(r), axis)))
    assert rel_inf(outs[0], oracle.penta_lines(coef, r, axis)) <= 1e-13
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


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


@pytest.mark.parametrize("axis", ["x", "y", "z"])
@pytest.mark.parametrize("shape", [(5, 7, 9), (1, 1, 1), (1, 1, 70),
                                   (70, 1, 1), (3, 65, 2), (2, 3, 130)])
def test_bt_lines_parity(m, axis, shape):
    banner(f"bt lines {axis} {shape}")
    coef, r = inputs.bt_problem(63, shape)
    x = m.bt_lines(dev(coef), dev(r), axis)
    assert rel_inf(host(x), oracle.bt_lines(coef, r, axis)) <= 1e-13


def test_bt_lines_full_size_162(m):
    # the BT-shaped workload the benchmark times: every line of 162^3 along
    # each axis against the oracle
    shape = (162, 162, 162)
    banner("bt lines 162^3")
    coef, r = inputs.bt_problem(70, shape)
    cg, rg = dev(coef), dev(r)
    work = torch.empty(shape + (5, 5), dtype=torch.float64, device="cuda")
    for axis in ("x", "y", "z"):
        x = m.bt_lines(cg, rg, axis, work=work)
        assert rel_inf(host(x), oracle.bt_lines(coef, r, axis)) <= 1e-13


def test_bt_lines_rejects_bad_arguments(m):
    coef = torch.zeros((3, 4, 4, 4, 5, 5), dtype=torch.float64,
                       device="cuda")
    r = torch.zeros((4, 4, 4, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="M2S_ERR_ALIAS"):
        m.bt_lines(coef, r, "x", x=r)
    with pytest.raises(ValueError):
        m.bt_lines(coef[:, :3], r, "x")
    with pytest.raises(ValueError, match="axis"):
        m.bt_lines(coef, r, "w")


@pytest.mark.parametrize("shape", [(9, 7, 6), (16, 16, 16), (13, 26, 9),
                                   (33, 20, 17), (1, 1, 5)])
@pytest.mark.parametrize("nw", ["1", "2"])
def test_dilu27_factor_and_apply(m, shape, nw, monkeypatch):
    banner(f"dilu27 {shape} nw {nw}")
    monkeypatch.setenv("M2S_C27_WAVES", nw)
    A = m.const27(shape)
    ws = m.Workspace(A)
    w = m.dilu27_factor(A, ws)
    d = oracle.dilu27_factor(shape)
    assert rel_inf(host(w), 1.0 / d) <= 1e-13
    r = inputs.standard_normal(50, shape)
    z = m.dilu27_apply(A, w, dev(r), ws=ws)
    assert rel_inf(host(z), oracle.dilu27_solve(d, r)) <= 1e-13


def test_dilu27_full_size_256(m):
    shape = (256, 256, 256)
    banner("dilu27 256^3")
    A = m.const27(shape)
    ws = m.Workspace(A)
    w = m.dilu27_factor(A, ws)
    d = oracle.dilu27_factor(shape)
    assert rel_inf(host(w), 1.0 / d) <= 1e-13
    r = inputs.standard_normal(51, shape)
    z = m.dilu27_apply(A, w, dev(r), ws=ws)
    assert rel_inf(host(z), oracle.dilu27_solve(d, r)) <= 1e-13


def test_dilu27_rejects_tall_tiles_and_f32(m, monkeypatch):
    monkeypatch.setenv("M2S_C27_WAVES", "4")
    A = m.const27((8, 8, 8))
    ws = m.Workspace(A)
    with pytest.raises(RuntimeError):
        m.dilu27_factor(A, ws)
    # a rejected call leaves the workspace usable
    rh = inputs.standard_normal(53, (8, 8, 8))
    x = dev(np.zeros((8, 8, 8)))
    m.symgs(A, dev(rh), x, "sym", ws)
    ref = oracle.symgs27(rh, np.zeros((8, 8, 8)), "sym")
    assert rel_inf(host(x), ref) <= 1e-13
    monkeypatch.setenv("M2S_C27_WAVES", "2")
    A32 = m.const27((8, 8, 8), dtype=torch.float32)
    with pytest.raises(RuntimeError):
        m.dilu27_factor(A32)


@pytest.mark.parametrize("shape", [(9, 7, 6), (16, 16, 16), (13, 26, 9),
                                   (1, 1, 5), (2, 2, 2), (5, 1, 7)])
def test_ilu0_factor_and_apply(m, shape):
    # ILU(0) (Sec. 7.2.1 / Sec. 9): the factor against the oracle's, entry by
    # entry, and the solve z = (L U)^{-1} r
    banner(f"ilu0 {shape}")
    A = m.const27(shape)
    Lg, Ug = m.ilu0_factor(A)
    Lo, Uo = oracle.ilu0_27_factor(shape)
    assert rel_inf(host(Lg), Lo) <= 1e-13
    assert rel_inf(host(Ug), Uo) <= 1e-13
    r = inputs.standard_normal(54, shape)
    z = m.ilu0_apply(A, Lg, Ug, dev(r))
    assert rel_inf(host(z), oracle.ilu0_27_solve(Lo, Uo, r)) <= 1e-13


def test_ilu0_full_size_256(m):
    shape = (256, 256, 256)
    banner("ilu0 256^3")
    A = m.const27(shape)
    Lg, Ug = m.ilu0_factor(A)
    Lo, Uo = oracle.ilu0_27_factor(shape)
    assert rel_inf(host(Lg), Lo) <= 1e-13
    assert rel_inf(host(Ug), Uo) <= 1e-13
    r = inputs.standard_normal(55, shape)
    z = m.ilu0_apply(A, Lg, Ug, dev(r))
    assert rel_inf(host(z), oracle.ilu0_27_solve(Lo, Uo, r)) <= 1e-13


def test_ilu0_rejects_other_kinds_and_aliasing(m):
    A32 = m.const27((4, 4, 4), dtype=torch.float32)
    with pytest.raises((RuntimeError, TypeError)):
        m.ilu0_factor(A32)
    A = m.const27((4, 4, 4))
    Lg, Ug = m.ilu0_factor(A)
    r = dev(np.ones((4, 4, 4)))
    with pytest.raises(RuntimeError, match="M2S_ERR_ALIAS"):
        m.ilu0_apply(A, Lg, Ug, r, r)


# (6, 9, 1): one column, so every odd plane diagonal i + 2j is empty (the
# packings' search for a position's diagonal skips them); (7, 1, 12): one row
ILB_SHAPES = [(9, 13, 17), (20, 5, 33), (1, 1, 1), (3, 64, 10),
              (16, 16, 16), (5, 300, 7), (4, 512, 3), (11, 100, 9),
              (2, 2, 130), (6, 9, 1), (7, 1, 12)]


@pytest.mark.parametrize("shape", ILB_SHAPES)
def test_ilu0_band_apply(m, shape):
    # the band-wavefront solves (bands of 512 / ny planes, records between
    # bands) against the oracle's ILU(0) solve; twice in a row on one
    # workspace, and beside the hyperplane solves
    banner(f"ilu0 band {shape}")
    A = m.const27(shape)
    ws = m.Workspace(A)
    Lg, Ug = m.ilu0_factor(A)
    Lp, Up = m.ilu0_pack(A, Lg, Ug, ws)
    r = inputs.standard_normal(56, shape)
    z = m.ilu0_apply_packed(A, Lp, Up, dev(r), ws=ws)
    ws.check()
    Lo, Uo = oracle.ilu0_27_factor(shape)
    assert rel_inf(host(z), oracle.ilu0_27_solve(Lo, Uo, r)) <= 1e-13
    z2 = m.ilu0_apply_packed(A, Lp, Up, dev(r), ws=ws)
    ws.check()
    assert torch.equal(z, z2)
    zh = m.ilu0_apply(A, Lg, Ug, dev(r))
    assert rel_inf(host(zh), host(z)) <= 1e-13


def test_ilu0_band_full_size_256(m):
    shape = (256, 256, 256)
    banner("ilu0 band 256^3")
    A = m.const27(shape)
    ws = m.Workspace(A)
    Lg, Ug = m.ilu0_factor(A)
    Lp, Up = m.ilu0_pack(A, Lg, Ug, ws)
    del Lg, Ug
    r = inputs.standard_normal(57, shape)
    z = m.ilu0_apply_packed(A, Lp, Up, dev(r), ws=ws)
    ws.check()
    Lo, Uo = oracle.ilu0_27_factor(shape)
    assert rel_inf(host(z), oracle.ilu0_27_solve(Lo, Uo, r)) <= 1e-13


def test_ilu0_band_rejects(m):
    A = m.const27((2, 513, 3))   # ny > 512: no band kernel
    ws = m.Workspace(A)
    Lg, Ug = m.ilu0_factor(A)
    with pytest.raises(RuntimeError, match="M2S_ERR_UNSUPPORTED"):
        m.ilu0_pack(A, Lg, Ug, ws)
    B = m.const27((4, 4, 4))
    wb = m.Workspace(B)
    Lg, Ug = m.ilu0_factor(B)
    Lp, Up = m.ilu0_pack(B, Lg, Ug, wb)
    r = dev(np.ones((4, 4, 4)))
    with pytest.raises(RuntimeError, match="M2S_ERR_ALIAS"):
        m.ilu0_apply_packed(B, Lp, Up, r, r, ws=wb)
