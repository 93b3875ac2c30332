"""GPU parity of the VAR7 operator (SpMV, sweeps, strict parts), the sweep
adjoints (element by element against the oracle's transposed sweeps, and
the dot-product identity against the forward sweep), the face-
coefficient gradient kernel, and the autograd solve (adjoint MG-PCG +
face gradient) against finite differences and the oracle gradient, and at
the benchmark's 128^3 size by its residuals and the face-gradient identity."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_13304_amd import inputs
from tests.gpu_util import (banner, dev, host, oracle_fixture, rel_inf,
                             rel_sample, strided)

pytestmark = pytest.mark.gpu

SHAPES = [(8, 8, 8), (5, 9, 13), (16, 16, 16), (1, 3, 7)]


@pytest.fixture(scope="module")
def m():
    import paper_2204_13304_amd as pkg
    assert torch.cuda.is_available()
    return pkg


def _A(m, pr, dtype=torch.float64):
    return m.var7(*(dev(pr[k], dtype) for k in ("kx", "ky", "kz")))


@pytest.mark.parametrize("shape", SHAPES)
def test_spmv_and_parts(m, shape):
    pr = inputs.var7_problem(21, shape)
    A = _A(m, pr)
    x = inputs.standard_normal(1, shape)
    f = (pr["kx"], pr["ky"], pr["kz"])
    assert rel_inf(host(m.spmv(A, dev(x))), oracle.spmv_var7(x, *f)) <= 1e-13
    for part in (-1, 1):
        assert rel_inf(host(m.spmv_part(A, dev(x), part)),
                       oracle.spmv_var7_part(x, *f, part)) <= 1e-13


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("direction", ["fwd", "bwd", "sym"])
def test_symgs_var7(m, shape, direction):
    banner(f"var7 symgs {direction} {shape}")
    pr = inputs.var7_problem(22, shape)
    A = _A(m, pr)
    r = inputs.standard_normal(2, shape)
    x0 = inputs.standard_normal(3, shape)
    xg = dev(x0)
    m.symgs(A, dev(r), xg, direction)
    ref = oracle.symgs_var7(r, x0, pr["kx"], pr["ky"], pr["kz"], direction)
    out = host(xg)
    assert rel_inf(out, ref) <= 1e-13
    xs = dev(x0)
    m.symgs_sequential(A, dev(r), xs, direction)
    assert np.array_equal(out, host(xs))


@pytest.mark.parametrize("direction", ["fwd", "bwd"])
def test_symgs_var7_tiles_bitwise(m, direction, monkeypatch):
    """Several tiles along j and k with ragged tails, every tile height:
    parity with the oracle and bitwise equality with the sequential
    kernel."""
    shape = (21, 37, 19)
    pr = inputs.var7_problem(24, shape)
    A = _A(m, pr)
    r = inputs.standard_normal(5, shape)
    x0 = inputs.standard_normal(6, shape)
    ref = oracle.symgs_var7(r, x0, pr["kx"], pr["ky"], pr["kz"], direction)
    xs = dev(x0)
    m.symgs_sequential(A, dev(r), xs, direction)
    seq = host(xs)
    for nw in ("1", "2", "4"):
        banner(f"var7 tiles nw={nw} {direction} {shape}")
        monkeypatch.setenv("M2S_V7_WAVES", nw)
        xg = dev(x0)
        m.symgs(A, dev(r), xg, direction, m.Workspace(A))
        out = host(xg)
        assert rel_inf(out, ref) <= 1e-13
        assert np.array_equal(out, seq)


@pytest.mark.parametrize("direction", ["fwd", "bwd"])
def test_symgs_var7_many_tiles_bitwise(m, direction):
    """More tiles than workgroups (9 j-tiles x 33 k-tiles on a thin grid):
    the sweep then polls 4 steps ahead instead of 2; parity with the oracle
    and bitwise equality with the sequential kernel."""
    shape = (132, 132, 6)
    banner(f"var7 many tiles {direction} {shape}")
    pr = inputs.var7_problem(26, shape)
    A = _A(m, pr)
    r = inputs.standard_normal(7, shape)
    x0 = inputs.standard_normal(8, shape)
    ref = oracle.symgs_var7(r, x0, pr["kx"], pr["ky"], pr["kz"], direction)
    xs = dev(x0)
    m.symgs_sequential(A, dev(r), xs, direction)
    xg = dev(x0)
    m.symgs(A, dev(r), xg, direction)
    out = host(xg)
    assert m.plan_sweep(A)["nslabs"] > 256
    assert rel_inf(out, ref) <= 1e-13
    assert np.array_equal(out, host(xs))


def test_var7_float32_tiles_bitwise(m):
    shape = (19, 35, 17)
    pr = inputs.var7_problem(25, shape)
    A = _A(m, pr, torch.float32)
    r = dev(inputs.standard_normal(7, shape), torch.float32)
    x0 = dev(inputs.standard_normal(8, shape), torch.float32)
    xg, xs = x0.clone(), x0.clone()
    m.symgs(A, r, xg, "sym")
    m.symgs_sequential(A, r, xs, "sym")
    assert torch.equal(xg, xs)


def test_var7_full_size_128(m):
    """The 128^3 workload of the differentiable solve: one forward and one
    backward half-sweep, bitwise against the sequential kernel."""
    shape = (128, 128, 128)
    banner(f"var7 full size {shape}")
    pr = inputs.var7_problem(5, shape)
    A = _A(m, pr)
    r = dev(inputs.standard_normal(9, shape))
    x0 = dev(inputs.standard_normal(10, shape))
    xg, xs = x0.clone(), x0.clone()
    m.symgs(A, r, xg, "sym")
    m.symgs_sequential(A, r, xs, "sym")
    assert torch.equal(xg, xs)


def test_var7_float32(m):
    shape = (12, 10, 14)
    pr = inputs.var7_problem(23, shape)
    A = _A(m, pr, torch.float32)
    r = inputs.standard_normal(4, shape)
    xg = torch.zeros(shape, dtype=torch.float32, device="cuda")
    m.symgs(A, dev(r, torch.float32), xg, "sym")
    ref = oracle.symgs_var7(r, np.zeros(shape), pr["kx"], pr["ky"],
                            pr["kz"], "sym")
    assert rel_inf(host(xg), ref) <= 1e-5


@pytest.mark.parametrize("kind", ["const27", "var7"])
@pytest.mark.parametrize("direction", ["fwd", "bwd", "sym"])
@pytest.mark.parametrize("shape", [(9, 10, 11), (6, 40, 37), (20, 33, 5)])
def test_sweep_adjoint_parity(m, kind, direction, shape):
    # gr and gx element by element against the oracle's transposed sweeps
    # run in reverse order, on shapes spanning several tiles with ragged
    # tails (tiles of 16 rows by 4-8 planes)
    banner(f"sweep adjoint {kind} {direction} {shape}")
    if kind == "const27":
        A = m.const27(shape)
        ref = oracle.symgs_adjoint(inputs.standard_normal(17, shape),
                                   direction)
    else:
        pr = inputs.var7_problem(26, shape)
        A = _A(m, pr)
        ref = oracle.symgs_adjoint(inputs.standard_normal(17, shape),
                                   direction, kind="var7",
                                   faces=(pr["kx"], pr["ky"], pr["kz"]))
    gr, gx = m.symgs_adjoint(A, dev(inputs.standard_normal(17, shape)),
                             direction)
    assert rel_inf(host(gr), ref[0]) <= 1e-13
    assert rel_inf(host(gx), ref[1]) <= 1e-13


@pytest.mark.parametrize("kind", ["const27", "var7"])
@pytest.mark.parametrize("direction", ["fwd", "bwd", "sym"])
def test_sweep_adjoint_dot_identity(m, kind, direction):
    # <g, S(r, x)> = <gr, r> + <gx, x> for the linear map (r, x) -> S(r, x)
    shape = (9, 10, 11)
    if kind == "const27":
        A = m.const27(shape)
    else:
        A = _A(m, inputs.var7_problem(24, shape))
    r = dev(inputs.standard_normal(5, shape))
    x = dev(inputs.standard_normal(6, shape))
    g = dev(inputs.standard_normal(7, shape))
    s = x.clone()
    m.symgs(A, r, s, direction)
    gr, gx = m.symgs_adjoint(A, g, direction)
    lhs = torch.dot(g.ravel(), s.ravel()).item()
    rhs = (torch.dot(gr.ravel(), r.ravel()) +
           torch.dot(gx.ravel(), x.ravel())).item()
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_symgs_autograd_function(m):
    shape = (7, 8, 9)
    A = m.const27(shape)
    r = dev(inputs.standard_normal(8, shape)).requires_grad_(True)
    x = dev(inputs.standard_normal(9, shape)).requires_grad_(True)
    w = dev(inputs.standard_normal(10, shape))
    y = m.symgs_fn(A, r, x, "sym")
    (y * w).sum().backward()
    gr, gx = m.symgs_adjoint(A, w, "sym")
    assert torch.equal(r.grad, gr) and torch.equal(x.grad, gx)


@pytest.mark.parametrize("shape", [(16, 16, 16), (7, 9, 11)])
def test_face_grad_parity(m, shape):
    pr = inputs.var7_problem(25, shape)
    A = _A(m, pr)
    u = inputs.standard_normal(11, shape)
    lam = inputs.standard_normal(12, shape)
    g = m.face_grad(A, dev(u), dev(lam))
    ref = oracle.var7_face_grad(u, lam)
    for a, b in zip(g, ref):
        assert rel_inf(host(a), b) <= 1e-14


def _loss(m, kx, ky, kz, f, ut, levels, rtol):
    u = m.solve(kx, ky, kz, f, levels=levels, rtol=rtol, max_iter=500)
    return 0.5 * ((u - ut) ** 2).sum(), u


def test_solve_gradient_fd_and_oracle(m):
    # 16^3 instance (seed 55), solved to 1e-13 so the finite differences
    # measure the gradient, not the solver tolerance
    shape = (16, 16, 16)
    banner("autograd solve 16^3")
    pr = inputs.var7_problem(55, shape)
    kx, ky, kz = (dev(pr[k]).requires_grad_(True) for k in ("kx", "ky",
                                                            "kz"))
    f = dev(pr["f"]).requires_grad_(True)
    ut = dev(pr["u_t"])
    L, u = _loss(m, kx, ky, kz, f, ut, 3, 1e-13)
    L.backward()
    # oracle gradient: u, lambda by oracle PCG, face gradient by the oracle
    faces = (pr["kx"], pr["ky"], pr["kz"])
    uo = oracle.pcg(pr["f"], kind="var7", faces=faces, precond="mg",
                    levels=3, max_iter=500, tol=1e-13)["x"]
    lo = oracle.pcg(uo - pr["u_t"], kind="var7", faces=faces, precond="mg",
                    levels=3, max_iter=500, tol=1e-13)["x"]
    gref = oracle.var7_face_grad(uo, lo)
    for t, gr in zip((kx, ky, kz), gref):
        assert rel_inf(host(t.grad), gr) <= 1e-8
    assert rel_inf(host(f.grad), lo) <= 1e-8
    # finite differences on a few faces and right-hand-side entries
    h = 1e-6
    rng = np.random.default_rng(1)
    with torch.no_grad():
        for t in (kx, ky, kz, f):
            for _ in range(3):
                idx = tuple(int(rng.integers(0, s)) for s in t.shape)
                old = t[idx].item()
                t[idx] = old + h
                Lp, _ = _loss(m, kx, ky, kz, f, ut, 3, 1e-13)
                t[idx] = old - h
                Lm, _ = _loss(m, kx, ky, kz, f, ut, 3, 1e-13)
                t[idx] = old
                fd = (Lp.item() - Lm.item()) / (2 * h)
                gv = t.grad[idx].item()
                assert abs(fd - gv) <= 1e-5 * max(1.0, abs(fd)), (idx, fd,
                                                                 gv)


def _var7_apply_np(u, kx, ky, kz):
    """(A u)_p = sum over the faces f of p of k_f (u_p - u_q), u = 0 outside:
    per axis the face differences of the zero-padded field, weighted, then
    differenced back onto the points (A = D^T K D)."""
    out = np.zeros_like(u)
    for ax, k in ((2, kx), (1, ky), (0, kz)):
        pad = [(0, 0)] * 3
        pad[ax] = (1, 1)
        w = k * np.diff(np.pad(u, pad), axis=ax)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        out += w[tuple(lo)] - w[tuple(hi)]
    return out


def test_solve_gradient_full_size_128(m):
    """The differentiable solve at the size the benchmark times (128^3, seed
    5, 4 levels, rtol 1e-10).  The oracle cannot run these solves at this
    size in a test, so the outputs are checked by what holds at any size:
    A u = f and A lam = u - u_t (lam = dL/df) to the solve tolerance, and
    sum_f k_f dL/dk_f = -lam.(A u), since dL/dk_f = -(D lam)_f (D u)_f face
    by face and A = D^T K D."""
    shape = (128, 128, 128)
    banner("autograd solve 128^3")
    pr = inputs.var7_problem(5, shape)
    kx, ky, kz = (dev(pr[k]).requires_grad_(True) for k in ("kx", "ky",
                                                            "kz"))
    f = dev(pr["f"]).requires_grad_(True)
    ut = dev(pr["u_t"])
    L, u = _loss(m, kx, ky, kz, f, ut, 4, 1e-10)
    L.backward()
    un, lam = host(u.detach()), host(f.grad)
    k = (pr["kx"], pr["ky"], pr["kz"])
    g = (host(kx.grad), host(ky.grad), host(kz.grad))
    Au = _var7_apply_np(un, *k)
    res_u = np.linalg.norm(Au - pr["f"]) / np.linalg.norm(pr["f"])
    du = un - pr["u_t"]
    res_l = (np.linalg.norm(_var7_apply_np(lam, *k) - du) /
             np.linalg.norm(du))
    assert res_u <= 2e-10 and res_l <= 2e-10, (res_u, res_l)
    kg = sum(float(np.sum(kk * gg)) for kk, gg in zip(k, g))
    scale = sum(float(np.sum(np.abs(kk * gg))) for kk, gg in zip(k, g))
    assert abs(kg + float(np.dot(lam.ravel(), Au.ravel()))) <= 1e-11 * scale


def test_tile_wait_timeout_is_reported_and_recovered(m, monkeypatch):
    # as for the 27-point tiles: a forced time-out is latched and reported,
    # and the workspace is usable afterwards
    shape = (16, 40, 10)
    banner("var7 forced tile wait time-out")
    pr = inputs.var7_problem(68, shape)
    A = _A(m, pr)
    ws = m.Workspace(A)
    r = inputs.standard_normal(69, shape)
    x0 = inputs.standard_normal(70, shape)
    monkeypatch.setenv("M2S_SPIN_LIMIT", "1")
    m.symgs(A, dev(r), dev(x0), "fwd", ws)
    with pytest.raises(RuntimeError, match="M2S_ERR_TIMEOUT"):
        ws.check()
    monkeypatch.delenv("M2S_SPIN_LIMIT")
    xg = dev(x0)
    m.symgs(A, dev(r), xg, "sym", ws)
    ws.check()
    ref = oracle.symgs_var7(r, x0, pr["kx"], pr["ky"], pr["kz"], "sym")
    assert rel_inf(host(xg), ref) <= 1e-13


def test_solve_128_against_oracle(m):
    """The differentiable solve's configuration at full size (128^3, seed 5,
    4 levels, rtol 1e-10) against the stored oracle run
    (oracle_c5_var7_128.json): forward and adjoint MG-PCG iteration counts
    within one, strided samples of u, lam = dL/df and dL/dk from the
    face-gradient kernel, and the first 20 residuals.  With these
    log-normal faces (contrast about e^4) the CG residual norms of two runs
    that differ only in summation order agree to 1e-13 for about 30
    iterations, then drift apart to a few per cent at the same iteration
    count (measured: up to 14 % in the late history) while the solutions
    still agree to 2e-10 -- so the later history is compared through the
    iteration count and the solutions."""
    shape = (128, 128, 128)
    fx = oracle_fixture("oracle_c5_var7_128.json")
    stride = fx["sample_stride"]
    banner("var7 128^3 solve, adjoint and gradient against the oracle")
    pr = inputs.var7_problem(5, shape)
    A = _A(m, pr)
    mg = m.MG(A, 4)
    out = {}
    for tag, rhs in (("forward", dev(pr["f"])), ("adjoint", None)):
        if tag == "adjoint":
            rhs = out["forward"] - dev(pr["u_t"])
        x, info = m.pcg_solve(A, rhs, None, "mg", mg, max_iter=500,
                              rtol=1e-10, history=True)
        ref = fx[tag]
        assert info["true_rel_res"] <= 1e-10, tag
        assert abs(info["iters"] - ref["iters"]) <= 1, (tag, info["iters"],
                                                        ref["iters"])
        h, hr = np.asarray(info["hist"][:21]), np.asarray(ref["hist"][:21])
        herr = float(np.max(np.abs(h - hr) / hr))
        print(f"[c5 {tag}] iters {info['iters']} (oracle {ref['iters']}), "
              f"first 20 residuals rel err {herr:.2e}", flush=True)
        assert herr <= 1e-9, (tag, herr)
        out[tag] = x
    u, lam = out["forward"], out["adjoint"]
    g = m.face_grad(A, u, lam)
    errs = {}
    for name, got in (("u_sample", u), ("lam_sample", lam), ("gkx_sample", g[0]),
                      ("gky_sample", g[1]), ("gkz_sample", g[2])):
        errs[name] = rel_sample(strided(host(got), stride), fx[name])
    print(f"[c5] sample rel errs {errs}", flush=True)
    for name, e in errs.items():
        assert e <= 1e-8, (name, e)


def test_vcycle_f32(m):
    """The VAR7 FP32 V-cycle (its FP64 output made by a conversion pass,
    unlike the 27-point one) against the float oracle."""
    shape = (16, 24, 32)
    banner(f"var7 vcycle f32 {shape}")
    pr = inputs.var7_problem(23, shape)
    A = _A(m, pr)
    mg = m.MG(A, 3, prec=torch.float32)
    r = inputs.standard_normal(3, shape)
    z = host(mg.vcycle(dev(r)))
    faces = tuple(pr[k] for k in ("kx", "ky", "kz"))
    ref32 = oracle.MG("var7", shape, 3, faces=faces,
                      dtype=np.float32).vcycle(r.astype(np.float32))
    ref64 = oracle.MG("var7", shape, 3, faces=faces).vcycle(r)
    assert rel_inf(z, ref32) <= 1e-4
    assert rel_inf(z, ref64) <= 1e-4
