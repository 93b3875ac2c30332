"""The C-ABI library loads and exports every symbol include/m2s.h declares;
host-only entry points behave (no GPU needed)."""
import ctypes as C

import pytest

from paper_2204_13304_amd import _lib as L


def test_library_exports_every_header_symbol():
    lib = L.load()
    names = L.header_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_version():
    lib = L.load()
    assert lib.m2s_version() >= 20000
    for s in range(10):
        assert lib.m2s_status_string(s)


def test_plan_validation_errors():
    lib = L.load()
    p = L.SweepPlanC()
    s = L.StencilC()
    s.kind, s.dtype = L.CONST27, L.F64
    s.diag, s.offdiag = 26.0, -1.0
    s.ext = L.Extent(0, 4, 4)
    assert lib.m2s_plan_sweep(C.byref(s), C.byref(p)) == 2  # SHAPE
    s.ext = L.Extent(4, 4, 4)
    s.dtype = 7
    assert lib.m2s_plan_sweep(C.byref(s), C.byref(p)) == 3  # DTYPE
    s.dtype = L.F64
    s.kind = L.VAR7  # no face arrays
    assert lib.m2s_plan_sweep(C.byref(s), C.byref(p)) == 1  # ARG
    s.kind = L.CONST27
    s.diag = 0.0
    assert lib.m2s_plan_sweep(C.byref(s), C.byref(p)) == 1
    s.diag = 26.0
    assert lib.m2s_plan_sweep(None, C.byref(p)) == 1
    assert lib.m2s_plan_sweep(C.byref(s), C.byref(p)) == 0
    assert p.lag_row == 2 and p.lag_plane == 4
    s.ext = L.Extent(64, 2048, 4)
    assert lib.m2s_plan_sweep(C.byref(s), C.byref(p)) == 0
    # the tiled 27-point sweep addresses a vector with 32-bit byte offsets
    s.ext = L.Extent(1024, 1024, 256)
    assert lib.m2s_plan_sweep(C.byref(s), C.byref(p)) == 2


@pytest.mark.parametrize("n", [16, 104, 256])
def test_plan_shapes(n):
    import paper_2204_13304_amd as m
    p = m.plan_sweep(m.const27((n, n, n)))
    # 27 points: tiles of 16 rows u = j + k by 4 planes per wavefront,
    # one lane per row
    assert p["row_slots"] == 16
    assert p["slab_planes"] % 4 == 0
    # nw = slab_planes / 4 compute, nw memory and 1 poll wavefronts
    assert p["threads"] == 64 * (2 * (p["slab_planes"] // 4) + 1)
    assert p["nslabs"] == len(c27_tiles((n, n, n), p["slab_planes"]))


def c27_tiles(shape, kt):
    """(u-tile, k-tile) pairs holding a grid row (j = u - k), in
    lexicographic (k-tile, u-tile) order."""
    nz, ny, nx = shape
    out = []
    for vt in range(-(-nz // kt)):
        for ut in range(0, (ny + nz) // 16 + 2):
            rows = [(u, k) for u in range(16 * ut, 16 * ut + 16)
                    for k in range(kt * vt, min(kt * vt + kt, nz))
                    if 0 <= u - k < ny]
            if rows:
                out.append((ut, vt))
    return out


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # no CPU fallback: without libm2s.so every entry point raises
    import torch

    import paper_2204_13304_amd as m
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIBPATH", str(tmp_path / "libm2s.so"))
    with pytest.raises(RuntimeError, match="libm2s.so not found"):
        L.load()
    A = m.const27((4, 4, 4))
    x = torch.zeros((4, 4, 4), dtype=torch.float64)
    for call in (lambda: m.spmv(A, x), lambda: m.symgs(A, x, x.clone()),
                 lambda: m.pcg_solve(A, x),
                 lambda: m.jacobi9(x[0], x[1].clone(), 1)):
        with pytest.raises(RuntimeError, match="libm2s.so not found"):
            call()


def test_cpu_tensors_are_rejected():
    # the library takes device memory only; host tensors never reach it
    import torch

    import paper_2204_13304_amd as m
    A = m.const27((4, 4, 4))
    x = torch.zeros((4, 4, 4), dtype=torch.float64)
    with pytest.raises(ValueError, match="must be on the GPU"):
        m.spmv(A, x)


def test_line_solves_reject_a_bad_axis():
    import torch

    import paper_2204_13304_amd as m
    r = torch.zeros((2, 2, 2, 5), dtype=torch.float64)
    coef = torch.zeros((3, 2, 2, 2, 5, 5), dtype=torch.float64)
    with pytest.raises(ValueError, match="axis"):
        m.bt_lines(coef, r, "w")
    with pytest.raises(ValueError, match="axis"):
        m.penta_lines(torch.zeros((5, 2, 2, 2), dtype=torch.float64),
                      r[..., 0], 3)


@pytest.mark.parametrize("fn,nc,nw", [("m2s_penta_lines", 5, 2),
                                      ("m2s_bt_lines", 75, 25)])
def test_line_solve_argument_errors(fn, nc, nw):
    """Validation happens on the host before anything is launched, so the
    error paths run without a GPU; overlap checks are pointer arithmetic
    (the addresses below are never dereferenced).  Every call here must
    fail validation: one that passed would launch on these fake addresses."""
    lib = L.load()
    f = getattr(lib, fn)
    nx, ny, nz = 4, 5, 6
    nb = 8 * nx * ny * nz * (5 if fn == "m2s_bt_lines" else 1)  # r, x
    cb = 8 * nx * ny * nz * nc
    wb = 8 * nx * ny * nz * nw
    base = 1 << 40
    coef, r = base, base + cb
    x, work = r + nb, r + 2 * nb
    P = C.c_void_p

    def call(nx_, ny_, nz_, axis, c, rr, xx, w):
        return f(nx_, ny_, nz_, axis, P(c), P(rr), P(xx), P(w), None)
    assert call(nx, ny, nz, 0, None, r, x, work) == 1   # ARG: null
    assert call(nx, ny, nz, 3, coef, r, x, work) == 1   # ARG: axis
    assert call(nx, ny, nz, -1, coef, r, x, work) == 1
    assert call(0, ny, nz, 0, coef, r, x, work) == 2    # SHAPE
    assert call(1 << 16, 1 << 15, 1, 0, coef, r, x, work) == 2  # n >= 2^31
    assert call(nx, ny, nz, 1, coef, r, r, work) == 4   # ALIAS: x = r
    assert call(nx, ny, nz, 1, coef, r, x, x + 8) == 4  # work overlaps x
    assert call(nx, ny, nz, 2, coef, coef + cb - 8, x, work) == 4  # r in coef
    assert call(nx, ny, nz, 2, coef, r, x, coef + cb - wb // 2) == 4


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: --gpus N > 1 exits with a message instead of a number
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "bench.py", "--gpus", "2"],
                         cwd=root, capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_pcg_workspace_argument_errors():
    """m2s_pcg_workspace_create and m2s_pcg_solve_ws validate on the host
    before anything is allocated or launched (no GPU needed)."""
    lib = L.load()
    s = L.StencilC()
    s.kind, s.dtype = L.CONST27, L.F64
    s.ext = L.Extent(8, 8, 8)
    s.diag, s.offdiag = 26.0, -1.0
    h = C.c_void_p()
    assert lib.m2s_pcg_workspace_create(C.byref(s), None) == 1      # ARG
    assert lib.m2s_pcg_workspace_create(None, C.byref(h)) == 1
    s.dtype = L.F32
    assert lib.m2s_pcg_workspace_create(C.byref(s), C.byref(h)) == 3  # DTYPE
    s.dtype = L.F64
    opts = L.PcgOpts(1, 0.0, 0, 1)
    info = L.PcgInfo()
    P = C.c_void_p
    b, x = P(1 << 40), P((1 << 40) + 8 * 512)
    # no workspace
    assert lib.m2s_pcg_solve_ws(C.byref(s), L.PC_NONE, None, b, x,
                                C.byref(opts), C.byref(info), None, None,
                                None) == 1
    lib.m2s_pcg_workspace_destroy(None)   # a null workspace is ignored


def test_profile_summary_lists_one_iteration(tmp_path):
    # a synthetic trace database: two iterations of three kernels each
    import sqlite3
    from paper_2204_13304_amd import profile_summary as ps
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, grid_x int, start int, "
                "\"end\" int, duration int)")
    t = 0
    for it in range(2):
        for name, dur in (("sweep", 500_000 + it), ("dot_kernel", 40_000),
                          ("update_xr_kernel", 130_000)):
            con.execute("insert into kernels values (?, ?, ?, ?, ?)",
                        (name, 64, t, t + dur, dur))
            t += dur
    con.commit()
    con.close()
    out = ps.iteration_table(str(db), "update_xr_kernel", 2)
    lines = out.splitlines()
    assert "iteration 2 of 2" in lines[0] and "sum 670.0 us" in lines[0]
    assert [ln.split(" | ")[0] for ln in lines[2:]] == [
        "sweep", "dot_kernel", "update_xr_kernel"]
    assert lines[2].endswith("| 500.0")
    assert "no iteration 3" in ps.iteration_table(str(db),
                                                  "update_xr_kernel", 3)
