"""CPU oracle for the Mat2Stencil hot path -- TEST INFRASTRUCTURE ONLY.

Thin numpy/ctypes front end over libm2s_oracle.so (plain single-threaded C,
built from m2s_oracle.c with -O2 -ffp-contract=off).  Only tests/, the smoke
check and the benchmark's CPU-baseline leg import this package; the HIP
library and its Python binding never do, and the two share no code.

Array conventions: scalar fields are numpy arrays of shape (nz, ny, nx)
(x fastest); BLOCK7 fields are (nz, ny, nx, 5); VAR7 face arrays are
kx (nz, ny, nx+1), ky (nz, ny+1, nx), kz (nz+1, ny, nx); BLOCK7 blocks are
(7, 5, 5) in the order centre, -x, +x, -y, +y, -z, +z.  Functions never
modify their inputs; "in-place" sweeps work on a copy that is returned.

Each wrapped routine cites the part of the paper it follows in the C source.

Every routine is pinned by a CPU test against something other than itself
(assembled sparse matrices, dense triangular solves, closed forms, exact
1-D elimination, finite differences); see the tests named test_oracle_*.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# M2S_ORACLE_LIB selects another build of the same source (e.g. one made
# with -fsanitize=address,undefined to check the oracle itself)
_LIBPATH = os.environ.get("M2S_ORACLE_LIB") or os.path.join(
    _HERE, "libm2s_oracle.so")
_lib = None

PC_NONE, PC_SYMGS, PC_MG, PC_MG_F32 = 0, 1, 2, 3

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b  # noqa: F401  (oracle/build.py)
        _b.build()
    lib = C.CDLL(_LIBPATH)
    i, d, f = C.c_int, C.c_double, C.c_float
    for sfx, P, R in (("_f64", _dp, d), ("_f32", _fp, f)):
        g = lambda n: getattr(lib, "m2so_" + n + sfx)  # noqa: E731
        g("spmv27").argtypes = [i, i, i, R, R, P, P]
        g("symgs27_fwd").argtypes = [i, i, i, R, R, P, P]
        g("symgs27_bwd").argtypes = [i, i, i, R, R, P, P]
        g("spmv27_part").argtypes = [i, i, i, R, i, P, P]
        g("spmv_var7").argtypes = [i, i, i, P, P, P, P, P]
        g("spmv_var7_part").argtypes = [i, i, i, P, P, P, i, P, P]
        g("symgs_var7_fwd").argtypes = [i, i, i, P, P, P, P, P]
        g("symgs_var7_bwd").argtypes = [i, i, i, P, P, P, P, P]
        g("var7_coarsen").argtypes = [i, i, i, P, P, P, P, P, P]
        g("var7_face_grad").argtypes = [i, i, i, P, P, P, P, P]
        g("spmv_block7").argtypes = [i, i, i, P, P, P]
        g("ssor_block7_fwd").argtypes = [i, i, i, P, R, P, P]
        g("ssor_block7_bwd").argtypes = [i, i, i, P, R, P, P]
        g("ssor_block7_fwd").restype = i
        g("ssor_block7_bwd").restype = i
        g("restrict_inject").argtypes = [i, i, i, P, P, P]
        g("prolong_inject").argtypes = [i, i, i, P, P]
        g("mg_create").restype = C.c_void_p
        g("mg_create").argtypes = [i, i, i, i, i, R, R, C.c_void_p,
                                   C.c_void_p, C.c_void_p]
        g("mg_destroy").argtypes = [C.c_void_p]
        g("mg_vcycle").argtypes = [C.c_void_p, P, P]
        g("mg_faces").restype = C.c_void_p
        g("mg_faces").argtypes = [C.c_void_p, i, i]
        g("lu5_factor").argtypes = [P, P, np.ctypeslib.ndpointer(
            dtype=np.int32, flags="C_CONTIGUOUS")]
        g("lu5_factor").restype = i
        g("jacobi9").argtypes = [i, i, R, R, P, P, i, P]
        g("dilu27_factor").argtypes = [i, i, i, R, R, P]
        g("dilu27_solve").argtypes = [i, i, i, R, P, P, P]
        g("ilu0_27_factor").argtypes = [i, i, i, R, R, P, P]
        g("ilu0_27_factor").restype = i
        g("ilu0_27_solve").argtypes = [i, i, i, P, P, P, P]
        g("penta_lines").argtypes = [i, i, i, i, P, P, P]
        g("bt_lines").argtypes = [i, i, i, i, P, P, P]
        g("bt_lines").restype = i
    lib.m2so_pcg.restype = i
    lib.m2so_pcg.argtypes = [i, i, i, i, d, d, C.c_void_p, C.c_void_p,
                             C.c_void_p, i, i, _dp, _dp, i, d, i,
                             C.POINTER(i), C.POINTER(d), C.POINTER(d),
                             C.c_void_p]
    _lib = lib
    return lib


def _sfx(dtype):
    if dtype == np.float64:
        return "_f64"
    if dtype == np.float32:
        return "_f32"
    raise TypeError(f"oracle supports float64/float32, got {dtype}")


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _fn(name, dtype):
    return getattr(_load(), "m2so_" + name + _sfx(np.dtype(dtype)))


# ---------------------------------------------------------------- CONST27
def spmv27(x, diag=26.0, off=-1.0, dtype=np.float64):
    """y = A x for the constant 27-point operator (Dirichlet truncation)."""
    x = _c(x, dtype)
    nz, ny, nx = x.shape
    y = np.empty_like(x)
    _fn("spmv27", dtype)(nx, ny, nz, diag, off, x, y)
    return y


def spmv27_part(x, part, off=-1.0, dtype=np.float64):
    """Strict lower (part=-1) or upper (part=+1) triangle of CONST27 times x."""
    x = _c(x, dtype)
    nz, ny, nx = x.shape
    y = np.empty_like(x)
    _fn("spmv27_part", dtype)(nx, ny, nz, off, int(part), x, y)
    return y


def symgs27(r, x, direction="sym", diag=26.0, off=-1.0, dtype=np.float64):
    """Lexicographic Gauss-Seidel sweep(s) on CONST27.

    direction: "fwd" (p ascending), "bwd" (p descending) or "sym" (fwd then
    bwd, one symmetric Gauss-Seidel).  Returns the updated copy of x."""
    r = _c(r, dtype)
    x = np.array(x, dtype=dtype, copy=True, order="C")
    nz, ny, nx = r.shape
    if direction in ("fwd", "sym"):
        _fn("symgs27_fwd", dtype)(nx, ny, nz, diag, off, r, x)
    if direction in ("bwd", "sym"):
        _fn("symgs27_bwd", dtype)(nx, ny, nz, diag, off, r, x)
    if direction not in ("fwd", "bwd", "sym"):
        raise ValueError(direction)
    return x


# ---------------------------------------------------------------- VAR7
def spmv_var7(x, kx, ky, kz, dtype=np.float64):
    x = _c(x, dtype)
    nz, ny, nx = x.shape
    y = np.empty_like(x)
    _fn("spmv_var7", dtype)(nx, ny, nz, _c(kx, dtype), _c(ky, dtype),
                            _c(kz, dtype), x, y)
    return y


def spmv_var7_part(x, kx, ky, kz, part, dtype=np.float64):
    x = _c(x, dtype)
    nz, ny, nx = x.shape
    y = np.empty_like(x)
    _fn("spmv_var7_part", dtype)(nx, ny, nz, _c(kx, dtype), _c(ky, dtype),
                                 _c(kz, dtype), int(part), x, y)
    return y


def symgs_var7(r, x, kx, ky, kz, direction="sym", dtype=np.float64):
    r = _c(r, dtype)
    x = np.array(x, dtype=dtype, copy=True, order="C")
    nz, ny, nx = r.shape
    args = (nx, ny, nz, _c(kx, dtype), _c(ky, dtype), _c(kz, dtype), r, x)
    if direction in ("fwd", "sym"):
        _fn("symgs_var7_fwd", dtype)(*args)
    if direction in ("bwd", "sym"):
        _fn("symgs_var7_bwd", dtype)(*args)
    if direction not in ("fwd", "bwd", "sym"):
        raise ValueError(direction)
    return x


def var7_coarsen(kx, ky, kz, dtype=np.float64):
    kx, ky, kz = _c(kx, dtype), _c(ky, dtype), _c(kz, dtype)
    nz, ny, nx1 = kx.shape
    nx = nx1 - 1
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    kxc = np.empty((cz, cy, cx + 1), dtype)
    kyc = np.empty((cz, cy + 1, cx), dtype)
    kzc = np.empty((cz + 1, cy, cx), dtype)
    _fn("var7_coarsen", dtype)(nx, ny, nz, kx, ky, kz, kxc, kyc, kzc)
    return kxc, kyc, kzc


def var7_face_grad(u, lam, dtype=np.float64):
    """dL/dk_f = -(lam_p - lam_q)(u_p - u_q) for every face (zero ghosts)."""
    u, lam = _c(u, dtype), _c(lam, dtype)
    nz, ny, nx = u.shape
    gx = np.empty((nz, ny, nx + 1), dtype)
    gy = np.empty((nz, ny + 1, nx), dtype)
    gz = np.empty((nz + 1, ny, nx), dtype)
    _fn("var7_face_grad", dtype)(nx, ny, nz, u, lam, gx, gy, gz)
    return gx, gy, gz


# ------------------------------------------------------- sweep adjoints
def symgs_adjoint(g, direction="fwd", kind="const27", faces=None, diag=26.0,
                  off=-1.0):
    """Gradients (gr, gx) of <g, S(r, x)> for the lexicographic sweep S of a
    symmetric operator A = D + L + U (the transposed sweeps in reverse
    order).  A forward sweep is x' = (D+L)^{-1} (r - U x), so
        gr = (D+L)^{-T} g,   gx = -U^T gr;
    with A symmetric (D+L)^T = D+U and U^T = L: gr is a backward sweep of g
    from zero and gx = -L gr.  A backward sweep x' = (D+U)^{-1} (r - L x)
    likewise gives gr = forward sweep of g from zero, gx = -U gr.  The
    symmetric sweep (forward, then backward) chains the two in reverse:
    the backward sweep's gradients first, its gx fed to the forward one;
    gr is the sum of both gr's."""
    g = _c(g, np.float64)
    zero = np.zeros_like(g)
    if kind == "const27":
        sweep = lambda rhs, d: symgs27(rhs, zero, d, diag, off)  # noqa: E731
        part = lambda v, s: spmv27_part(v, s, off)  # noqa: E731
    elif kind == "var7":
        kx, ky, kz = faces
        sweep = lambda rhs, d: symgs_var7(rhs, zero, kx, ky, kz, d)  # noqa
        part = lambda v, s: spmv_var7_part(v, kx, ky, kz, s)  # noqa: E731
    else:
        raise ValueError(kind)
    if direction == "fwd":
        gr = sweep(g, "bwd")
        return gr, -part(gr, -1)
    if direction == "bwd":
        gr = sweep(g, "fwd")
        return gr, -part(gr, +1)
    if direction == "sym":
        grb, gmid = symgs_adjoint(g, "bwd", kind, faces, diag, off)
        grf, gx = symgs_adjoint(gmid, "fwd", kind, faces, diag, off)
        return grb + grf, gx
    raise ValueError(direction)


# ---------------------------------------------------------------- BLOCK7
def spmv_block7(x, blocks, dtype=np.float64):
    x = _c(x, dtype)
    nz, ny, nx, nv = x.shape
    assert nv == 5
    y = np.empty_like(x)
    _fn("spmv_block7", dtype)(nx, ny, nz, _c(blocks, dtype), x, y)
    return y


def ssor_block7(b, x, blocks, omega, direction="sym", dtype=np.float64):
    """Block SSOR half-sweeps: "fwd", "bwd" or "sym" (fwd then bwd)."""
    b = _c(b, dtype)
    x = np.array(x, dtype=dtype, copy=True, order="C")
    nz, ny, nx, nv = b.shape
    assert nv == 5
    blk = _c(blocks, dtype)
    if direction in ("fwd", "sym"):
        if _fn("ssor_block7_fwd", dtype)(nx, ny, nz, blk, omega, b, x):
            raise ZeroDivisionError("singular diagonal block")
    if direction in ("bwd", "sym"):
        if _fn("ssor_block7_bwd", dtype)(nx, ny, nz, blk, omega, b, x):
            raise ZeroDivisionError("singular diagonal block")
    if direction not in ("fwd", "bwd", "sym"):
        raise ValueError(direction)
    return x


def lu5(a, dtype=np.float64):
    lu = np.empty((5, 5), dtype)
    piv = np.empty(5, np.int32)
    if _fn("lu5_factor", dtype)(_c(a, dtype), lu, piv):
        raise ZeroDivisionError("singular block")
    return lu, piv


# ---------------------------------------------------------------- MG
def restrict_inject(r, az, dtype=np.float64):
    r, az = _c(r, dtype), _c(az, dtype)
    nz, ny, nx = r.shape
    rc = np.empty((nz // 2, ny // 2, nx // 2), dtype)
    _fn("restrict_inject", dtype)(nx, ny, nz, r, az, rc)
    return rc


def prolong_inject(zc, z, dtype=np.float64):
    z = np.array(z, dtype=dtype, copy=True, order="C")
    nz, ny, nx = z.shape
    _fn("prolong_inject", dtype)(nx, ny, nz, _c(zc, dtype), z)
    return z


class MG:
    """Multigrid hierarchy (kind "const27" or "var7"), levels >= 1."""

    def __init__(self, kind, shape, levels, diag=26.0, off=-1.0,
                 faces=None, dtype=np.float64):
        self.dtype = np.dtype(dtype)
        self.kind = {"const27": 0, "var7": 1}[kind]
        nz, ny, nx = shape
        self.shape = (nz, ny, nx)
        self._keep = None
        ptrs = (None, None, None)
        if self.kind == 1:
            kx, ky, kz = (_c(a, self.dtype) for a in faces)
            self._keep = (kx, ky, kz)
            ptrs = tuple(a.ctypes.data_as(C.c_void_p) for a in self._keep)
        self._h = _fn("mg_create", self.dtype)(self.kind, levels, nx, ny, nz,
                                               diag, off, *ptrs)
        if not self._h:
            raise ValueError("extents must be divisible by 2^(levels-1)")
        self.levels = levels

    def vcycle(self, r):
        r = _c(r, self.dtype)
        z = np.empty_like(r)
        _fn("mg_vcycle", self.dtype)(self._h, r, z)
        return z

    def faces(self, level):
        """Copies of the VAR7 face arrays of a level."""
        nz, ny, nx = (s >> level for s in self.shape)
        out = []
        for axis, shp in enumerate(((nz, ny, nx + 1), (nz, ny + 1, nx),
                                    (nz + 1, ny, nx))):
            p = _fn("mg_faces", self.dtype)(self._h, level, axis)
            ct = C.c_double if self.dtype == np.float64 else C.c_float
            arr = np.ctypeslib.as_array(C.cast(p, C.POINTER(ct)),
                                        shape=shp).copy()
            out.append(arr)
        return tuple(out)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _fn("mg_destroy", self.dtype)(h)
            self._h = None


# ---------------------------------------------------------------- PCG
# ------------------------------------------- microbenchmarks, Sec. 7.2.1
def jacobi9(b, x0, iters, diag=8.0, off=-1.0, dtype=np.float64):
    """iters Jacobi iterations of the 2-D 9-point operator (diag on the
    diagonal, off on the 8 neighbours, Dirichlet) on b, x0 of shape (ny, nx);
    returns x_iters."""
    b = _c(b, dtype)
    x = _c(x0, dtype).copy()
    ny, nx = b.shape
    _fn("jacobi9", dtype)(nx, ny, diag, off, b, x, int(iters), np.empty_like(x))
    return x


def dilu27_factor(shape, diag=26.0, off=-1.0, dtype=np.float64):
    """Factor diagonal d of the 27-point ILU M = (D + L) D^{-1} (D + U)."""
    nz, ny, nx = shape
    d = np.empty(shape, dtype=dtype)
    _fn("dilu27_factor", dtype)(nx, ny, nz, diag, off, d)
    return d


def dilu27_solve(d, r, off=-1.0, dtype=np.float64):
    """z = M^{-1} r (lower solve p ascending, then upper solve p descending)."""
    d, r = _c(d, dtype), _c(r, dtype)
    nz, ny, nx = r.shape
    z = np.empty_like(r)
    _fn("dilu27_solve", dtype)(nx, ny, nz, off, d, r, z)
    return z


def ilu0_27_factor(shape, diag=26.0, off=-1.0, dtype=np.float64):
    """ILU(0) of the 27-point operator: (L, U) with L of shape shape + (13,)
    (the lower offsets' l_pq, unit diagonal implied) and U of shape
    shape + (14,) (the pivot u_pp, then the upper offsets' u_pq), offsets in
    lexicographic (dk, dj, di) order, 0 outside the grid."""
    nz, ny, nx = shape
    Lf = np.zeros(shape + (13,), dtype=dtype)
    Uf = np.zeros(shape + (14,), dtype=dtype)
    if _fn("ilu0_27_factor", dtype)(nx, ny, nz, diag, off, Lf, Uf) != 0:
        raise ZeroDivisionError("ILU(0): zero pivot")
    return Lf, Uf


def ilu0_27_solve(Lf, Uf, r, dtype=np.float64):
    """z = (L U)^{-1} r: lower solve p ascending, upper solve p
    descending."""
    Lf, Uf, r = _c(Lf, dtype), _c(Uf, dtype), _c(r, dtype)
    nz, ny, nx = r.shape
    z = np.empty_like(r)
    _fn("ilu0_27_solve", dtype)(nx, ny, nz, Lf, Uf, r, z)
    return z


def penta_lines(coef, r, axis, dtype=np.float64):
    """Solve the pentadiagonal systems along every grid line of `axis`
    ("x", "y" or "z"); coef has shape (5, nz, ny, nx) = bands a..e."""
    coef, r = _c(coef, dtype), _c(r, dtype)
    nz, ny, nx = r.shape
    x = np.empty_like(r)
    _fn("penta_lines", dtype)(nx, ny, nz, {"x": 0, "y": 1, "z": 2}[axis], coef,
                              r, x)
    return x


def bt_lines(coef, r, axis, dtype=np.float64):
    """Solve the 5x5 block-tridiagonal systems along every grid line of
    `axis` ("x", "y" or "z"); coef has shape (3, nz, ny, nx, 5, 5) = the
    blocks A (coupling to the previous point), B, C (to the next point);
    r has shape (nz, ny, nx, 5)."""
    coef, r = _c(coef, dtype), _c(r, dtype)
    nz, ny, nx = r.shape[:3]
    if r.shape[3:] != (5,) or coef.shape != (3, nz, ny, nx, 5, 5):
        raise ValueError("bt_lines: coef (3, nz, ny, nx, 5, 5), r (nz, ny, nx, 5)")
    x = np.empty_like(r)
    st = _fn("bt_lines", dtype)(nx, ny, nz, {"x": 0, "y": 1, "z": 2}[axis],
                                coef, r, x)
    if st != 0:
        raise ValueError("bt_lines: a pivot block is singular")
    return x


def pcg(b, x0=None, kind="const27", precond="mg", levels=4, faces=None,
        diag=26.0, off=-1.0, max_iter=50, tol=0.0, replace_every=0):
    """HPCG-form preconditioned CG in double.

    precond: "none", "symgs", "mg" or "mg_f32" (V-cycle in float).
    Returns dict(x, status, iters, relres, true_relres, hist)."""
    lib = _load()
    b = _c(b, np.float64)
    nz, ny, nx = b.shape
    x = (np.zeros_like(b) if x0 is None
         else np.array(x0, dtype=np.float64, copy=True, order="C"))
    pc = {"none": PC_NONE, "symgs": PC_SYMGS, "mg": PC_MG,
          "mg_f32": PC_MG_F32}[precond]
    k = {"const27": 0, "var7": 1}[kind]
    keep = None
    ptrs = (None, None, None)
    if k == 1:
        keep = tuple(_c(a, np.float64) for a in faces)
        ptrs = tuple(a.ctypes.data_as(C.c_void_p) for a in keep)
    it, rr, tr = C.c_int(), C.c_double(), C.c_double()
    hist = np.zeros(max_iter + 1)
    st = lib.m2so_pcg(k, nx, ny, nz, diag, off, *ptrs, pc, levels, b, x,
                      max_iter, tol, replace_every, C.byref(it), C.byref(rr),
                      C.byref(tr), hist.ctypes.data_as(C.c_void_p))
    del keep
    if st < 0:
        raise ValueError("bad PCG arguments")
    return dict(x=x, status=st, iters=it.value, relres=rr.value,
                true_relres=tr.value, hist=hist[: it.value + 1])
