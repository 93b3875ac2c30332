"""Torch-facing binding of libm2s.so.

Every function marshals torch tensors (device memory, current HIP stream)
into the C ABI of include/m2s.h; every arithmetic step runs in the HIP
kernels.  Tensors must be contiguous, on the GPU and of the stencil's dtype;
otherwise TypeError / ValueError is raised before anything is launched.

Fields are shaped (nz, ny, nx) (x fastest), BLOCK7 fields (nz, ny, nx, 5);
VAR7 face arrays kx (nz, ny, nx+1), ky (nz, ny+1, nx), kz (nz+1, ny, nx).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

_DT = {torch.float64: L.F64, torch.float32: L.F32}
_DIRS = {"fwd": L.FWD, "bwd": L.BWD, "sym": L.SYM}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(None)


def _need(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got "
                         f"{tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Stencil:
    """Matrix-free operator descriptor (m2s_stencil)."""

    def __init__(self, kind, shape, dtype=torch.float64, diag=26.0, off=-1.0,
                 faces=None, blocks=None):
        self.kind = kind
        self.shape = tuple(int(s) for s in shape)
        self.dtype = dtype
        if dtype not in _DT:
            raise TypeError("dtype must be torch.float64 or torch.float32")
        self.diag, self.off = float(diag), float(off)
        self.faces = faces
        self.blocks = None
        nz, ny, nx = self.shape
        if kind == L.VAR7:
            kx, ky, kz = faces
            _need(kx, dtype, (nz, ny, nx + 1), "kx")
            _need(ky, dtype, (nz, ny + 1, nx), "ky")
            _need(kz, dtype, (nz + 1, ny, nx), "kz")
        if kind == L.BLOCK7_5:
            if dtype != torch.float64:
                raise TypeError("BLOCK7 is float64 only")
            b = np.ascontiguousarray(np.asarray(blocks, dtype=np.float64))
            if b.shape != (7, 5, 5):
                raise ValueError("blocks must have shape (7, 5, 5)")
            self.blocks = b
        self._c = self._make_c()

    def _make_c(self):
        nz, ny, nx = self.shape
        s = L.StencilC()
        s.kind = self.kind
        s.dtype = _DT[self.dtype]
        s.ext = L.Extent(nx, ny, nz)
        s.diag, s.offdiag = self.diag, self.off
        if self.kind == L.VAR7:
            s.kx, s.ky, s.kz = (t.data_ptr() for t in self.faces)
        if self.kind == L.BLOCK7_5:
            s.blocks = self.blocks.ctypes.data
        return s

    @property
    def field_shape(self):
        return self.shape + ((5,) if self.kind == L.BLOCK7_5 else ())

    def ref(self):
        return C.byref(self._c)

    def with_dtype(self, dtype):
        faces = None
        if self.kind == L.VAR7:
            faces = tuple(f.to(dtype).contiguous() for f in self.faces)
        return Stencil(self.kind, self.shape, dtype, self.diag, self.off,
                       faces, self.blocks)


def const27(shape, dtype=torch.float64, diag=26.0, off=-1.0):
    return Stencil(L.CONST27, shape, dtype, diag, off)


def var7(kx, ky, kz):
    nz, ny, nx1 = kx.shape
    return Stencil(L.VAR7, (nz, ny, nx1 - 1), kx.dtype,
                   faces=(kx.contiguous(), ky.contiguous(), kz.contiguous()))


def block7(shape, blocks):
    return Stencil(L.BLOCK7_5, shape, torch.float64, blocks=blocks)


class Workspace:
    def __init__(self, A: Stencil):
        lib = L.load()
        self.A = A
        h = C.c_void_p()
        L.check(lib.m2s_workspace_create(A.ref(), C.byref(h)),
                "m2s_workspace_create")
        self._h = h
        # bound now: module globals may already be gone when the object is
        # collected at interpreter exit
        self._destroy = lib.m2s_workspace_destroy

    @property
    def handle(self):
        return self._h

    def check(self):
        L.check(L.load().m2s_check(self._h, _stream()), "m2s_check")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None


def spmv(A: Stencil, x, y=None):
    lib = L.load()
    _need(x, A.dtype, A.field_shape, "x")
    if y is None:
        y = torch.empty_like(x)
    _need(y, A.dtype, A.field_shape, "y")
    L.check(lib.m2s_spmv(A.ref(), _ptr(x), _ptr(y), _stream()), "m2s_spmv")
    return y


def spmv_part(A: Stencil, x, part, y=None):
    lib = L.load()
    _need(x, A.dtype, A.field_shape, "x")
    if y is None:
        y = torch.empty_like(x)
    L.check(lib.m2s_spmv_part(A.ref(), int(part), _ptr(x), _ptr(y),
                              _stream()), "m2s_spmv_part")
    return y


def symgs(A: Stencil, r, x, direction="sym", ws: Workspace | None = None):
    """In-place exact lexicographic Gauss-Seidel sweep(s) on x."""
    lib = L.load()
    _need(r, A.dtype, A.field_shape, "r")
    _need(x, A.dtype, A.field_shape, "x")
    ws = ws or Workspace(A)
    L.check(lib.m2s_symgs(A.ref(), _ptr(r), _ptr(x), _DIRS[direction],
                          ws.handle, _stream()), "m2s_symgs")
    return x


def symgs_oop(A: Stencil, r, x_in, x_out, direction="fwd",
              ws: Workspace | None = None):
    lib = L.load()
    _need(r, A.dtype, A.field_shape, "r")
    if x_in is not None:
        _need(x_in, A.dtype, A.field_shape, "x_in")
    _need(x_out, A.dtype, A.field_shape, "x_out")
    ws = ws or Workspace(A)
    L.check(lib.m2s_symgs_oop(A.ref(), _ptr(r), _ptr(x_in), _ptr(x_out),
                              _DIRS[direction], ws.handle, _stream()),
            "m2s_symgs_oop")
    return x_out


def symgs_sequential(A: Stencil, r, x, direction="sym"):
    lib = L.load()
    _need(r, A.dtype, A.field_shape, "r")
    _need(x, A.dtype, A.field_shape, "x")
    L.check(lib.m2s_symgs_sequential(A.ref(), _ptr(r), _ptr(x),
                                     _DIRS[direction], _stream()),
            "m2s_symgs_sequential")
    return x


def symgs_xline(A: Stencil, r, x, direction="sym",
                ws: Workspace | None = None):
    """In-place 27-point sweep(s) on x, lines scheduled at j + 2k and each
    x-line solved by an affine prefix scan (FP64; equal to the
    lexicographic sweep up to rounding)."""
    lib = L.load()
    _need(r, A.dtype, A.field_shape, "r")
    _need(x, A.dtype, A.field_shape, "x")
    ws = ws or Workspace(A)
    L.check(lib.m2s_symgs_xline(A.ref(), _ptr(r), _ptr(x), _DIRS[direction],
                                ws.handle, _stream()), "m2s_symgs_xline")
    return x


def symgs_adjoint(A: Stencil, g, direction="fwd", ws: Workspace | None = None):
    """(gr, gx): gradients of <g, sweep(r, x)> w.r.t. r and x."""
    lib = L.load()
    _need(g, A.dtype, A.field_shape, "g")
    gr, gx = torch.empty_like(g), torch.empty_like(g)
    ws = ws or Workspace(A)
    L.check(lib.m2s_symgs_adjoint(A.ref(), _ptr(g), _ptr(gr), _ptr(gx),
                                  _DIRS[direction], ws.handle, _stream()),
            "m2s_symgs_adjoint")
    return gr, gx


def ssor_sweep(A: Stencil, b, x, omega, direction="sym",
               ws: Workspace | None = None):
    lib = L.load()
    _need(b, A.dtype, A.field_shape, "b")
    _need(x, A.dtype, A.field_shape, "x")
    ws = ws or Workspace(A)
    L.check(lib.m2s_ssor_sweep(A.ref(), _ptr(b), _ptr(x), float(omega),
                               _DIRS[direction], ws.handle, _stream()),
            "m2s_ssor_sweep")
    return x


def ssor_sweep_sequential(A: Stencil, b, x, omega, direction="sym"):
    """The block SSOR sweep by one GPU thread in lexicographic order (the
    reference the wavefront kernel must match bitwise; slow)."""
    lib = L.load()
    _need(b, A.dtype, A.field_shape, "b")
    _need(x, A.dtype, A.field_shape, "x")
    L.check(lib.m2s_ssor_sweep_sequential(A.ref(), _ptr(b), _ptr(x),
                                          float(omega), _DIRS[direction],
                                          _stream()),
            "m2s_ssor_sweep_sequential")
    return x


class MG:
    """Multigrid hierarchy; prec torch.float64 or torch.float32."""

    def __init__(self, A: Stencil, levels=4, prec=torch.float64):
        lib = L.load()
        self.A = A
        h = C.c_void_p()
        L.check(lib.m2s_mg_create(A.ref(), int(levels), _DT[prec],
                                  C.byref(h)), "m2s_mg_create")
        self._h = h
        self._destroy = lib.m2s_mg_destroy
        self.levels = levels
        self.prec = prec

    @property
    def handle(self):
        return self._h

    def vcycle(self, r, z=None):
        lib = L.load()
        _need(r, torch.float64, self.A.shape, "r")
        if z is None:
            z = torch.empty_like(r)
        L.check(lib.m2s_mg_vcycle(self._h, _ptr(r), _ptr(z), _stream()),
                "m2s_mg_vcycle")
        return z

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None


class PcgWorkspace:
    """The CG vectors and scalars of one operator (m2s_pcg_workspace), made
    once so that solves with it allocate nothing."""

    def __init__(self, A: Stencil):
        lib = L.load()
        self.A = A
        h = C.c_void_p()
        L.check(lib.m2s_pcg_workspace_create(A.ref(), C.byref(h)),
                "m2s_pcg_workspace_create")
        self._h = h
        self._destroy = lib.m2s_pcg_workspace_destroy

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None


def pcg_solve(A: Stencil, b, x=None, precond="mg", mg: MG | None = None,
              max_iter=50, rtol=0.0, replace_every=0, history=False,
              raise_on_error=True, ws: PcgWorkspace | None = None,
              check_every=1):
    """HPCG-form PCG; returns (x, info dict).  With a PcgWorkspace the solve
    allocates nothing (m2s_pcg_solve_ws); without one the library allocates
    and frees the CG vectors inside the call (m2s_pcg_solve).  check_every:
    the convergence test reads the residual back every that many
    iterations."""
    lib = L.load()
    _need(b, torch.float64, A.shape, "b")
    if x is None:
        x = torch.zeros_like(b)
    _need(x, torch.float64, A.shape, "x")
    pc = {"none": L.PC_NONE, "symgs": L.PC_SYMGS, "mg": L.PC_MG}[precond]
    opts = L.PcgOpts(int(max_iter), float(rtol), int(replace_every),
                     int(check_every))
    info = L.PcgInfo()
    hist = np.zeros(max_iter + 1) if history else None
    hp = hist.ctypes.data_as(C.c_void_p) if history else None
    if ws is not None:
        st = lib.m2s_pcg_solve_ws(A.ref(), pc, mg.handle if mg else None,
                                  _ptr(b), _ptr(x), C.byref(opts),
                                  C.byref(info), hp, ws.handle, _stream())
    else:
        st = lib.m2s_pcg_solve(A.ref(), pc, mg.handle if mg else None,
                               _ptr(b), _ptr(x), C.byref(opts),
                               C.byref(info), hp, _stream())
    out = dict(status=L.STATUS.get(st, st), iters=info.iters,
               rel_res=info.rel_res, true_rel_res=info.true_rel_res,
               r0_norm=info.r0_norm, seconds=info.seconds)
    if history:
        out["hist"] = hist[: info.iters + 1]
    if raise_on_error and st not in (L.M2S_OK,):
        raise L.M2SError(st, "m2s_pcg_solve")
    return x, out


def jacobi9(b, x, iters, tblock=8, diag=8.0, off=-1.0, tmp=None):
    """iters Jacobi iterations of the 2-D 9-point operator on x (ny, nx),
    in place; tblock iterations fused per pass over memory."""
    lib = L.load()
    if b.dim() != 2:
        raise ValueError("jacobi9 takes 2-D fields (ny, nx)")
    _need(b, torch.float64, tuple(b.shape), "b")
    _need(x, torch.float64, tuple(b.shape), "x")
    if tmp is None:
        tmp = torch.empty_like(x)
    _need(tmp, torch.float64, tuple(b.shape), "tmp")
    ny, nx = b.shape
    L.check(lib.m2s_jacobi9(nx, ny, float(diag), float(off), _ptr(b), _ptr(x),
                            _ptr(tmp), int(iters), int(tblock), _stream()),
            "m2s_jacobi9")
    return x


def dilu27_factor(A: Stencil, ws: Workspace | None = None):
    """w = 1/d, the factor of the 27-point D-ILU M = (D+L) D^-1 (D+U) (the
    factored-diagonal variant; ILU(0) is ilu0_factor)."""
    lib = L.load()
    w = torch.empty(A.field_shape, dtype=A.dtype, device="cuda")
    ws = ws or Workspace(A)
    L.check(lib.m2s_dilu27_factor(A.ref(), _ptr(w), ws.handle, _stream()),
            "m2s_dilu27_factor")
    return w


def dilu27_apply(A: Stencil, w, r, z=None, ws: Workspace | None = None):
    """z = M^-1 r (lower, then upper triangular sweep)."""
    lib = L.load()
    _need(w, A.dtype, A.field_shape, "w")
    _need(r, A.dtype, A.field_shape, "r")
    if z is None:
        z = torch.empty_like(r)
    _need(z, A.dtype, A.field_shape, "z")
    ws = ws or Workspace(A)
    L.check(lib.m2s_dilu27_apply(A.ref(), _ptr(w), _ptr(r), _ptr(z),
                                ws.handle, _stream()), "m2s_dilu27_apply")
    return z


def ilu0_factor(A: Stencil):
    """ILU(0) of the 27-point operator: (L, U) with L of shape
    field_shape + (13,) (the lower offsets' l_pq) and U of shape
    field_shape + (14,) (u_pp, then the upper offsets' u_pq), offsets in
    lexicographic (dk, dj, di) order."""
    lib = L.load()
    if A.dtype != torch.float64:
        raise TypeError("ilu0_factor takes an F64 operator")
    Lf = torch.empty(A.field_shape + (13,), dtype=A.dtype, device="cuda")
    Uf = torch.empty(A.field_shape + (14,), dtype=A.dtype, device="cuda")
    L.check(lib.m2s_ilu0_factor(A.ref(), _ptr(Lf), _ptr(Uf), _stream()),
            "m2s_ilu0_factor")
    return Lf, Uf


def ilu0_apply(A: Stencil, Lf, Uf, r, z=None):
    """z = (L U)^{-1} r (lower, then upper triangular solve)."""
    lib = L.load()
    _need(Lf, A.dtype, A.field_shape + (13,), "L")
    _need(Uf, A.dtype, A.field_shape + (14,), "U")
    _need(r, A.dtype, A.field_shape, "r")
    if z is None:
        z = torch.empty_like(r)
    _need(z, A.dtype, A.field_shape, "z")
    L.check(lib.m2s_ilu0_apply(A.ref(), _ptr(Lf), _ptr(Uf), _ptr(r),
                               _ptr(z), _stream()), "m2s_ilu0_apply")
    return z


def ilu0_pack(A: Stencil, Lf, Uf, ws: Workspace | None = None):
    """The ILU(0) factor in the layout of the band-wavefront solves:
    (Lp, Up), flat device arrays of 13 n and 14 n doubles."""
    lib = L.load()
    _need(Lf, A.dtype, A.field_shape + (13,), "L")
    _need(Uf, A.dtype, A.field_shape + (14,), "U")
    ws = ws or Workspace(A)
    n = Lf.numel() // 13
    Lp = torch.empty(13 * n, dtype=Lf.dtype, device=Lf.device)
    Up = torch.empty(14 * n, dtype=Uf.dtype, device=Uf.device)
    L.check(lib.m2s_ilu0_pack(A.ref(), _ptr(Lf), _ptr(Uf), _ptr(Lp),
                              _ptr(Up), ws.handle, _stream()),
            "m2s_ilu0_pack")
    return Lp, Up


def ilu0_apply_packed(A: Stencil, Lp, Up, r, z=None,
                      ws: Workspace | None = None):
    """z = (L U)^{-1} r by the band-wavefront solves (packed factor)."""
    lib = L.load()
    n = r.numel()
    _need(Lp, A.dtype, (13 * n,), "Lp")
    _need(Up, A.dtype, (14 * n,), "Up")
    _need(r, A.dtype, A.field_shape, "r")
    if z is None:
        z = torch.empty_like(r)
    _need(z, A.dtype, A.field_shape, "z")
    ws = ws or Workspace(A)
    L.check(lib.m2s_ilu0_apply_packed(A.ref(), _ptr(Lp), _ptr(Up), _ptr(r),
                                      _ptr(z), ws.handle, _stream()),
            "m2s_ilu0_apply_packed")
    return z


_AXES = {"x": 0, "y": 1, "z": 2}


def _axis(axis):
    if axis not in _AXES:
        raise ValueError(f"axis must be 'x', 'y' or 'z', got {axis!r}")
    return _AXES[axis]


def penta_lines(coef, r, axis, x=None, work=None):
    """Solve the pentadiagonal systems along every grid line of `axis`
    ("x", "y" or "z"); coef (5, nz, ny, nx) holds the bands a..e."""
    lib = L.load()
    ax = _axis(axis)
    if r.dim() != 3:
        raise ValueError("penta_lines takes 3-D fields (nz, ny, nx)")
    nz, ny, nx = r.shape
    _need(r, torch.float64, (nz, ny, nx), "r")
    _need(coef, torch.float64, (5, nz, ny, nx), "coef")
    if x is None:
        x = torch.empty_like(r)
    if work is None:
        work = torch.empty((2, nz, ny, nx), dtype=torch.float64,
                           device=r.device)
    _need(x, torch.float64, (nz, ny, nx), "x")
    _need(work, torch.float64, (2, nz, ny, nx), "work")
    L.check(lib.m2s_penta_lines(nx, ny, nz, ax,
                                _ptr(coef), _ptr(r), _ptr(x), _ptr(work),
                                _stream()), "m2s_penta_lines")
    return x


def bt_lines(coef, r, axis, x=None, work=None):
    """Solve the 5x5 block-tridiagonal systems along every grid line of
    `axis` ("x", "y" or "z"); coef (3, nz, ny, nx, 5, 5) holds the blocks
    A, B, C of every point, r and x are (nz, ny, nx, 5)."""
    lib = L.load()
    ax = _axis(axis)
    if r.dim() != 4 or r.shape[3] != 5:
        raise ValueError("bt_lines takes fields of shape (nz, ny, nx, 5)")
    nz, ny, nx = r.shape[:3]
    _need(r, torch.float64, (nz, ny, nx, 5), "r")
    _need(coef, torch.float64, (3, nz, ny, nx, 5, 5), "coef")
    if x is None:
        x = torch.empty_like(r)
    if work is None:
        work = torch.empty((nz, ny, nx, 5, 5), dtype=torch.float64,
                           device=r.device)
    _need(x, torch.float64, (nz, ny, nx, 5), "x")
    _need(work, torch.float64, (nz, ny, nx, 5, 5), "work")
    L.check(lib.m2s_bt_lines(nx, ny, nz, ax,
                             _ptr(coef), _ptr(r), _ptr(x), _ptr(work),
                             _stream()), "m2s_bt_lines")
    return x


def face_grad(A: Stencil, u, lam):
    lib = L.load()
    nz, ny, nx = A.shape
    _need(u, torch.float64, A.shape, "u")
    _need(lam, torch.float64, A.shape, "lam")
    opts = dict(dtype=torch.float64, device=u.device)
    gx = torch.empty((nz, ny, nx + 1), **opts)
    gy = torch.empty((nz, ny + 1, nx), **opts)
    gz = torch.empty((nz + 1, ny, nx), **opts)
    L.check(lib.m2s_face_grad(A.ref(), _ptr(u), _ptr(lam), _ptr(gx),
                              _ptr(gy), _ptr(gz), _stream()), "m2s_face_grad")
    return gx, gy, gz


def dot(x, y):
    lib = L.load()
    if x.dtype != torch.float64 or y.dtype != torch.float64:
        raise TypeError("dot takes float64 tensors")
    if x.numel() != y.numel() or not x.is_contiguous() or \
            not y.is_contiguous():
        raise ValueError("dot needs contiguous tensors of equal size")
    out = torch.empty((), dtype=torch.float64, device=x.device)
    L.check(lib.m2s_dot(_ptr(x), _ptr(y), x.numel(), _ptr(out), _stream()),
            "m2s_dot")
    return out


def convert(src, dtype):
    lib = L.load()
    dst = torch.empty(src.shape, dtype=dtype, device=src.device)
    L.check(lib.m2s_convert(_ptr(src), _DT[src.dtype], _ptr(dst), _DT[dtype],
                            src.numel(), _stream()), "m2s_convert")
    return dst


def stream(kind, a, c, b=None, s=1.0):
    """STREAM reference pass (measurement only): "copy" c = a, "triad"
    c = a + s b, over double tensors."""
    lib = L.load()
    k = {"copy": 0, "triad": 1}[kind]
    n = a.numel()
    _need(a, torch.float64, tuple(a.shape), "a")
    _need(c, torch.float64, tuple(a.shape), "c")
    if k == 1:
        _need(b, torch.float64, tuple(a.shape), "b")
    L.check(lib.m2s_stream(k, _ptr(a), _ptr(b) if b is not None else None,
                           _ptr(c), float(s), n, _stream()), "m2s_stream")
    return c


def plan_sweep(A: Stencil):
    """Host-only schedule of the wavefront sweep (no GPU needed)."""
    lib = L.load()
    p = L.SweepPlanC()
    L.check(lib.m2s_plan_sweep(A.ref(), C.byref(p)), "m2s_plan_sweep")
    return {f: getattr(p, f) for f, _ in L.SweepPlanC._fields_}


# --------------------------------------------------------------------------
# Autograd.
# --------------------------------------------------------------------------
class SolveFn(torch.autograd.Function):
    """u = A(k)^{-1} f by MG-PCG on the VAR7 operator.  Backward: one adjoint
    MG-PCG solve A^T lam = du (A symmetric) and the face-gradient kernel:
    df = lam, dk_f = -(lam_p - lam_q)(u_p - u_q)."""

    @staticmethod
    def forward(ctx, kx, ky, kz, f, levels, rtol, max_iter):
        A = var7(kx, ky, kz)
        mg = MG(A, levels)
        pws = PcgWorkspace(A)
        u, info = pcg_solve(A, f.contiguous(), None, "mg", mg,
                            max_iter=max_iter, rtol=rtol, ws=pws)
        ctx.save_for_backward(kx, ky, kz, u)
        ctx.cfg = (levels, rtol, max_iter)
        ctx.info = info
        # the backward solves with the same operator: it reuses the
        # hierarchy and the CG vectors (autograd rejects a backward after an
        # in-place change of the saved faces, so they still describe it)
        ctx.A, ctx.mg, ctx.pws = A, mg, pws
        return u

    @staticmethod
    def backward(ctx, gu):
        kx, ky, kz, u = ctx.saved_tensors
        levels, rtol, max_iter = ctx.cfg
        A, mg, pws = ctx.A, ctx.mg, ctx.pws
        lam, _ = pcg_solve(A, gu.contiguous(), None, "mg", mg,
                           max_iter=max_iter, rtol=rtol, ws=pws)
        gx, gy, gz = face_grad(A, u, lam)
        ctx.A = ctx.mg = ctx.pws = None
        return gx, gy, gz, lam, None, None, None


def solve(kx, ky, kz, f, levels=3, rtol=1e-10, max_iter=200):
    return SolveFn.apply(kx, ky, kz, f, levels, rtol, max_iter)


class SymGSFn(torch.autograd.Function):
    """x_new = sweep(r, x_old) for a symmetric stencil (CONST27 / VAR7 with
    fixed coefficients).  Backward: the transposed sweeps in reverse order
    (m2s_symgs_adjoint)."""

    @staticmethod
    def forward(ctx, r, x, A, direction):
        ctx.A, ctx.direction = A, direction
        out = x.detach().clone()
        symgs(A, r.detach().contiguous(), out, direction)
        return out

    @staticmethod
    def backward(ctx, g):
        gr, gx = symgs_adjoint(ctx.A, g.contiguous(), ctx.direction)
        return gr, gx, None, None


def symgs_fn(A, r, x, direction="sym"):
    return SymGSFn.apply(r, x, A, direction)
