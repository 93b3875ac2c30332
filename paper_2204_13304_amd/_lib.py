"""ctypes declarations of libm2s.so (include/m2s.h).  Argument marshalling
only; raises if the library cannot be loaded -- there is no fallback."""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libm2s.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "m2s.h")

M2S_OK = 0
STATUS = {0: "M2S_OK", 1: "M2S_ERR_ARG", 2: "M2S_ERR_SHAPE",
          3: "M2S_ERR_DTYPE", 4: "M2S_ERR_ALIAS", 5: "M2S_ERR_HIP",
          6: "M2S_ERR_TIMEOUT", 7: "M2S_ERR_BREAKDOWN",
          8: "M2S_ERR_NOT_CONVERGED", 9: "M2S_ERR_UNSUPPORTED"}
F64, F32 = 0, 1
CONST27, VAR7, BLOCK7_5 = 0, 1, 2
FWD, BWD, SYM = 1, 2, 3
PC_NONE, PC_SYMGS, PC_MG = 0, 1, 2


class Extent(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32)]


class StencilC(C.Structure):
    _fields_ = [("kind", C.c_int), ("dtype", C.c_int), ("ext", Extent),
                ("diag", C.c_double), ("offdiag", C.c_double),
                ("kx", C.c_void_p), ("ky", C.c_void_p), ("kz", C.c_void_p),
                ("blocks", C.c_void_p)]


class PcgOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("rtol", C.c_double),
                ("replace_every", C.c_int), ("check_every", C.c_int)]


class PcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("r0_norm", C.c_double),
                ("status", C.c_int), ("seconds", C.c_double)]


class SweepPlanC(C.Structure):
    _fields_ = [("slab_planes", C.c_int32), ("nslabs", C.c_int32),
                ("row_slots", C.c_int32), ("lag_row", C.c_int32),
                ("lag_plane", C.c_int32), ("steps", C.c_int32),
                ("threads", C.c_int32), ("publish_every", C.c_int32)]


class M2SError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)}")


_lib = None

_P = C.c_void_p
_S = C.POINTER(StencilC)
_SIGS = {
    "m2s_status_string": (C.c_char_p, [C.c_int]),
    "m2s_version": (C.c_int, []),
    "m2s_workspace_create": (C.c_int, [_S, C.POINTER(C.c_void_p)]),
    "m2s_workspace_destroy": (None, [_P]),
    "m2s_check": (C.c_int, [_P, _P]),
    "m2s_spmv": (C.c_int, [_S, _P, _P, _P]),
    "m2s_spmv_part": (C.c_int, [_S, C.c_int, _P, _P, _P]),
    "m2s_symgs": (C.c_int, [_S, _P, _P, C.c_int, _P, _P]),
    "m2s_symgs_oop": (C.c_int, [_S, _P, _P, _P, C.c_int, _P, _P]),
    "m2s_symgs_sequential": (C.c_int, [_S, _P, _P, C.c_int, _P]),
    "m2s_symgs_xline": (C.c_int, [_S, _P, _P, C.c_int, _P, _P]),
    "m2s_symgs_adjoint": (C.c_int, [_S, _P, _P, _P, C.c_int, _P, _P]),
    "m2s_ssor_sweep": (C.c_int, [_S, _P, _P, C.c_double, C.c_int, _P, _P]),
    "m2s_ssor_sweep_sequential": (C.c_int, [_S, _P, _P, C.c_double, C.c_int,
                                            _P]),
    "m2s_mg_create": (C.c_int, [_S, C.c_int, C.c_int,
                                C.POINTER(C.c_void_p)]),
    "m2s_mg_vcycle": (C.c_int, [_P, _P, _P, _P]),
    "m2s_mg_destroy": (None, [_P]),
    "m2s_pcg_solve": (C.c_int, [_S, C.c_int, _P, _P, _P,
                                C.POINTER(PcgOpts), C.POINTER(PcgInfo), _P,
                                _P]),
    "m2s_pcg_workspace_create": (C.c_int, [_S, C.POINTER(C.c_void_p)]),
    "m2s_pcg_workspace_destroy": (None, [_P]),
    "m2s_pcg_solve_ws": (C.c_int, [_S, C.c_int, _P, _P, _P,
                                   C.POINTER(PcgOpts), C.POINTER(PcgInfo),
                                   _P, _P, _P]),
    "m2s_face_grad": (C.c_int, [_S, _P, _P, _P, _P, _P, _P]),
    "m2s_jacobi9": (C.c_int, [C.c_int32, C.c_int32, C.c_double, C.c_double,
                              _P, _P, _P, C.c_int32, C.c_int32, _P]),
    "m2s_penta_lines": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                  _P, _P, _P, _P, _P]),
    "m2s_bt_lines": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                               _P, _P, _P, _P, _P]),
    "m2s_dilu27_factor": (C.c_int, [_S, _P, _P, _P]),
    "m2s_dilu27_apply": (C.c_int, [_S, _P, _P, _P, _P, _P]),
    "m2s_ilu0_factor": (C.c_int, [_S, _P, _P, _P]),
    "m2s_ilu0_apply": (C.c_int, [_S, _P, _P, _P, _P, _P]),
    "m2s_ilu0_pack": (C.c_int, [_S, _P, _P, _P, _P, _P, _P]),
    "m2s_ilu0_apply_packed": (C.c_int, [_S, _P, _P, _P, _P, _P, _P]),
    "m2s_dot": (C.c_int, [_P, _P, C.c_int64, _P, _P]),
    "m2s_dot_noalloc": (C.c_int, [_P, _P, C.c_int64, _P, _P]),
    "m2s_convert": (C.c_int, [_P, C.c_int, _P, C.c_int, C.c_int64, _P]),
    "m2s_stream": (C.c_int, [C.c_int32, _P, _P, _P, C.c_double, C.c_int64,
                             _P]),
    "m2s_plan_sweep": (C.c_int, [_S, C.POINTER(SweepPlanC)]),
}


def header_symbols(path: str = HEADER):
    """Names of the functions declared in include/m2s.h."""
    with open(path) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(m2s_[a-z0-9_]+)\s*\(", text)))


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(
            f"libm2s.so not found at {LIBPATH}; build it with "
            "`python -m paper_2204_13304_amd.build` (hipcc, gfx950)")
    lib = C.CDLL(LIBPATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status, what=""):
    if status != M2S_OK:
        raise M2SError(status, what)
