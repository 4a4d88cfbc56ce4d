"""ctypes declarations of libdmrg's C ABI (include/dmrg.h), same names.

Loading imports torch first so that the library binds to the HIP runtime
torch already has in the process.  There is no fallback: if the library is
not built, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# DMRG_LIB may name another build of the same library (the host-sanitizer
# build used by the CPU tests)
LIB_PATH = os.environ.get("DMRG_LIB") or os.path.join(_HERE, "libdmrg.so")

DMRG_OK = 0
STATUS = {0: "DMRG_OK", 1: "DMRG_E_ARG", 2: "DMRG_E_QN", 3: "DMRG_E_SHAPE", 4: "DMRG_E_NOMEM",
          5: "DMRG_E_DEVICE", 6: "DMRG_E_NOCONV", 7: "DMRG_E_UNSUPPORTED"}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp64_plain": 3}


class DmrgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class dmrg_basis(C.Structure):
    _fields_ = [("nsec", C.c_int32), ("q", C.POINTER(C.c_int64)), ("dim", C.POINTER(C.c_int32))]


class dmrg_op(C.Structure):
    _fields_ = [("delta", C.c_int64), ("nblk", C.c_int32), ("row_sec", C.POINTER(C.c_int32)),
                ("col_sec", C.POINTER(C.c_int32)), ("blk", C.POINTER(C.POINTER(C.c_double)))]


class dmrg_term(C.Structure):
    _fields_ = [("c", C.c_double), ("A", C.POINTER(dmrg_op)), ("B", C.POINTER(dmrg_op)),
                ("group", C.c_int32)]


class dmrg_tblock(C.Structure):
    _fields_ = [("o_off", C.c_int64), ("rows", C.c_int32), ("cols", C.c_int32),
                ("wr_off", C.c_int64), ("kr", C.c_int32), ("wc_off", C.c_int64), ("kc", C.c_int32),
                ("out_off", C.c_int64), ("o_ld", C.c_int32), ("out_ld", C.c_int32)]


class dmrg_trunc(C.Structure):
    _fields_ = [("trunc_err", C.c_double), ("kept", C.c_int32), ("straddle", C.c_int32),
                ("lambda_", C.POINTER(C.c_double)), ("lambda_sec", C.POINTER(C.c_int32)),
                ("nsec", C.c_int32), ("kept_per_sec", C.POINTER(C.c_int32)),
                ("W", C.POINTER(C.POINTER(C.c_double))),
                ("W_all", C.POINTER(C.c_double)), ("W_total", C.c_int64)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_SIGS = {
    "dmrg_ctx_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "dmrg_ctx_destroy": (None, [_P]),
    "dmrg_ctx_set_stream": (C.c_int, [_P, _P]),
    "dmrg_ctx_set_timing": (C.c_int, [_P, C.c_int32]),
    "dmrg_ctx_timing": (C.c_int, [_P, C.c_int32, _D, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                  C.c_int32]),
    "dmrg_last_error": (C.c_char_p, []),
    "dmrg_version": (C.c_char_p, []),
    "dmrg_build_superblock": (C.c_int, [_P, C.POINTER(dmrg_basis), C.POINTER(dmrg_basis), C.c_int64,
                                        C.c_int32, C.POINTER(dmrg_term), C.c_int, C.POINTER(_P)]),
    "dmrg_sb_destroy": (None, [_P]),
    "dmrg_build_operator": (C.c_int, [_P, C.POINTER(dmrg_basis), C.POINTER(dmrg_basis), C.c_int64,
                                      C.c_int64, C.c_int32, C.POINTER(dmrg_term), C.c_int,
                                      C.POINTER(_P)]),
    "dmrg_sb_dims": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "dmrg_lanczos_tridiag": (C.c_int, [_P, _P, C.c_int32, _D, _D, C.POINTER(C.c_int32), _D]),
    "dmrg_host_ldos": (C.c_int, [C.c_int32, _D, _D, C.c_double, C.c_double, C.c_int32, _D,
                                 C.c_double, _D]),
    "dmrg_sb_layout": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                 C.POINTER(C.POINTER(C.c_int64)), C.POINTER(C.POINTER(C.c_int32)),
                                 C.POINTER(C.POINTER(C.c_int32))]),
    "dmrg_sb_stats": (C.c_int, [_P, _D, _D, _D, C.POINTER(C.c_int32)]),
    "dmrg_sb_set_coeffs": (C.c_int, [_P, _D]),
    "dmrg_sb_set_prec": (C.c_int, [_P, C.c_int]),
    "dmrg_hpsi": (C.c_int, [_P, _P, _P, C.c_double, C.c_double]),
    "dmrg_hpsi_noalloc": (C.c_int, [_P, _P, _P, C.c_double, C.c_double]),
    "dmrg_hpsi_adjoint": (C.c_int, [_P, _P, _P, _P, _D]),
    "dmrg_lanczos_ground": (C.c_int, [_P, _P, C.c_int32, C.c_double, _D, _P,
                                      C.POINTER(C.c_int32), _D]),
    "dmrg_rho_truncate": (C.c_int, [_P, _P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(dmrg_trunc)]),
    "dmrg_transform_blocks": (C.c_int, [_P, C.c_int32, C.POINTER(dmrg_tblock), _P, _P, _P]),
    "dmrg_host_sym_eigen": (C.c_int, [C.c_int32, _D, _D]),
    "dmrg_sb_autotune": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32)]),
    "dmrg_sb_set_variant": (C.c_int, [_P, C.c_int32]),
    "dmrg_sb_set_reorth": (C.c_int, [_P, C.c_int32]),
    "dmrg_sb_set_graphs": (C.c_int, [_P, C.c_int32]),
    "dmrg_ctx_set_mem_cap": (C.c_int, [_P, C.c_int64]),
    "dmrg_ctx_mem": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "dmrg_sb_graph_stats": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "dmrg_host_tridiag_lowest": (C.c_int, [C.c_int32, _D, _D, _D, _D]),
}

_lib = None
_shutting_down = False


def _at_exit():
    global _shutting_down
    _shutting_down = True


import atexit  # noqa: E402

atexit.register(_at_exit)


def alive():
    """False once the interpreter is shutting down (handles are then leaked,
    not freed, so no HIP call races the runtime's own teardown)."""
    return not _shutting_down


def lib():
    """The loaded library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_0902_3185_amd.build` "
                               "(or __graft_entry__.build())")
        import torch  # noqa: F401  -- bind to torch's HIP runtime
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != DMRG_OK:
        msg = lib().dmrg_last_error().decode(errors="replace")
        raise DmrgError(status, msg)
    return status


def declared_symbols():
    """Names of the functions declared in include/dmrg.h."""
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "dmrg.h")
    text = open(hdr).read()
    return sorted(set(re.findall(r"\b(dmrg_[a-z0-9_]+)\s*\(", text)))
