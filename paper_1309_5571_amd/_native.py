"""ctypes view of the C ABI in include/dmrg.h (argument marshalling only).

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation of any entry point.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdmrg.so")

OK = 0
W_NOT_CONVERGED = 1
E_INVALID_ARG = -1
E_SECTOR = -2
E_LAYOUT = -3
E_NOMEM = -4
E_HIP = -5
E_NONFINITE = -6
E_BREAKDOWN = -7
E_UNSUPPORTED = -8

F64, F32, BF16 = 0, 1, 2
PREC = {"f64": F64, "fp64": F64, "f32": F32, "fp32": F32, "bf16": BF16}
OP_IDENTITY, OP_DIAG, OP_DENSE = 0, 1, 2
OP_KIND = {"identity": OP_IDENTITY, "diag": OP_DIAG, "dense": OP_DENSE}


class Space(ctypes.Structure):
    _fields_ = [("nsec", c_int32), ("rank", c_int32), ("label", POINTER(c_int32)), ("dim", POINTER(c_int64))]


class Op(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("nblk", c_int32), ("src", POINTER(c_int32)), ("dst", POINTER(c_int32)),
                ("off", POINTER(c_int64)), ("data", c_void_p)]


class Term(ctypes.Structure):
    _fields_ = [("a", c_int32), ("b", c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("left", Space), ("right", Space), ("target", POINTER(c_int32)),
                ("nop_left", c_int32), ("nop_right", c_int32),
                ("ops_left", POINTER(Op)), ("ops_right", POINTER(Op)),
                ("nterm", c_int32), ("terms", POINTER(Term))]


class DavidsonOpts(ctypes.Structure):
    _fields_ = [("tol", c_double), ("kmax", c_int32), ("kmin", c_int32), ("max_iter", c_int32),
                ("precond_floor", c_double), ("prec", c_int32), ("tol_lowprec", c_double),
                ("refine", c_int32), ("use_graph", c_int32), ("graph_chunk", c_int32),
                ("eig_solver", c_int32)]


class DavidsonInfo(ctypes.Structure):
    _fields_ = [("energy", c_double), ("residual", c_double), ("iterations", c_int32),
                ("iterations_low", c_int32), ("projections", c_int32), ("restarts", c_int32),
                ("converged", c_int32), ("breakdown", c_int32), ("host_waits", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RenormBlock(ctypes.Structure):
    _fields_ = [("o", c_int64), ("u_dst", c_int64), ("u_src", c_int64), ("out", c_int64),
                ("rows", c_int32), ("cols", c_int32), ("k_dst", c_int32), ("k_src", c_int32), ("diag", c_int32)]


class Place(ctypes.Structure):
    _fields_ = [("src", c_int64), ("dst", c_int64), ("rows", c_int32), ("cols", c_int32), ("ld_src", c_int32),
                ("ld_dst", c_int32), ("coef", c_double), ("identity", c_int32)]


class BlockOpts(ctypes.Structure):
    _fields_ = [("tol", c_double), ("nroots", c_int32), ("kmax", c_int32), ("kmin", c_int32), ("max_iter", c_int32),
                ("precond_floor", c_double), ("chunk", c_int32)]


class BlockInfo(ctypes.Structure):
    _fields_ = [("iterations", c_int32), ("projections", c_int32), ("restarts", c_int32), ("converged", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KronTerm(ctypes.Structure):
    _fields_ = [("out", c_int32), ("a", c_int32), ("b", c_int32), ("coef", c_double)]


class EnlargeSizes(ctypes.Structure):
    _fields_ = [("nsec", c_int32), ("nblk_total", c_int32), ("m", c_int64), ("data_len", c_int64)]


class Term4(ctypes.Structure):
    _fields_ = [("a", c_int32), ("b", c_int32), ("c", c_int32), ("d", c_int32)]


class Problem4(ctypes.Structure):
    _fields_ = [("space", Space * 4), ("target", POINTER(c_int32)), ("nop", c_int32 * 4),
                ("ops", POINTER(Op) * 4), ("nterm", c_int32), ("terms", POINTER(Term4))]


class DmrgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"dmrg status {status}: {message}")
        self.status = status


_lib = None

SIGNATURES = {
    "dmrg_problem_check": (c_int32, [POINTER(Problem)]),
    "dmrg_plan_create": (c_int32, [POINTER(c_void_p), c_int32, POINTER(Problem), c_int32, c_int32, c_void_p,
                                   c_size_t, c_void_p]),
    "dmrg_plan_workspace_size": (c_int32, [c_int32, POINTER(Problem), c_int32, c_int32, POINTER(c_size_t)]),
    "dmrg_plan_sizes": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int32), POINTER(c_int32),
                                  POINTER(c_int64), POINTER(c_int64)]),
    "dmrg_plan_layout": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                   POINTER(c_int64), POINTER(c_int64)]),
    "dmrg_plan_records": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                    POINTER(c_int32)]),
    "dmrg_project": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "dmrg_project_backward": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "dmrg_project_block": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p]),
    "dmrg_davidson_default_opts": (None, [POINTER(DavidsonOpts)]),
    "dmrg_davidson": (c_int32, [c_void_p, c_void_p, POINTER(DavidsonOpts), c_void_p, POINTER(c_double),
                                POINTER(DavidsonInfo), c_void_p]),
    "dmrg_diagonal": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "dmrg_gemv_t": (c_int32, [c_int64, c_int32, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "dmrg_gemv_n": (c_int32, [c_int64, c_int32, c_void_p, c_int64, c_void_p, c_double, c_void_p, c_void_p]),
    "dmrg_gemv_t_noalloc": (c_int32, [c_int64, c_int32, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "dmrg_density_layout": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64)]),
    "dmrg_density": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "dmrg_eigh_blocks": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p]),
    "dmrg_truncate": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_void_p]),
    "dmrg_renormalize": (c_int32, [c_int32, POINTER(RenormBlock), c_void_p, c_void_p, c_void_p, c_void_p]),
    "dmrg_place_blocks": (c_int32, [c_int32, POINTER(Place), c_void_p, c_void_p, c_void_p]),
    "dmrg_set_tile_table": (c_int32, [c_int32, POINTER(c_int32), POINTER(c_int32)]),
    "dmrg_enlarge": (c_int32, [POINTER(Space), c_int32, POINTER(Op), POINTER(Space), c_int32, POINTER(Op), c_int32,
                               POINTER(KronTerm), c_int32, POINTER(EnlargeSizes), c_void_p, c_void_p, c_void_p,
                               c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "dmrg_plan_create_l11r": (c_int32, [POINTER(c_void_p), c_int32, POINTER(Problem4), c_void_p]),
    "dmrg_block_default_opts": (None, [POINTER(BlockOpts)]),
    "dmrg_block_davidson": (c_int32, [c_void_p, c_void_p, POINTER(BlockOpts), c_void_p, POINTER(c_double),
                                      POINTER(c_double), POINTER(BlockInfo), c_void_p]),
    "dmrg_plan_destroy": (None, [c_void_p]),
    "dmrg_last_error": (c_char_p, []),
    "dmrg_version": (c_char_p, []),
}


def lib():
    """Load libdmrg.so (built by paper_1309_5571_amd.build); raise if missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1309_5571_amd.build` "
                              "(there is no non-HIP implementation)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def last_error() -> str:
    return lib().dmrg_last_error().decode()


def check(status: int, allow_warning: bool = False) -> int:
    if status < 0 or (status > 0 and not allow_warning):
        raise DmrgError(status, last_error())
    return status
