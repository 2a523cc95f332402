"""ctypes binding of libpbcgs.so (include/pbcgs.h).  Argument marshalling only:
every step of a solve runs in the library's HIP kernels.  The library is
loaded from this package directory; if it has not been built, loading fails
with an error instead of falling back to anything else."""

from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbcgs.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pbcgs.h")

SUCCESS, MAXIT, BREAKDOWN, NONFINITE = 0, 1, 2, 3
ERR_INVALID_ARG, ERR_ALLOC, ERR_HIP, ERR_UNSUPPORTED = -1, -2, -3, -4

BICGSTAB, PBICGSTAB, PBICGSTAB_RR, CA_BICGSTAB, CG, CGCG, PIPE_CG = 0, 1, 2, 3, 4, 5, 6
PRECOND_NONE, PRECOND_JACOBI, PRECOND_JACOBI_FOLDED = 0, 1, 2
FP64, FP32_RR64 = 0, 1
COLS_INT32, COLS_BLOCK16, COLS_DIAG16, COLS_NONE = 0, 1, 2, 3

FLAG_DIRECT = 1       # launch kernels directly instead of replaying a HIP graph
FLAG_TIME_KERNELS = 2  # time the two fused kernels of each iteration with events
FLAG_ALPHA_EQ5 = 4     # alpha_{i+1} of the pipelined variants by eq. (5) instead of eq. (3)
FLAG_INDEX32 = 8       # read the int32 columns even where the operator holds a compact copy
FLAG_NO_DIA = 16       # read the CSR arrays even where the operator has a diagonal layout
FLAG_POISON = 32       # test hook: NaN-fill the workspace before the solve writes it


class Opts(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("maxit", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("rr_period", ctypes.c_int32),
        ("rr_max", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("history", ctypes.c_void_p),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("n_rr", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("syncs_per_iter", ctypes.c_int32),
        ("relres_rec", ctypes.c_double),
        ("relres_true", ctypes.c_double),
        ("ms", ctypes.c_double),
        ("kernel_ms", ctypes.c_double * 2),
        ("kernel_calls", ctypes.c_int32 * 2),
        ("rows_per_wave_blocks", ctypes.c_int32),
        ("workgroups", ctypes.c_int32),
        ("value_codes", ctypes.c_int32),
    ]


class TuneReport(ctypes.Structure):
    _fields_ = [
        ("best", ctypes.c_int32),
        ("ncand", ctypes.c_int32),
        ("cand", ctypes.c_int32 * 12),
        ("ms_per_iter", ctypes.c_double * 12),
        ("best_ms_per_iter", ctypes.c_double),
    ]


class TuneEntry(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_char * 64),
        ("build", ctypes.c_char * 32),
        ("nnz", ctypes.c_int64),
        ("n", ctypes.c_int32),
        ("op_kind", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("read_path", ctypes.c_int32),
        ("best", ctypes.c_int32),
    ]


class PbcgsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pbcgs error {code}: {msg}")
        self.code = code


_lib = None

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double

_SIGNATURES = {
    "pbcgs_ctx_create": (ctypes.c_int, [ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "pbcgs_ctx_destroy": (ctypes.c_int, [_vp]),
    "pbcgs_last_error": (ctypes.c_char_p, [_vp]),
    "pbcgs_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "pbcgs_op_csr": (ctypes.c_int, [_vp, _i32, _i64, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "pbcgs_op_stencil": (ctypes.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _i32, ctypes.POINTER(_vp)]),
    "pbcgs_op_convdiff27": (ctypes.c_int, [_vp, _i32, _vp, ctypes.POINTER(_f64), _f64, ctypes.POINTER(_vp)]),
    "pbcgs_op_destroy": (ctypes.c_int, [_vp]),
    "pbcgs_op_transpose": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(_vp)]),
    "pbcgs_csr_outer_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "pbcgs_op_rows": (_i64, [_vp]),
    "pbcgs_op_index_bytes": (ctypes.c_int, [_vp]),
    "pbcgs_op_column_form": (ctypes.c_int, [_vp]),
    "pbcgs_op_diagonals": (ctypes.c_int, [_vp]),
    "pbcgs_spmv": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "pbcgs_dot": (ctypes.c_int, [_vp, _i64, _vp, _vp, ctypes.POINTER(_f64)]),
    "pbcgs_jacobi_dinv": (ctypes.c_int, [_vp, _vp, _vp]),
    "pbcgs_solve": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.POINTER(Opts), ctypes.POINTER(Info)]),
    "pbcgs_solve_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.POINTER(Opts), ctypes.POINTER(Info)]),
    "pbcgs_solve_batched": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                           ctypes.POINTER(_vp), ctypes.POINTER(Opts), ctypes.POINTER(Info)]),
    "pbcgs_tune": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(Opts), _i32, ctypes.POINTER(TuneReport)]),
    "pbcgs_tune_batched": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(Opts),
                                          _i32, ctypes.POINTER(TuneReport)]),
    "pbcgs_debug_perturb": (ctypes.c_int, [_vp, _i32, _f64]),
    "pbcgs_tune_cache_size": (_i32, []),
    "pbcgs_tune_cache_get": (ctypes.c_int, [_i32, ctypes.POINTER(TuneEntry)]),
    "pbcgs_tune_cache_put": (ctypes.c_int, [ctypes.POINTER(TuneEntry)]),
    "pbcgs_tune_cache_clear": (ctypes.c_int, []),
    "pbcgs_tune_cache_key": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32, ctypes.POINTER(TuneEntry)]),
    "pbcgs_convdiff_nnz": (_i64, [_i32, _i32, _i32]),
    "pbcgs_assemble_convdiff": (ctypes.c_int, [_vp, _i32, _i32, _i32, ctypes.POINTER(_f64), _vp, _f64,
                                               _vp, _vp, _vp]),
}


def declared_functions() -> list[str]:
    """Names of the functions include/pbcgs.h declares."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pbcgs_[a-z_0-9]+)\s*\(", text)))


def lib():
    """The loaded library; raises if libpbcgs.so is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built: the HIP library is required (run "
                "`python -c 'import __graft_entry__ as g; g.build()'` or "
                "`python paper_1612_01395_amd/build.py`)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error(ctx=None) -> str:
    msg = lib().pbcgs_last_error(ctx)
    return msg.decode() if msg else ""


def check(code: int, ctx=None) -> int:
    if code < 0:
        raise PbcgsError(code, last_error(ctx) or lib().pbcgs_status_str(code).decode())
    return code
