"""CPU oracle for the pipelined BiCGStab solvers -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around ``oracle.c`` (plain FP64 C, no fused multiply-add).
Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package; the HIP library never does, and the two share no
code.  ``exact.py`` next to it is an exact-rational twin used to pin the FP64
oracle on tiny systems.

Algorithms (numbered as in arXiv 1612.01395, in order of appearance):
``ALG_BICGSTAB`` -> Algorithm 7 (Algorithm 10 when ``dinv`` is given);
``ALG_PBICGSTAB`` -> Algorithm 9 (Algorithm 11 with ``dinv``);
``ALG_PBICGSTAB_RR`` -> the same with residual replacement (Section 4.2);
``ALG_CA_BICGSTAB`` -> Algorithm 8 (Section 3.1); ``ALG_CG``, ``ALG_CGCG``,
``ALG_PIPE_CG`` -> Algorithms 2, 4 and 6 (Section 2).
:func:`solve_folded` runs Algorithm 7 / 9 on A M^{-1} formed explicitly (the
right preconditioning of Section 3.6 with the product built).
:func:`solve_mp` is the precision form of Algorithm 9 with replacement; an
exact-rational twin with IEEE 754 rounding of every operation
(``exact.pbicgstab_mp``, ``ieee.py``) pins its rounding sequence bit for bit.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ALG_BICGSTAB = 0
ALG_PBICGSTAB = 1
ALG_PBICGSTAB_RR = 2
ALG_CA_BICGSTAB = 3  # Algorithm 8, unpreconditioned (a preconditioned solve folds A M^{-1})
ALG_CG = 4         # Algorithm 2 (symmetric positive definite A)
ALG_CGCG = 5       # Algorithm 4
ALG_PIPE_CG = 6    # Algorithm 6 (p-CG)

SUCCESS, MAXIT, BREAKDOWN, NONFINITE = 0, 1, 2, 3
STATUS_NAMES = {0: "success", 1: "maxit", 2: "breakdown", 3: "nonfinite"}

_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


def build() -> None:
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, -ffp-contract=off)."""
    subprocess.run(["sh", os.path.join(_HERE, "build.sh")], check=True)


def _nullable(ptr_type):
    """ndpointer that also accepts None (passed as NULL)."""

    class _P(ptr_type):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return ptr_type.from_param(obj)

    return _P


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_assemble_nnz.restype = ctypes.c_int64
        L.or_assemble_nnz.argtypes = [ctypes.c_int32] * 3
        L.or_assemble.restype = ctypes.c_int64
        L.or_assemble.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _f64p,
                                  _nullable(_f64p), ctypes.c_double, _i32p, _i32p, _f64p]
        L.or_assemble_rows.restype = ctypes.c_int64
        L.or_assemble_rows.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _f64p,
                                       _nullable(_f64p), ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                       _i32p, _i32p, _f64p]
        L.or_spmv.restype = None
        L.or_spmv.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.or_dot.restype = ctypes.c_double
        L.or_dot.argtypes = [ctypes.c_int64, _f64p, _f64p]
        L.or_pairwise_sum.restype = ctypes.c_double
        L.or_pairwise_sum.argtypes = [ctypes.c_int64, _f64p]
        L.or_jacobi_dinv.restype = ctypes.c_int
        L.or_jacobi_dinv.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p]
        L.or_solve.restype = ctypes.c_int
        L.or_solve.argtypes = [ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _f64p,
                               _nullable(_f64p), _f64p, _f64p, ctypes.c_double, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_int32, _nullable(_f64p), _nullable(_f64p),
                               _i32p, _f64p]
        L.or_solve_mp.restype = ctypes.c_int
        L.or_solve_mp.argtypes = [ctypes.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p, ctypes.c_double,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _nullable(_f64p),
                                  _nullable(_f64p), _i32p, _f64p]
        L.or_dot32.restype = ctypes.c_double
        L.or_dot32.argtypes = [ctypes.c_int64, _f32p, _f32p]
        L.or_spmv32.restype = None
        L.or_spmv32.argtypes = [ctypes.c_int32, _i32p, _i32p, _f32p, _f32p, _f32p]
        L.or_set_alpha_form.restype = None
        L.or_set_alpha_form.argtypes = [ctypes.c_int32]
        L.or_set_perturb.restype = None
        L.or_set_perturb.argtypes = [ctypes.c_int32, ctypes.c_double]
        L.or_counters_get.restype = None
        L.or_counters_get.argtypes = [np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")]
        L.or_counters_reset.restype = None
        L.or_counters_reset.argtypes = []
        L.or_set_threads.restype = None
        L.or_set_threads.argtypes = [ctypes.c_int32]
        L.or_get_threads.restype = ctypes.c_int32
        L.or_get_threads.argtypes = []
        _lib = L
    return _lib


def set_threads(t: int) -> None:
    lib().or_set_threads(int(t))


def get_threads() -> int:
    return int(lib().or_get_threads())


class CSR:
    """Host CSR matrix: int32 row_ptr[n+1], int32 col[nnz], float64 val[nnz]."""

    def __init__(self, row_ptr, col, val):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.n = len(self.row_ptr) - 1

    @property
    def nnz(self) -> int:
        return len(self.val)

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def assemble_nnz(dim: int, n: int, npts: int) -> int:
    return int(lib().or_assemble_nnz(dim, n, npts))


def assemble(dim: int, n: int, npts: int, beta, kappa=None, shift: float = 0.0) -> CSR:
    """The convection-diffusion operator of the workloads, assembled plainly in C."""
    nnz = assemble_nnz(dim, n, npts)
    if nnz < 0:
        raise ValueError(f"unsupported operator dim={dim} npts={npts} n={n}")
    N = n ** dim
    rp = np.zeros(N + 1, np.int32)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz, np.float64)
    b = np.zeros(3, np.float64)
    b[:dim] = beta
    k = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
    got = lib().or_assemble(dim, n, npts, b, k, float(shift), rp, col, val)
    if got != nnz:
        raise RuntimeError("oracle assembly failed")
    return CSR(rp, col, val)


def assemble_rows(dim: int, n: int, npts: int, beta, row_begin: int, row_end: int, kappa=None,
                  shift: float = 0.0):
    """Rows [row_begin, row_end) of the operator: (row_ptr relative to row_begin, col, val)."""
    cnt = row_end - row_begin
    rp = np.zeros(cnt + 1, np.int32)
    col = np.zeros(cnt * npts, np.int32)
    val = np.zeros(cnt * npts, np.float64)
    b = np.zeros(3, np.float64)
    b[:dim] = beta
    k = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
    got = lib().or_assemble_rows(dim, n, npts, b, k, float(shift), row_begin, row_end, rp, col, val)
    if got < 0:
        raise ValueError("unsupported operator")
    return rp, col[:got], val[:got]


def assemble_workload(w, kappa=None) -> CSR:
    """Assemble a :class:`paper_1612_01395_amd.inputs.Workload`."""
    return assemble(w.dim, w.n, w.npts, w.beta, kappa, w.shift)


def spmv(A: CSR, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.n, np.float64)
    lib().or_spmv(A.n, A.row_ptr, A.col, A.val, x, y)
    return y


def dot(x, y) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    return float(lib().or_dot(len(x), x, y))


def pairwise_sum(a) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return float(lib().or_pairwise_sum(len(a), a))


def jacobi_dinv(A: CSR) -> np.ndarray:
    d = np.empty(A.n, np.float64)
    st = lib().or_jacobi_dinv(A.n, A.row_ptr, A.col, A.val, d)
    if st != 0:
        raise ValueError("zero or missing diagonal entry")
    return d


def solve(A: CSR, b, *, algo: int = ALG_PBICGSTAB_RR, dinv=None, x0=None, tol: float = 1e-8,
          maxit: int = 2000, rr_period: int = 50, rr_max: int = -1, history: bool = False,
          scalars: bool = False, alpha_form: int = 3, perturb=None):
    """Run one solver of the paper; returns ``(x, info)``.

    ``info`` holds iters, n_rr, status, relres_rec (last ||r_i||/||r_0||),
    relres_true (||b - A x|| / ||r_0||) and, on request, the residual
    history (length maxit+1) and the per-iteration scalars alpha, omega, beta.
    ``alpha_form`` 5 computes alpha_{i+1} of the pipelined solvers by eq. (5)
    instead of eq. (3).  ``perturb = (j, c)`` multiplies the recursive
    residual r_{j+1} of the pipelined solvers by c at the end of iteration j,
    after its reductions (a test hook for the replacement of Section 4.2).
    """
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    dv = None if dinv is None else np.ascontiguousarray(dinv, dtype=np.float64)
    hist = np.full(maxit + 1, np.nan) if history else None
    sc = np.full(3 * max(maxit, 1), np.nan) if scalars else None
    ints = np.zeros(3, np.int32)
    dbl = np.zeros(2, np.float64)
    lib().or_set_alpha_form(int(alpha_form))
    if perturb is not None:
        lib().or_set_perturb(int(perturb[0]), float(perturb[1]))
    try:
        st = lib().or_solve(algo, A.n, A.row_ptr, A.col, A.val, dv, b, x, float(tol), int(maxit),
                            int(rr_period), int(rr_max), hist, sc, ints, dbl)
    finally:
        lib().or_set_alpha_form(3)
        lib().or_set_perturb(-1, 1.0)
    if st < 0:
        raise ValueError(f"oracle solve failed with code {st}")
    info = {"iters": int(ints[0]), "n_rr": int(ints[1]), "status": int(ints[2]),
            "relres_rec": float(dbl[0]), "relres_true": float(dbl[1])}
    if history:
        info["history"] = hist[: info["iters"] + 1]
    if scalars:
        info["scalars"] = sc[: 3 * info["iters"]].reshape(-1, 3)
    return x, info


def fold_columns(A: CSR, dinv) -> CSR:
    """A M^{-1} for M^{-1} = diag(dinv): entry (i, j) times dinv_j, one
    rounding per entry.  Section 3.6 right-preconditions as A M^{-1} y = b,
    M x = y; with this product formed, the unpreconditioned algorithms apply."""
    d = np.ascontiguousarray(dinv, dtype=np.float64)
    return CSR(A.row_ptr, A.col, A.val * d[A.col])


def solve_folded(A: CSR, b, *, algo: int, dinv, x0=None, **kw):
    """Right-preconditioned solve with A M^{-1} formed (Section 3.6): Algorithm 7
    (``ALG_BICGSTAB``) or 9 (``ALG_PBICGSTAB``, ``ALG_PBICGSTAB_RR``) on
    A M^{-1} y = b from y_0 = M x_0 = x_0 / dinv; returns x = M^{-1} y = dinv * y.

    In exact arithmetic the iterates x_i are those of Algorithm 10 / 11.  The
    stopping test and the history use the residual of the folded system,
    b - A M^{-1} y_i (the unpreconditioned residual of x_i);
    ``relres_true`` is ||b - A x|| / ||r_0|| with the original A and the
    returned x, r_0 = b - A M^{-1} y_0.  Other keywords as :func:`solve`."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    d = np.ascontiguousarray(dinv, dtype=np.float64)
    Ah = fold_columns(A, d)
    x0a = np.zeros(A.n) if x0 is None else np.asarray(x0, dtype=np.float64)
    y0 = x0a / d
    y, info = solve(Ah, b, algo=algo, dinv=None, x0=y0, **kw)
    x = d * y
    r0 = b - spmv(Ah, y0)
    rho0 = math.sqrt(dot(r0, r0))
    r = b - spmv(A, x)
    info["relres_true"] = math.sqrt(dot(r, r)) / rho0 if rho0 > 0.0 else 0.0
    return x, info


def dot32(x, y) -> float:
    """(x, y) in binary32: pairwise sum of the binary32 products, widened."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    return float(lib().or_dot32(len(x), x, y))


def spmv32(A: CSR, x) -> np.ndarray:
    """y = f(A) x in binary32 (values rounded to binary32, rows in stored order)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty(A.n, np.float32)
    lib().or_spmv32(A.n, A.row_ptr, A.col, np.ascontiguousarray(A.val.astype(np.float32)), x, y)
    return y


def solve_mp(A: CSR, b, *, dinv=None, x0=None, tol: float = 1e-10, maxit: int = 4000, rr_period: int = 50,
             rr_max: int = -1, history: bool = False, scalars: bool = False, alpha_form: int = 3):
    """Precision form of p-BiCGStab with residual replacement: binary32
    vectors, SpMV, recurrences and dot products; binary64 replacement steps
    (Section 4.2), x update and alpha, beta, omega; convergence of the
    binary32 recursive residual confirmed by the binary64 true residual.
    With ``dinv`` the solve runs on A M^{-1} formed (see :func:`solve_folded`).
    Returns ``(x, info)`` like :func:`solve`."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    Ah, d = A, None
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    if dinv is not None:
        d = np.ascontiguousarray(dinv, dtype=np.float64)
        Ah = fold_columns(A, d)
        x = x / d
    y0 = x.copy()
    hist = np.full(maxit + 1, np.nan) if history else None
    sc = np.full(3 * max(maxit, 1), np.nan) if scalars else None
    ints = np.zeros(3, np.int32)
    dbl = np.zeros(2, np.float64)
    lib().or_set_alpha_form(int(alpha_form))
    try:
        st = lib().or_solve_mp(Ah.n, Ah.row_ptr, Ah.col, Ah.val, b, x, float(tol), int(maxit), int(rr_period),
                               int(rr_max), hist, sc, ints, dbl)
    finally:
        lib().or_set_alpha_form(3)
    if st < 0:
        raise ValueError(f"oracle solve failed with code {st}")
    info = {"iters": int(ints[0]), "n_rr": int(ints[1]), "status": int(ints[2]),
            "relres_rec": float(dbl[0]), "relres_true": float(dbl[1])}
    if d is not None:
        x = d * x
        r0 = (b - spmv(Ah, y0)).astype(np.float32)
        rho0 = math.sqrt(dot32(r0, r0))
        r = b - spmv(A, x)
        info["relres_true"] = math.sqrt(dot(r, r)) / rho0 if rho0 > 0.0 else 0.0
    if history:
        info["history"] = hist[: info["iters"] + 1]
    if scalars:
        info["scalars"] = sc[: 3 * info["iters"]].reshape(-1, 3)
    return x, info


def transpose(A: CSR) -> CSR:
    """A^T by its definition: row j lists column j of A in ascending row order
    (a stable sort of the entries by column; the row-major entry order breaks
    ties)."""
    rows = np.repeat(np.arange(A.n, dtype=np.int32), np.diff(A.row_ptr))
    order = np.argsort(A.col, kind="stable")
    counts = np.bincount(A.col, minlength=A.n)
    rp = np.zeros(A.n + 1, np.int64)
    rp[1:] = np.cumsum(counts)
    return CSR(rp.astype(np.int32), rows[order], A.val[order])


def outer_grad(A: CSR, lam, x) -> np.ndarray:
    """dL/da_ij = -lambda_i x_j at every stored entry (i, j): the gradient of a
    loss through A x = b, with lambda = A^{-T} dL/dx."""
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    return -(np.asarray(lam, dtype=np.float64)[rows] * np.asarray(x, dtype=np.float64)[A.col])


def counters() -> dict:
    out = np.zeros(6, np.int64)
    lib().or_counters_get(out)
    return dict(zip(["spmv", "pc", "glred", "dots", "flops", "rec"], (int(v) for v in out)))


def reset_counters() -> None:
    lib().or_counters_reset()
