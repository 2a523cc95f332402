"""PyTorch-facing wrapper of the pipelined BiCGStab library.

Tensors provide device memory and the current HIP stream; every computation
is a call into libpbcgs.so.  The solvers are those of Cools & Vanroose,
arXiv 1612.01395: standard BiCGStab (Algorithm 7, preconditioned: 10),
pipelined BiCGStab (Algorithm 9, preconditioned: 11), pipelined BiCGStab
with residual replacement (Section 4.2), communication-avoiding BiCGStab
(Algorithm 8), and the CG family of Section 2 for symmetric positive definite
systems: CG (Algorithm 2), Chronopoulos & Gear CG (Algorithm 4) and
pipelined CG (Algorithm 6).

A context is bound to the stream that was current when it was created (the
default context of each device and stream is cached), and an operator runs
its solves on its context's stream.  A CSR operator keeps a compact 16-bit
copy of its column indices where one fits (``Operator.column_form``); it
changes how columns are read, never a result.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

VARIANTS = {"bicgstab": L.BICGSTAB, "pbicgstab": L.PBICGSTAB, "pbicgstab_rr": L.PBICGSTAB_RR,
            "ca_bicgstab": L.CA_BICGSTAB, "cg": L.CG, "cgcg": L.CGCG, "pipe_cg": L.PIPE_CG}
STATUS = {0: "success", 1: "maxit", 2: "breakdown", 3: "nonfinite"}
# "jacobi": M^{-1} = diag(1/a_ii) applied inside Algorithm 10 / 11; "jacobi_folded":
# the same right preconditioning with A M^{-1} formed, Algorithm 7 / 9 run on it.
PRECONDS = {None: L.PRECOND_NONE, "none": L.PRECOND_NONE, "jacobi": L.PRECOND_JACOBI,
            "jacobi_folded": L.PRECOND_JACOBI_FOLDED}
# "fp64": every operation in binary64; "fp32_rr64": binary32 vectors, SpMV, recurrences and
# dot products with binary64 residual replacement, x update and scalars (p-BiCGStab+RR only).
PRECISIONS = {"fp64": L.FP64, "fp32_rr64": L.FP32_RR64}


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_alpha_form(alpha_form: int):
    if alpha_form not in (3, 5):
        raise ValueError("alpha_form must be 3 (eq. (3)) or 5 (eq. (5))")


def _check_vec(t: torch.Tensor, n: int, name: str, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous {dtype} tensor with {n} elements")


class Context:
    """A library context bound to one device and one HIP stream.

    The library requires a context's operators to be destroyed before the
    context (``pbcgs_op_destroy`` uses it).  Python may finalize the two in
    either order when they are garbage in one reference cycle, so the
    context counts its live operators and :meth:`close` destroys it only
    once the last of them is closed."""

    def __init__(self, device: int | None = None, stream: torch.cuda.Stream | None = None):
        self._live_ops = 0
        self._closing = False
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        raw = stream.cuda_stream
        h = ctypes.c_void_p()
        L.check(L.lib().pbcgs_ctx_create(self.device, ctypes.c_void_p(raw) if raw else None, ctypes.byref(h)))
        self.handle = h

    def close(self):
        self._closing = True
        if getattr(self, "_live_ops", 0) == 0 and getattr(self, "handle", None):
            L.lib().pbcgs_ctx_destroy(self.handle)
            self.handle = None

    def _op_closed(self):
        self._live_ops -= 1
        if self._closing and self._live_ops == 0:
            self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return L.last_error(self.handle)

    def debug_perturb(self, iteration: int = -1, scale: float = 1.0) -> None:
        """Test hook of the residual replacement (Section 4.2): later binary64
        p-BiCGStab solves on this context multiply the recursive residual
        r_{iteration+1} by ``scale`` at the end of iteration ``iteration``,
        after its reductions.  ``iteration=-1`` switches it off."""
        L.check(L.lib().pbcgs_debug_perturb(self.handle, int(iteration), float(scale)), self.handle)


_contexts: dict = {}


def default_context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    stream = torch.cuda.current_stream(device)
    key = (int(device), stream.cuda_stream)
    ctx = _contexts.get(key)
    if ctx is None:
        ctx = Context(device, stream)
        _contexts[key] = ctx
    return ctx


class Operator:
    """A sparse operator known to the library (CSR or matrix-free stencil)."""

    def __init__(self, ctx: Context, handle, n: int, keep: tuple, kind: str):
        self.ctx = ctx
        self.handle = handle
        ctx._live_ops += 1
        self.n = n
        self._keep = keep  # the borrowed device arrays stay alive with the operator
        self.kind = kind

    @property
    def index_bytes(self) -> int:
        """Bytes per column index the solves read: 2 (a compact copy), 4
        (int32 columns) or 0 (stencil)."""
        return L.check(L.lib().pbcgs_op_index_bytes(self.handle), self.ctx.handle)

    @property
    def column_form(self) -> str:
        """The column form the solves read: "int32", "block16" (int16 offsets
        from the 64-row block start), "diag16" (diagonal codes) or "none"
        (stencil)."""
        f = L.check(L.lib().pbcgs_op_column_form(self.handle), self.ctx.handle)
        return {L.COLS_INT32: "int32", L.COLS_BLOCK16: "block16", L.COLS_DIAG16: "diag16", L.COLS_NONE: "none"}[f]

    @property
    def diagonals(self) -> int:
        """Diagonals of the operator's diagonal layout (0: it has none; see
        ``pbcgs_op_diagonals``)."""
        return L.check(L.lib().pbcgs_op_diagonals(self.handle), self.ctx.handle)

    def close(self):
        if getattr(self, "handle", None):
            L.lib().pbcgs_op_destroy(self.handle)
            self.handle = None
            self.ctx._op_closed()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def csr(row_ptr: torch.Tensor, col_idx: torch.Tensor, val: torch.Tensor, ctx: Context | None = None) -> Operator:
    """CSR operator from int32 row_ptr[n+1], int32 col_idx[nnz], float64 val[nnz] on the GPU."""
    ctx = ctx or default_context(row_ptr.device.index)
    n = row_ptr.numel() - 1
    nnz = val.numel()
    _check_vec(row_ptr, n + 1, "row_ptr", torch.int32)
    _check_vec(col_idx, nnz, "col_idx", torch.int32)
    _check_vec(val, nnz, "val")
    h = ctypes.c_void_p()
    L.check(L.lib().pbcgs_op_csr(ctx.handle, n, nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(val), ctypes.byref(h)),
            ctx.handle)
    return Operator(ctx, h, n, (row_ptr, col_idx, val), "csr")


def stencil(nx: int, ny: int, nz: int, coef, ctx: Context | None = None, npts: int | None = None) -> Operator:
    """Matrix-free 5- (nz == 1), 7- or 27-point stencil on an nx x ny x nz grid
    (rows x fastest, Dirichlet boundaries).  ``coef``: a sequence of npts
    constant coefficients in ascending-column order ({-y,-x,c,+x,+y},
    {-z,-y,-x,c,+x,+y,+z}, or the 27 offsets (dz, dy, dx) with dz slowest), or
    a float64 device tensor of npts * n per-row coefficients (coefficient d of
    row r at ``coef[d * n + r]``, borrowed by the operator; ``npts`` may be
    given, else it is coef.numel() // n)."""
    ctx = ctx or default_context()
    n = nx * ny * nz
    if isinstance(coef, torch.Tensor):
        if npts is None:
            npts = coef.numel() // n if n > 0 else 0
        _check_vec(coef, npts * n, "coef")
        h = ctypes.c_void_p()
        L.check(L.lib().pbcgs_op_stencil(ctx.handle, nx, ny, nz, int(npts), ctypes.c_void_p(coef.data_ptr()), 1,
                                         ctypes.byref(h)), ctx.handle)
        return Operator(ctx, h, n, (coef,), f"stencil{npts}_per_row")
    coef = [float(c) for c in coef]
    arr = (ctypes.c_double * len(coef))(*coef)
    h = ctypes.c_void_p()
    L.check(L.lib().pbcgs_op_stencil(ctx.handle, nx, ny, nz, len(coef), ctypes.cast(arr, ctypes.c_void_p), 0,
                                     ctypes.byref(h)), ctx.handle)
    return Operator(ctx, h, n, (), f"stencil{len(coef)}")


def convdiff27(n: int, kappa: torch.Tensor, beta, shift: float = 0.0, ctx: Context | None = None) -> Operator:
    """Matrix-free 27-point variable-coefficient convection-diffusion operator
    on the n^3 grid: the operator ``assemble_convdiff(3, n, 27, beta, kappa,
    shift)`` assembles, applied without a stored matrix (bitwise the same
    products).  ``kappa``: (n+1)^3 cell coefficients on the GPU, kept alive by
    the operator."""
    ctx = ctx or default_context(kappa.device.index)
    _check_vec(kappa, (n + 1) ** 3, "kappa")
    b = (ctypes.c_double * 3)(*[float(v) for v in beta])
    h = ctypes.c_void_p()
    L.check(L.lib().pbcgs_op_convdiff27(ctx.handle, n, _ptr(kappa), b, float(shift), ctypes.byref(h)), ctx.handle)
    return Operator(ctx, h, n ** 3, (kappa,), "convdiff27")


def transpose(A: Operator) -> Operator:
    """The transposed CSR operator (the library owns its arrays)."""
    h = ctypes.c_void_p()
    L.check(L.lib().pbcgs_op_transpose(A.ctx.handle, A.handle, ctypes.byref(h)), A.ctx.handle)
    return Operator(A.ctx, h, A.n, (A,), "csr")


def csr_outer_grad(A: Operator, lam: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """grad[k] = -lam[i] x[j] for every stored entry k = (i, j) of the CSR operator A."""
    _check_vec(lam, A.n, "lam")
    _check_vec(x, A.n, "x")
    nnz = A._keep[2].numel() if A.kind == "csr" and len(A._keep) == 3 else None
    if nnz is None:
        raise ValueError("csr_outer_grad needs a CSR operator built from row_ptr, col_idx, val")
    g = torch.empty(nnz, dtype=torch.float64, device=lam.device)
    L.check(L.lib().pbcgs_csr_outer_grad(A.ctx.handle, A.handle, _ptr(lam), _ptr(x), _ptr(g)), A.ctx.handle)
    return g


def convdiff_nnz(dim: int, n: int, npts: int) -> int:
    return int(L.check(L.lib().pbcgs_convdiff_nnz(dim, n, npts)))


def assemble_convdiff(dim: int, n: int, npts: int, beta, kappa: torch.Tensor | None = None, shift: float = 0.0,
                      device: int | None = None, ctx: Context | None = None):
    """Device assembly of the workloads' convection-diffusion operator -> (row_ptr, col_idx, val)."""
    ctx = ctx or default_context(device)
    dev = torch.device("cuda", ctx.device)
    N = n ** dim
    nnz = convdiff_nnz(dim, n, npts)
    rp = torch.empty(N + 1, dtype=torch.int32, device=dev)
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    val = torch.empty(nnz, dtype=torch.float64, device=dev)
    b = (ctypes.c_double * 3)(*([float(v) for v in beta] + [0.0] * (3 - len(beta))))
    if npts == 27:
        _check_vec(kappa, (n + 1) ** 3, "kappa")
    L.check(L.lib().pbcgs_assemble_convdiff(ctx.handle, dim, n, npts, b, _ptr(kappa), float(shift),
                                            _ptr(rp), _ptr(col), _ptr(val)), ctx.handle)
    return rp, col, val


def spmv(A: Operator, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    _check_vec(x, A.n, "x")
    y = torch.empty_like(x) if out is None else out
    _check_vec(y, A.n, "out")
    L.check(L.lib().pbcgs_spmv(A.ctx.handle, A.handle, _ptr(x), _ptr(y)), A.ctx.handle)
    return y


def dot(x: torch.Tensor, y: torch.Tensor, ctx: Context | None = None) -> float:
    """(x, y) in pairwise order (bit-reproducible)."""
    ctx = ctx or default_context(x.device.index)
    _check_vec(x, x.numel(), "x")
    _check_vec(y, x.numel(), "y")
    res = ctypes.c_double()
    L.check(L.lib().pbcgs_dot(ctx.handle, x.numel(), _ptr(x), _ptr(y), ctypes.byref(res)), ctx.handle)
    return res.value


def jacobi_dinv(A: Operator) -> torch.Tensor:
    d = torch.empty(A.n, dtype=torch.float64, device=torch.device("cuda", A.ctx.device))
    L.check(L.lib().pbcgs_jacobi_dinv(A.ctx.handle, A.handle, _ptr(d)), A.ctx.handle)
    return d


@dataclass
class SolveInfo:
    iters: int
    n_rr: int
    status: int
    syncs_per_iter: int
    relres_rec: float
    relres_true: float
    ms: float
    kernel_ms: tuple
    kernel_calls: tuple
    history: torch.Tensor | None = None
    shape: tuple = (0, 0)  # the launch shape that ran: (64-row blocks per wave, workgroups)
    value_codes: bool = False  # the layout's values were read as codes into per-diagonal tables

    @property
    def status_name(self) -> str:
        return STATUS.get(self.status, str(self.status))


def solve(A: Operator, b: torch.Tensor, x0: torch.Tensor | None = None, *, variant: str = "pbicgstab_rr",
          precond: str | None = None, dinv: torch.Tensor | None = None, tol: float = 1e-8, maxit: int = 2000,
          rr_period: int = 50, rr_max: int = -1, history: bool = False, check_every: int = 0,
          graph: bool = True, time_kernels: bool = False, out: torch.Tensor | None = None,
          precision: str = "fp64", alpha_form: int = 3, index32: bool = False, diagonal_layout: bool = True,
          poison: bool = False):
    """Solve A x = b; returns (x, SolveInfo).  x0 defaults to zero; ``out``
    (optional) receives the iterate in place of a new tensor.  ``alpha_form``
    5 takes alpha_{i+1} of the pipelined variants from eq. (5) instead of
    eq. (3) (Section 3.1).  ``index32`` reads the int32 column indices even
    where the operator holds a compact copy; ``diagonal_layout=False`` reads
    the CSR arrays even where the operator has a diagonal layout (same
    results either way).  ``poison`` (a test hook) fills the workspace with
    NaN bits before the solve writes it."""
    return _solve(L.lib().pbcgs_solve, A, b, x0, variant=variant, precond=precond, dinv=dinv, tol=tol,
                  maxit=maxit, rr_period=rr_period, rr_max=rr_max, history=history, check_every=check_every,
                  graph=graph, time_kernels=time_kernels, out=out, precision=precision, alpha_form=alpha_form,
                  index32=index32, diagonal_layout=diagonal_layout, poison=poison)


def solve_noalloc(A: Operator, b: torch.Tensor, x: torch.Tensor, *, variant: str = "pbicgstab_rr",
                  precond: str | None = None, dinv: torch.Tensor | None = None, tol: float = 1e-8,
                  maxit: int = 2000, rr_period: int = 50, rr_max: int = -1, history: torch.Tensor | None = None,
                  check_every: int = 0, alpha_form: int = 3, index32: bool = False, poison: bool = False):
    """``pbcgs_solve_noalloc``: the binary64 solve with every device buffer
    taken from the library's static scratch array, for callers that cannot
    allocate.  ``x`` holds x_0 and receives the iterate in place; ``history``
    (optional) is a caller-provided tensor of maxit + 1 doubles.  Nothing is
    allocated here either.  Returns (x, SolveInfo)."""
    return _solve(L.lib().pbcgs_solve_noalloc, A, b, None, variant=variant, precond=precond, dinv=dinv, tol=tol,
                  maxit=maxit, rr_period=rr_period, rr_max=rr_max, history=history, check_every=check_every,
                  graph=False, time_kernels=False, out=x, keep_x=True, precision="fp64", alpha_form=alpha_form,
                  index32=index32, poison=poison)


def _solve(entry, A: Operator, b: torch.Tensor, x0, *, variant, precond, dinv, tol, maxit, rr_period, rr_max,
           history, check_every, graph, time_kernels, out, precision, alpha_form, index32, keep_x=False,
           diagonal_layout=True, poison=False):
    _check_vec(b, A.n, "b")
    _check_alpha_form(alpha_form)
    if variant not in VARIANTS:
        raise ValueError(f"variant must be one of {sorted(VARIANTS)}")
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
    if precond not in PRECONDS:
        raise ValueError(f"precond must be one of {sorted(k for k in PRECONDS if k)} or None")
    if out is not None:
        _check_vec(out, A.n, "out")
        x = out
        if keep_x:
            pass  # the caller's x holds x_0
        elif x0 is None:
            x.zero_()
        else:
            x.copy_(x0)
    else:
        x = torch.zeros_like(b) if x0 is None else x0.clone()
    _check_vec(x, A.n, "x")
    if dinv is not None:
        _check_vec(dinv, A.n, "dinv")
    if isinstance(history, torch.Tensor):
        _check_vec(history, maxit + 1, "history")
        hist = history
    else:
        hist = torch.full((maxit + 1,), float("nan"), dtype=torch.float64, device=b.device) if history else None
    o = L.Opts()
    o.variant = VARIANTS[variant]
    o.precond = PRECONDS[precond]
    o.precision = PRECISIONS[precision]
    o.maxit = int(maxit)
    o.tol = float(tol)
    o.rr_period = int(rr_period)
    o.rr_max = int(rr_max)
    o.check_every = int(check_every)
    o.flags = ((0 if graph else L.FLAG_DIRECT) | (L.FLAG_TIME_KERNELS if time_kernels else 0)
               | (L.FLAG_ALPHA_EQ5 if alpha_form == 5 else 0) | (L.FLAG_INDEX32 if index32 else 0)
               | (0 if diagonal_layout else L.FLAG_NO_DIA) | (L.FLAG_POISON if poison else 0))
    o.history = hist.data_ptr() if hist is not None else None
    info = L.Info()
    L.check(entry(A.ctx.handle, A.handle, _ptr(b), _ptr(x), _ptr(dinv), ctypes.byref(o), ctypes.byref(info)),
            A.ctx.handle)
    si = SolveInfo(info.iters, info.n_rr, info.status, info.syncs_per_iter, info.relres_rec, info.relres_true,
                   info.ms, tuple(info.kernel_ms), tuple(info.kernel_calls))
    si.shape = (int(info.rows_per_wave_blocks), int(info.workgroups))
    si.value_codes = bool(info.value_codes)
    if hist is not None:
        si.history = hist[: info.iters + 1]
    return x, si


def solve_batched(ops: list, bs: list, x0s: list | None = None, *, variant: str = "pbicgstab_rr", tol: float = 1e-8,
                  maxit: int = 2000, rr_period: int = 50, rr_max: int = -1, check_every: int = 0, graph: bool = True,
                  outs: list | None = None, alpha_form: int = 3, index32: bool = False, diagonal_layout: bool = True,
                  poison: bool = False):
    """Solve the independent systems ops[k] x_k = bs[k] in one batched call
    (CSR operators of one context, no preconditioner, binary64).  Returns
    (xs, infos); each system's result equals its own :func:`solve` bit for bit.
    The batch reads every system through its diagonal layout when every
    operator has one (``diagonals > 0``) and neither ``index32`` nor
    ``diagonal_layout=False`` asks for the CSR arrays; else the int16 block
    offsets when every operator holds them (``column_form == "block16"``) and
    ``index32`` is false; else the int32 columns."""
    _check_alpha_form(alpha_form)
    nsys = len(ops)
    if nsys == 0 or len(bs) != nsys:
        raise ValueError("ops and bs must be non-empty lists of the same length")
    if variant not in VARIANTS:
        raise ValueError(f"variant must be one of {sorted(VARIANTS)}")
    ctx = ops[0].ctx
    xs = []
    for k, (A, b) in enumerate(zip(ops, bs)):
        if A.ctx is not ctx:
            raise ValueError("all operators must belong to one context")
        _check_vec(b, A.n, f"bs[{k}]")
        if outs is not None:
            x = outs[k]
            _check_vec(x, A.n, f"outs[{k}]")
            if x0s is None:
                x.zero_()
            else:
                x.copy_(x0s[k])
        else:
            x = torch.zeros_like(b) if x0s is None else x0s[k].clone()
        _check_vec(x, A.n, f"x[{k}]")
        xs.append(x)
    o = L.Opts()
    o.variant = VARIANTS[variant]
    o.precond = L.PRECOND_NONE
    o.precision = L.FP64
    o.maxit = int(maxit)
    o.tol = float(tol)
    o.rr_period = int(rr_period)
    o.rr_max = int(rr_max)
    o.check_every = int(check_every)
    o.flags = ((0 if graph else L.FLAG_DIRECT) | (L.FLAG_ALPHA_EQ5 if alpha_form == 5 else 0)
               | (L.FLAG_INDEX32 if index32 else 0) | (0 if diagonal_layout else L.FLAG_NO_DIA)
               | (L.FLAG_POISON if poison else 0))
    o.history = None
    VP = ctypes.c_void_p * nsys
    hs = VP(*[A.handle.value for A in ops])
    bp = VP(*[b.data_ptr() for b in bs])
    xp = VP(*[x.data_ptr() for x in xs])
    infos = (L.Info * nsys)()
    L.check(L.lib().pbcgs_solve_batched(ctx.handle, nsys, hs, bp, xp, ctypes.byref(o), infos), ctx.handle)
    out = [SolveInfo(i.iters, i.n_rr, i.status, i.syncs_per_iter, i.relres_rec, i.relres_true, i.ms,
                     tuple(i.kernel_ms), tuple(i.kernel_calls), shape=(int(i.rows_per_wave_blocks), int(i.workgroups)))
           for i in infos]
    return xs, out


class NotConvergedError(RuntimeError):
    """A solve inside :class:`SolveFn` ended without meeting its tolerance; the
    gradient it would feed is not the gradient of the loss."""

    def __init__(self, what: str, info: "SolveInfo"):
        super().__init__(f"{what} solve ended with status {info.status_name} after {info.iters} iterations "
                         f"(recursive relative residual {info.relres_rec:.3e})")
        self.info = info


def require_converged(info: "SolveInfo", what: str) -> None:
    """Raise :class:`NotConvergedError` unless the solve reported SUCCESS."""
    if info.status != L.SUCCESS:
        raise NotConvergedError(what, info)


class SolveFn(torch.autograd.Function):
    """x = A^{-1} b for the CSR matrix (row_ptr, col_idx, vals), differentiable
    in vals and b.  The backward pass is the adjoint solve with A^T on the
    same solver: lambda = A^{-T} dL/dx, dL/db = lambda, dL/dvals_k =
    -lambda_i x_j for the stored entry k = (i, j).  ``opts`` are keyword
    arguments of :func:`solve` (the adjoint solve uses them too, with
    ``adjoint_tol`` / ``adjoint_maxit`` in place of ``tol`` / ``maxit`` when
    given).  A forward or adjoint solve that ends without SUCCESS raises
    :class:`NotConvergedError` (its x or lambda would not give the gradient),
    unless ``allow_unconverged=True``."""

    @staticmethod
    def forward(ctx, vals, b, row_ptr, col_idx, opts):
        opts = dict(opts or {})
        adj = {k: opts.pop(f"adjoint_{k}") for k in ("tol", "maxit") if f"adjoint_{k}" in opts}
        lenient = bool(opts.pop("allow_unconverged", False))
        A = csr(row_ptr, col_idx, vals)
        x, info = solve(A, b, **opts)
        if not lenient:
            require_converged(info, "forward")
        ctx.save_for_backward(vals, row_ptr, col_idx, x)
        ctx.opts = opts
        ctx.adj = adj
        ctx.lenient = lenient
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        vals, row_ptr, col_idx, x = ctx.saved_tensors
        A = csr(row_ptr, col_idx, vals)
        AT = transpose(A)
        opts = dict(ctx.opts)
        opts.pop("x0", None)
        opts.pop("out", None)
        opts.update(ctx.adj)
        lam, info = solve(AT, gx.contiguous(), **opts)
        if not ctx.lenient:
            require_converged(info, "adjoint")
        gvals = csr_outer_grad(A, lam, x) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return gvals, gb, None, None, None


def solve_adjoint_batched(ops: list, gs: list, **kw):
    """lambda_k = A_k^{-T} g_k for a batch of CSR operators (one batched call on
    their transposes); returns (lambdas, infos, transposes)."""
    ts = [transpose(A) for A in ops]
    lams, infos = solve_batched(ts, gs, **kw)
    return lams, infos, ts


def _opts(variant="pbicgstab_rr", precond=None, precision="fp64", tol=1e-8, maxit=2000, rr_period=50, rr_max=-1,
          index32=False, diagonal_layout=True):
    o = L.Opts()
    o.variant = VARIANTS[variant]
    o.precond = PRECONDS[precond]
    o.precision = PRECISIONS[precision]
    o.maxit = int(maxit)
    o.tol = float(tol)
    o.rr_period = int(rr_period)
    o.rr_max = int(rr_max)
    o.check_every = 0
    o.flags = (L.FLAG_INDEX32 if index32 else 0) | (0 if diagonal_layout else L.FLAG_NO_DIA)
    o.history = None
    return o


def _report(r) -> dict:
    return {"best": r.best, "best_ms_per_iter": r.best_ms_per_iter,
            "tried": {int(r.cand[i]): float(r.ms_per_iter[i]) for i in range(r.ncand)}}


def tune(A: Operator, b: torch.Tensor, iters: int = 20, **opts) -> dict:
    """Time `iters` iterations for each launch shape (rows-per-wave blocks R)
    and keep the fastest on A, and in the process-wide launch-shape cache,
    for later solves of the same variant and precision; returns the report.  ``index32`` / ``diagonal_layout=False``
    time the solves on those read paths."""
    _check_vec(b, A.n, "b")
    o = _opts(**opts)
    r = L.TuneReport()
    L.check(L.lib().pbcgs_tune(A.ctx.handle, A.handle, _ptr(b), ctypes.byref(o), int(iters), ctypes.byref(r)),
            A.ctx.handle)
    return _report(r)


OP_KINDS = {0: "csr", 1: "stencil5", 2: "stencil7", 3: "convdiff27", 4: "stencil27", 5: "stencil_per_row"}
READ_PATHS = {0: "default", 1: "csr_arrays", 2: "int32_columns"}
_TUNE_CACHE_FORMAT = "pbcgs launch-shape cache"


def _entry_dict(e) -> dict:
    inv_v = {v: k for k, v in VARIANTS.items()}
    inv_p = {v: k for k, v in PRECISIONS.items()}
    return {"device": e.device.decode(), "build": e.build.decode(), "n": int(e.n), "nnz": int(e.nnz),
            "operator": OP_KINDS[e.op_kind], "variant": inv_v[e.variant], "precision": inv_p[e.precision],
            "read_path": READ_PATHS[e.read_path], "rows_per_wave_blocks": int(e.best)}


def tune_cache() -> list:
    """The process-wide launch-shape cache (``pbcgs_tune_entry``): one dict
    per entry, keyed by device, library build, rows, non-zeros, operator kind,
    variant and precision."""
    lib = L.lib()
    out = []
    for i in range(lib.pbcgs_tune_cache_size()):
        e = L.TuneEntry()
        L.check(lib.pbcgs_tune_cache_get(i, ctypes.byref(e)))
        out.append(_entry_dict(e))
    return out


def tune_cache_put(entry: dict) -> None:
    """Add one entry (a dict as :func:`tune_cache` returns them)."""
    kinds = {v: k for k, v in OP_KINDS.items()}
    paths = {v: k for k, v in READ_PATHS.items()}
    e = L.TuneEntry()
    e.device = str(entry["device"]).encode()[:63]
    e.build = str(entry["build"]).encode()[:31]
    e.n = int(entry["n"])
    e.nnz = int(entry["nnz"])
    e.op_kind = kinds[entry["operator"]]
    e.variant = VARIANTS[entry["variant"]]
    e.precision = PRECISIONS[entry["precision"]]
    e.read_path = paths[entry["read_path"]]
    e.best = int(entry["rows_per_wave_blocks"])
    L.check(L.lib().pbcgs_tune_cache_put(ctypes.byref(e)))


def tune_cache_clear() -> None:
    L.check(L.lib().pbcgs_tune_cache_clear())


def tune_cache_key(A: Operator, variant: str = "pbicgstab_rr", precision: str = "fp64", index32: bool = False,
                   diagonal_layout: bool = True) -> dict:
    """A's cache key for this variant, precision and read path, as a dict
    like :func:`tune_cache`'s entries; ``rows_per_wave_blocks`` holds the
    cached shape, or 0 when the cache has none."""
    flags = (L.FLAG_INDEX32 if index32 else 0) | (0 if diagonal_layout else L.FLAG_NO_DIA)
    e = L.TuneEntry()
    L.check(L.lib().pbcgs_tune_cache_key(A.ctx.handle, A.handle, VARIANTS[variant], PRECISIONS[precision], flags,
                                         ctypes.byref(e)), A.ctx.handle)
    return _entry_dict(e)


def tuned_shape(A: Operator, variant: str = "pbicgstab_rr", precision: str = "fp64", index32: bool = False,
                diagonal_layout: bool = True):
    """The cached shape (rows-per-wave blocks) of A's key for this variant,
    precision and read path, or None when the cache has none."""
    best = tune_cache_key(A, variant, precision, index32, diagonal_layout)["rows_per_wave_blocks"]
    return best if best > 0 else None


def save_tune_cache(path: str) -> int:
    """Write the cache to a JSON file; returns the number of entries."""
    import json
    import os

    entries = tune_cache()
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump({"format": _TUNE_CACHE_FORMAT, "version": 1, "entries": entries}, f, indent=1)
    os.replace(tmp, path)
    return len(entries)


def load_tune_cache(path: str) -> int:
    """Put the entries of a JSON file written by :func:`save_tune_cache`
    into the cache; returns how many were put (entries the library refuses
    are skipped).  A missing file puts nothing."""
    import json
    import os

    if not os.path.exists(path):
        return 0
    with open(path) as f:
        doc = json.load(f)
    if doc.get("format") != _TUNE_CACHE_FORMAT or doc.get("version") != 1:
        raise ValueError(f"{path} is not a launch-shape cache of this format")
    put = 0
    for entry in doc.get("entries", []):
        try:
            tune_cache_put(entry)
            put += 1
        except (L.PbcgsError, KeyError, TypeError, ValueError):
            continue
    return put


def tune_batched(ops: list, bs: list, iters: int = 20, **opts) -> dict:
    """The same for batched solves: the per-system workgroup cap, kept on the
    context.  ``iters=0`` times complete solves at the given tol and maxit
    (``tried`` then holds ms per whole batched solve)."""
    nsys = len(ops)
    ctx = ops[0].ctx
    VP = ctypes.c_void_p * nsys
    o = _opts(**opts)
    r = L.TuneReport()
    L.check(L.lib().pbcgs_tune_batched(ctx.handle, nsys, VP(*[A.handle.value for A in ops]),
                                       VP(*[b.data_ptr() for b in bs]), ctypes.byref(o), int(iters),
                                       ctypes.byref(r)), ctx.handle)
    return _report(r)
