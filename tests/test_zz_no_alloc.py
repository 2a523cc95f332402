"""pbcgs_solve_noalloc against pbcgs_solve, through the C ABI.

The entry point for callers that cannot allocate takes every device buffer
of the solve from the library's static scratch array.  It runs the same
kernels, so its results must equal pbcgs_solve's bit for bit: the iterate,
counts, status, residuals and the residual history.  Two calls in a row use
the same array, the second on a smaller system than the first, so stale
contents of the first call must not leak into the second.  The size limit and
the refused options return errors without touching x.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1612_01395_amd import _lib as L
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say, stencil_coefs

pytestmark = pytest.mark.gpu

POOL = 1 << 23  # doubles of the scratch pool for vectors and folded values


def _system(name, n):
    A = oracle.assemble_workload(inputs.workload(name, n=n))
    b = oracle.spmv(A, inputs.x_true(A.n))
    return A, b


def _pair(op, b, kw, maxit):
    """(x, info, history) of pbcgs_solve and of pbcgs_solve_noalloc."""
    bd = dev_t(b)
    x_ref, i_ref = solver.solve(op, bd, maxit=maxit, history=True, **kw)
    x = torch.zeros_like(bd)
    hist = torch.full((maxit + 1,), float("nan"), dtype=torch.float64, device=bd.device)
    x_na, i_na = solver.solve_noalloc(op, bd, x, maxit=maxit, history=hist, **kw)
    assert x_na.data_ptr() == x.data_ptr()
    return (host(x_ref), i_ref, host(i_ref.history)), (host(x_na), i_na, host(i_na.history))


def _assert_same(ref, got):
    (xr, ir, hr), (xg, ig, hg) = ref, got
    assert (ig.iters, ig.n_rr, ig.status) == (ir.iters, ir.n_rr, ir.status)
    assert ig.relres_rec == ir.relres_rec and ig.relres_true == ir.relres_true
    assert same(xg, xr)
    assert same(hg, hr)


@pytest.mark.parametrize("kw", [
    dict(variant="pbicgstab_rr", precond="jacobi_folded", tol=1e-10, rr_period=20),
    dict(variant="pbicgstab", precond="jacobi", tol=1e-9),
    dict(variant="bicgstab", precond=None, tol=1e-9),
])
def test_two_calls_in_a_row_second_smaller(kw):
    require_gpu()
    big, b_big = _system("c2", 40)     # 64,000 rows, 3-D 7-point
    small, b_small = _system("c1", 23)  # 529 rows, 2-D 5-point (ragged last block)
    say(f"noalloc {kw} rows {big.n} then {small.n}")
    op_big, op_small = csr_op(big), csr_op(small)
    r1 = _pair(op_big, b_big, kw, 600)
    r2 = _pair(op_small, b_small, kw, 600)
    _assert_same(*r1)
    _assert_same(*r2)
    assert r1[0][1].status == r2[0][1].status == solver.L.SUCCESS
    # the normal entry point still works on the context afterwards, with the same bits
    x_again, i_again = solver.solve(op_small, dev_t(b_small), maxit=600, **kw)
    assert same(host(x_again), r2[0][0]) and i_again.iters == r2[0][1].iters


def test_stencil_and_other_variants():
    require_gpu()
    A, b = _system("c2", 24)
    say(f"noalloc stencil rows {A.n}")
    st = solver.stencil(24, 24, 24, stencil_coefs(A, 3, 24))
    for kw in (dict(variant="pbicgstab_rr", precond="jacobi_folded", tol=1e-10, rr_period=7),
               dict(variant="ca_bicgstab", precond="jacobi_folded", tol=1e-10),
               dict(variant="pipe_cg", precond="jacobi", tol=1e-10)):
        if kw["variant"] == "pipe_cg":
            S = oracle.assemble_workload(inputs.workload("c2s", n=24))
            op, bb = csr_op(S), oracle.spmv(S, inputs.x_true(S.n))
        else:
            op, bb = st, b
        ref, got = _pair(op, bb, kw, 400)
        _assert_same(ref, got)


def test_limits_and_refusals_leave_x_untouched():
    require_gpu()
    # 14 vectors of 128^3 rows exceed the pool
    n = 128
    assert 14 * n ** 3 > POOL
    A, b = _system("c2", n)
    op = csr_op(A)
    x = dev_t(np.full(A.n, 0.5))
    with pytest.raises(L.PbcgsError) as e:
        solver.solve_noalloc(op, dev_t(b), x, precond="jacobi_folded")
    assert e.value.code == L.ERR_UNSUPPORTED and "scratch" in str(e.value)
    # folded CSR counts one double per non-zero on top: 80^3 fits unfolded, not folded
    A80, b80 = _system("c2", 80)
    op80 = csr_op(A80)
    assert 14 * A80.n <= POOL < 14 * A80.n + A80.nnz
    x80 = torch.zeros(A80.n, dtype=torch.float64, device="cuda")
    with pytest.raises(L.PbcgsError):
        solver.solve_noalloc(op80, dev_t(b80), x80, precond="jacobi_folded")
    xs, info = solver.solve_noalloc(op80, dev_t(b80), x80, precond="jacobi", tol=1e-8)
    ref, iref = solver.solve(op80, dev_t(b80), precond="jacobi", tol=1e-8)
    assert same(host(xs), host(ref)) and info.iters == iref.iters
    # refused options: the precision form and kernel timing
    small, bs = _system("c1", 16)
    ops = csr_op(small)
    o = L.Opts()
    o.variant, o.precond, o.precision, o.maxit, o.tol = L.PBICGSTAB_RR, L.PRECOND_NONE, L.FP32_RR64, 50, 1e-8
    o.rr_period, o.rr_max = 10, -1
    info = L.Info()
    bd = dev_t(bs)
    xs = torch.full_like(bd, 0.25)
    rc = L.lib().pbcgs_solve_noalloc(ops.ctx.handle, ops.handle, solver._ptr(bd), solver._ptr(xs), None, o, info)
    assert rc == L.ERR_UNSUPPORTED
    o.precision, o.flags = L.FP64, L.FLAG_TIME_KERNELS
    rc = L.lib().pbcgs_solve_noalloc(ops.ctx.handle, ops.handle, solver._ptr(bd), solver._ptr(xs), None, o, info)
    assert rc == L.ERR_UNSUPPORTED
    assert bool((xs == 0.25).all()) and bool((x == 0.5).all())
