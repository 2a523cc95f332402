"""GPU parity of the kernels that take two neighbouring rows per lane.

When every wave owns at least two 64-row blocks, the binary32 fused kernels of
the precision form, the five BiCGStab kernels and (on the diagonal layout) the
two p-BiCGStab fused kernels let each lane handle rows 2l and 2l + 1 of a
128-row block: wider vector accesses, the same arithmetic per row, and the
pair's sum as the bottom node of the same reduction tree.  Launch shapes that
force it (few workgroups, so many blocks per wave), row counts odd (a last
pair with a single row) and even, on the diagonal layout and on the
matrix-free stencils, must equal the oracle bit for bit.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say, stencil_coefs

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR}


def _check(op, A, b, gtarget, monkeypatch):
    monkeypatch.setenv("PBCGS_GTARGET", str(gtarget))
    d = oracle.jacobi_dinv(A)
    x, info = solver.solve(op, dev_t(b), variant="pbicgstab_rr", precond="jacobi_folded", precision="fp32_rr64",
                           tol=1e-10, maxit=2000, rr_period=10, history=True)
    x_or, i_or = oracle.solve_mp(A, b, dinv=d, tol=1e-10, maxit=2000, rr_period=10, history=True)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
    assert same(host(x), x_or)
    assert same(host(info.history), i_or["history"])
    for variant in ("pbicgstab_rr", "pbicgstab", "bicgstab"):
        x, info = solver.solve(op, dev_t(b), variant=variant, precond="jacobi_folded", tol=1e-10, maxit=2000,
                               rr_period=7, history=True)
        x_or, i_or = oracle.solve_folded(A, b, algo=ALG[variant], dinv=d, tol=1e-10, maxit=2000, rr_period=7,
                                         history=True)
        assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
        assert same(host(x), x_or)
        assert same(host(info.history), i_or["history"])


@pytest.mark.parametrize("name,n", [("c2", 23), ("c1", 45), ("c3", 13), ("c2", 32)])
@pytest.mark.parametrize("gtarget", [8, 64, 1024])
@pytest.mark.parametrize("cached", ["0", "1"])
def test_diagonal_layout(name, n, gtarget, cached, monkeypatch):
    require_gpu()
    monkeypatch.setenv("PBCGS_DIA_CACHED", cached)
    w = inputs.workload(name, n=n)
    A = oracle.assemble_workload(w, inputs.kappa_cells(n) if w.npts == 27 else None)
    b = oracle.spmv(A, inputs.x_true(A.n))
    op = csr_op(A)
    assert op.diagonals > 0
    say(f"two rows, diagonal layout {name} n={n} rows={A.n} gtarget={gtarget}")
    _check(op, A, b, gtarget, monkeypatch)


@pytest.mark.parametrize("name,n", [("c2", 23), ("c1", 45), ("c2", 32)])
@pytest.mark.parametrize("gtarget", [8, 64])
def test_stencil(name, n, gtarget, monkeypatch):
    require_gpu()
    w = inputs.workload(name, n=n)
    A = oracle.assemble_workload(w)
    b = oracle.spmv(A, inputs.x_true(A.n))
    st = solver.stencil(n, n, n if w.dim == 3 else 1, stencil_coefs(A, w.dim, n))
    say(f"two rows, stencil {name} n={n} rows={A.n} gtarget={gtarget}")
    _check(st, A, b, gtarget, monkeypatch)


@pytest.mark.parametrize("precision,variant", [("fp64", "pbicgstab_rr"), ("fp64", "bicgstab"),
                                               ("fp32_rr64", "pbicgstab_rr")])
def test_caller_x_not_16_byte_aligned(precision, variant, monkeypatch):
    """The iterate lives in the caller's buffer: a view one element into a
    larger tensor (8-byte aligned only) is updated row by row, an aligned one
    by 16-byte pairs; both give the oracle's bits."""
    require_gpu()
    monkeypatch.setenv("PBCGS_GTARGET", "8")
    w = inputs.workload("c2", n=23)
    A = oracle.assemble_workload(w)
    b = oracle.spmv(A, inputs.x_true(A.n))
    op = csr_op(A)
    d = oracle.jacobi_dinv(A)
    kw = dict(tol=1e-10, maxit=2000, rr_period=10)
    if precision == "fp64":
        x_or, i_or = oracle.solve_folded(A, b, algo=ALG[variant], dinv=d, **kw)
    else:
        x_or, i_or = oracle.solve_mp(A, b, dinv=d, **kw)
    for shift in (1, 2):
        buf = torch.full((A.n + 3,), 7.0, dtype=torch.float64, device="cuda")
        out = buf[shift:shift + A.n]
        assert (out.data_ptr() % 16 == 0) == (shift == 2)
        say(f"two rows, x at element offset {shift}, {precision} {variant}")
        x, info = solver.solve(op, dev_t(b), variant=variant, precond="jacobi_folded", precision=precision,
                               out=out, **kw)
        assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
        assert same(host(out), x_or)
        hb = host(buf)
        assert (hb[:shift] == 7.0).all() and (hb[shift + A.n:] == 7.0).all()
