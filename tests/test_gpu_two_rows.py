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
def test_diagonal_layout(name, n, gtarget, monkeypatch):
    require_gpu()
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
