"""GPU parity of the diagonal layout of CSR operators (``pbcgs_op_diagonals``).

A CSR operator with at most 32 distinct diagonals, rows stored with strictly
ascending columns and few empty slots is read by the solves through a
diagonal-by-diagonal copy of its values and a per-row mask of the diagonals the
row holds.  Each row is still summed over its own entries in ascending column
order, so every solve must equal the oracle bit for bit, and equal the same
solve read through the CSR arrays (``diagonal_layout=False``):

* which operators get the layout: the 5-, 7- and 27-point workloads (5, 7, 27
  diagonals) do; a matrix with 33 diagonals, one with a reversed row, one with
  mostly empty diagonals and a random sparse matrix do not;
* every BiCGStab variant with no, literal and folded Jacobi, CA-BiCGStab, the
  CG family and the precision form (binary32 values laid out from the folded
  binary64 ones) on 2-D and 3-D systems with ragged last blocks;
* values changed in place between solves (the layout's values are copied for
  each solve);
* the values read with ordinary loads and with the nontemporal hint (chosen
  by the working set's size; both forced here);
* exactly 32 diagonals, the widest layout.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR,
       "ca_bicgstab": oracle.ALG_CA_BICGSTAB, "cg": oracle.ALG_CG, "cgcg": oracle.ALG_CGCG,
       "pipe_cg": oracle.ALG_PIPE_CG}


def banded(n, offsets, fill=1.0, seed=0):
    """Matrix with the given diagonals (each kept where it fits, a fraction
    ``fill`` of its entries present), diagonally dominant, ascending columns."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for d in offsets:
        i = np.arange(max(0, -d), min(n, n - d))
        if fill < 1.0:
            i = i[rng.random(len(i)) < fill]
        rows.append(i)
        cols.append(i + d)
    r, c = np.concatenate(rows), np.concatenate(cols)
    v = rng.uniform(-1.0, 1.0, len(r))
    M = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    M = M + sp.diags(np.asarray(abs(M).sum(axis=1)).ravel() + 1.0)
    M = M.tocsr()
    M.sort_indices()
    return oracle.CSR(M.indptr, M.indices, M.data)


def systems():
    return {
        "c1": oracle.assemble_workload(inputs.workload("c1")),
        "c2_24": oracle.assemble_workload(inputs.workload("c2", n=24)),
        "c3_10": oracle.assemble_workload(inputs.workload("c3", n=10), inputs.kappa_cells(10)),
        "band32": banded(5000, list(range(-40, 41, 3))[:16] + list(range(1, 33, 2))),
    }


SYS = systems()


def test_which_operators_get_the_layout():
    require_gpu()
    want = {"c1": 5, "c2_24": 7, "c3_10": 27, "band32": 32}
    for name, A in SYS.items():
        assert csr_op(A).diagonals == want[name], name
    B = SYS["band32"]
    assert len(set(B.col - np.repeat(np.arange(B.n), np.diff(B.row_ptr)))) == 32
    # 33 diagonals, mostly empty diagonals, a random pattern: no layout
    assert csr_op(banded(3000, list(range(-16, 17)))).diagonals == 0
    assert csr_op(banded(3000, [-7, -1, 0, 1, 7], fill=0.3)).diagonals == 0
    R = sp.random(2000, 2000, density=0.004, random_state=np.random.default_rng(1)).tocsr() + sp.eye(2000)
    R = R.tocsr()
    R.sort_indices()
    assert csr_op(oracle.CSR(R.indptr, R.indices, R.data)).diagonals == 0
    # one row with descending columns: no layout, and the CSR stream sums it in stored order
    A = SYS["c2_24"]
    col, val = A.col.copy(), A.val.copy()
    lo, hi = A.row_ptr[100], A.row_ptr[101]
    col[lo:hi], val[lo:hi] = col[lo:hi][::-1], val[lo:hi][::-1]
    U = oracle.CSR(A.row_ptr, col, val)
    op = csr_op(U)
    assert op.diagonals == 0
    x = inputs.random_vector(U.n, 2)
    assert same(host(solver.spmv(op, dev_t(x))), oracle.spmv(U, x))


CASES = [
    ("pbicgstab_rr", "jacobi_folded", 7), ("pbicgstab_rr", "jacobi", 5), ("pbicgstab_rr", None, 11),
    ("pbicgstab", "jacobi_folded", 0), ("bicgstab", "jacobi_folded", 0), ("bicgstab", "jacobi", 0),
    ("bicgstab", None, 0), ("ca_bicgstab", "jacobi_folded", 0),
]


@pytest.mark.parametrize("cached", ["0", "1"])
@pytest.mark.parametrize("name", ["c1", "c2_24", "c3_10", "band32"])
@pytest.mark.parametrize("variant,precond,k", CASES)
def test_solves_bitwise(name, variant, precond, k, cached, monkeypatch):
    """cached: the layout's values read with ordinary loads (1) or with the
    nontemporal hint (0); the choice is by working-set size, forced here."""
    require_gpu()
    monkeypatch.setenv("PBCGS_DIA_CACHED", cached)
    A = SYS[name]
    b = oracle.spmv(A, inputs.x_true(A.n))
    op = csr_op(A)
    assert op.diagonals > 0
    say(f"dia {name} {variant} {precond} k={k}")
    kw = dict(tol=1e-10, maxit=600, rr_period=k)
    x, info = solver.solve(op, dev_t(b), variant=variant, precond=precond, history=True, **kw)
    d = oracle.jacobi_dinv(A)
    if precond == "jacobi_folded":
        x_or, i_or = oracle.solve_folded(A, b, algo=ALG[variant], dinv=d, history=True, **kw)
    else:
        x_or, i_or = oracle.solve(A, b, algo=ALG[variant], dinv=d if precond else None, history=True, **kw)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
    assert same(host(x), x_or)
    assert same(host(info.history), i_or["history"])
    xc, ic = solver.solve(op, dev_t(b), variant=variant, precond=precond, diagonal_layout=False, **kw)
    assert same(host(xc), x_or) and ic.iters == info.iters


@pytest.mark.parametrize("variant", ["cg", "cgcg", "pipe_cg"])
def test_cg_family_bitwise(variant):
    require_gpu()
    A = oracle.assemble_workload(inputs.workload("c2s", n=20))
    b = oracle.spmv(A, inputs.x_true(A.n))
    op = csr_op(A)
    assert op.diagonals == 7
    x, info = solver.solve(op, dev_t(b), variant=variant, precond="jacobi", tol=1e-10, maxit=500)
    x_or, i_or = oracle.solve(A, b, algo=ALG[variant], dinv=oracle.jacobi_dinv(A), tol=1e-10, maxit=500)
    assert (info.status, info.iters) == (i_or["status"], i_or["iters"])
    assert same(host(x), x_or)


@pytest.mark.parametrize("name", ["c1", "c2_24", "c3_10"])
@pytest.mark.parametrize("precond", ["jacobi_folded", None])
def test_precision_form_bitwise(name, precond):
    require_gpu()
    A = SYS[name]
    b = oracle.spmv(A, inputs.x_true(A.n))
    op = csr_op(A)
    say(f"dia precision form {name} {precond}")
    d = oracle.jacobi_dinv(A) if precond else None
    x, info = solver.solve(op, dev_t(b), variant="pbicgstab_rr", precond=precond, precision="fp32_rr64",
                           tol=1e-10, maxit=2000, rr_period=10, history=True)
    x_or, i_or = oracle.solve_mp(A, b, dinv=d, tol=1e-10, maxit=2000, rr_period=10, history=True)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
    assert same(host(x), x_or)
    assert same(host(info.history), i_or["history"])


def test_values_changed_between_solves():
    require_gpu()
    A = SYS["c2_24"]
    rp, col, val = dev_t(A.row_ptr), dev_t(A.col), dev_t(A.val)
    op = solver.csr(rp, col, val)
    b = oracle.spmv(A, inputs.x_true(A.n))
    kw = dict(variant="pbicgstab_rr", precond="jacobi_folded", tol=1e-10, maxit=400, rr_period=20)
    x1, _ = solver.solve(op, dev_t(b), **kw)
    val.mul_(1.25)
    torch.cuda.synchronize()
    A2 = oracle.CSR(A.row_ptr, A.col, A.val * 1.25)
    b2 = oracle.spmv(A2, inputs.x_true(A.n))
    x2, i2 = solver.solve(op, dev_t(b2), **kw)
    x_or, i_or = oracle.solve_folded(A2, b2, algo=oracle.ALG_PBICGSTAB_RR, dinv=oracle.jacobi_dinv(A2), tol=1e-10,
                                     maxit=400, rr_period=20)
    assert i2.iters == i_or["iters"] and same(host(x2), x_or)
