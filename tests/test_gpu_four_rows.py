"""GPU parity of the binary32 kernels that take four neighbouring rows per lane.

When every wave owns at least four 64-row blocks, the precision form's fused
kernels on the diagonal layout let lane l of a 256-row block handle rows
4l .. 4l + 3: 16-byte binary32 accesses, the same arithmetic per row, and the
four rows' sum as a two-level subtree of the same reduction tree.  Row counts
of every residue modulo 4 (a last four with one, two or three rows), diagonal
offsets of every residue modulo 4 (aligned fours, aligned pairs, single loads)
with rows that miss diagonals, launch shapes with two and four rows per lane,
and the caller's x 8- and 16-byte aligned must all equal the oracle bit for
bit.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say

pytestmark = pytest.mark.gpu

# one offset of each residue modulo 4 on both sides, and a wide band
OFFSETS = (-41, -8, -6, -3, -1, 0, 1, 2, 4, 7, 37)


def banded(n, seed):
    """A random unsymmetric banded matrix, diagonally dominant, rows with
    ascending columns (entries outside [0, n) dropped), so it has a diagonal
    layout with the offsets above."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(n):
        for o in OFFSETS:
            j = i + o
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
                vals.append(float(len(OFFSETS)) + rng.uniform(0.5, 1.5) if o == 0 else rng.uniform(-1.0, 1.0))
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, np.asarray(rows) + 1, 1)
    return oracle.CSR(np.cumsum(rp).astype(np.int32), np.asarray(cols, np.int32), np.asarray(vals))


def _check(A, b, folded, monkeypatch, gtarget, four, out=None):
    monkeypatch.setenv("PBCGS_GTARGET", str(gtarget))
    monkeypatch.setenv("PBCGS_FOUR_ROWS", four)
    d = oracle.jacobi_dinv(A) if folded else None
    kw = dict(tol=1e-9, maxit=1500, rr_period=10)
    x_or, i_or = oracle.solve_mp(A, b, dinv=d, history=True, **kw)
    op = csr_op(A)
    assert op.diagonals > 0
    x, info = solver.solve(op, dev_t(b), variant="pbicgstab_rr", precond="jacobi_folded" if folded else None,
                           precision="fp32_rr64", history=True, out=out, **kw)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
    assert same(host(x), x_or), float(np.abs(host(x) - x_or).max())
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])
    assert same(host(info.history), i_or["history"])
    return info, x_or


@pytest.mark.parametrize("n", [1002, 1003, 1004, 1005, 4097])
@pytest.mark.parametrize("gtarget", [1, 2, 8])
@pytest.mark.parametrize("four", ["1", "0"])
def test_banded_every_residue(n, gtarget, four, monkeypatch):
    require_gpu()
    A = banded(n, seed=n)
    b = oracle.spmv(A, inputs.random_vector(n, 3))
    say(f"four rows={four}: banded n={n} (n mod 4 = {n % 4}) gtarget={gtarget}")
    for folded in (False, True):
        info, _ = _check(A, b, folded, monkeypatch, gtarget, four)
        R = info.shape[0]
        say(f"  folded={folded}: R={R} iters={info.iters} status={info.status_name}")
        if gtarget == 1:
            assert R >= 4  # one workgroup: every wave owns at least four blocks


@pytest.mark.parametrize("name,n", [("c2", 23), ("c1", 45), ("c3", 13), ("c2", 32), ("c1", 64)])
@pytest.mark.parametrize("gtarget", [1, 8])
def test_convection_diffusion(name, n, gtarget, monkeypatch):
    require_gpu()
    w = inputs.workload(name, n=n)
    A = oracle.assemble_workload(w, inputs.kappa_cells(n) if w.npts == 27 else None)
    b = oracle.spmv(A, inputs.x_true(A.n))
    say(f"four rows: {name} n={n} rows={A.n} gtarget={gtarget}")
    info, _ = _check(A, b, True, monkeypatch, gtarget, "1")
    say(f"  R={info.shape[0]} iters={info.iters}")


def test_caller_x_not_16_byte_aligned(monkeypatch):
    """x a view one element into a larger tensor (8-byte aligned only) is
    updated row by row, an aligned one by 16-byte pairs; both give the
    oracle's bits and leave the rest of the buffer alone."""
    require_gpu()
    A = banded(4097, seed=7)
    b = oracle.spmv(A, inputs.random_vector(A.n, 5))
    for shift in (1, 2):
        buf = torch.full((A.n + 3,), 7.0, dtype=torch.float64, device="cuda")
        out = buf[shift:shift + A.n]
        assert (out.data_ptr() % 16 == 0) == (shift == 2)
        say(f"four rows, x at element offset {shift}")
        _, x_or = _check(A, b, True, monkeypatch, 8, "1", out=out)
        assert same(host(out), x_or)
        hb = host(buf)
        assert (hb[:shift] == 7.0).all() and (hb[shift + A.n:] == 7.0).all()
