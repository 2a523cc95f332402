"""Seeded randomized parity: the HIP path against the oracle on random systems.

Each case draws a sparse system of a random size (1 to a few thousand rows, so
most sizes leave a ragged last 64-row block and a ragged last workgroup), a
random pattern and values, and random solver options (variant, Jacobi form,
tolerance, iteration budget, replacement period, x0, alpha form), then asserts
that the library reproduces the oracle's iterate, counts, status and residual
history bit for bit.  Unsymmetric cases run the BiCGStab variants; symmetric
positive definite cases run the CG family.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR,
       "ca_bicgstab": oracle.ALG_CA_BICGSTAB, "cg": oracle.ALG_CG, "cgcg": oracle.ALG_CGCG,
       "pipe_cg": oracle.ALG_PIPE_CG}


def random_system(rng, spd):
    n = int(rng.choice([1, 2, 3, 63, 64, 65, 127, 200, 511, 1000, 2049, 3001]))
    density = min(1.0, rng.uniform(2.0, 9.0) / n)
    M = sp.random(n, n, density=density, random_state=rng, data_rvs=lambda k: rng.uniform(-1.0, 1.0, k)).tocsr()
    if spd:
        M = M + M.T
    # diagonal dominance keeps every variant convergent; a varying diagonal
    # makes Jacobi a true vector
    rowsum = np.asarray(abs(M).sum(axis=1)).ravel()
    d = rowsum * rng.uniform(1.05, 2.0, n) + rng.uniform(0.1, 1.0, n)
    M = (M + sp.diags(d)).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    return oracle.CSR(M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


def run_case(seed):
    rng = np.random.default_rng(1000 + seed)
    spd = bool(seed % 3 == 2)
    A = random_system(rng, spd)
    if spd:
        variant = str(rng.choice(["cg", "cgcg", "pipe_cg"]))
        precond = [None, "jacobi"][int(rng.integers(2))]
    else:
        variant = str(rng.choice(["bicgstab", "pbicgstab", "pbicgstab_rr", "ca_bicgstab"]))
        choices = [None, "jacobi_folded"] if variant == "ca_bicgstab" else [None, "jacobi", "jacobi_folded"]
        precond = choices[int(rng.integers(len(choices)))]
    tol = float(rng.choice([0.0, 1e-6, 1e-10, 1e-13]))
    maxit = int(rng.choice([0, 1, 5, 40, 500]))
    rr = int(rng.choice([1, 3, 7, 50]))
    alpha_form = 5 if (variant in ("pbicgstab", "pbicgstab_rr", "ca_bicgstab") and rng.random() < 0.3) else 3
    x0 = rng.standard_normal(A.n) if rng.random() < 0.4 else None
    b = rng.standard_normal(A.n) * 10.0 ** rng.uniform(-3, 3)
    say(f"random case {seed}: n={A.n} nnz={len(A.val)} {variant} precond={precond} tol={tol} maxit={maxit} "
        f"rr={rr} alpha=eq.({alpha_form}) x0={x0 is not None}")
    dv = oracle.jacobi_dinv(A) if precond else None
    kw = dict(tol=tol, maxit=maxit, rr_period=rr, history=True, alpha_form=alpha_form)
    if precond == "jacobi_folded":
        x_or, i_or = oracle.solve_folded(A, b, algo=ALG[variant], dinv=dv, x0=x0, **kw)
    else:
        x_or, i_or = oracle.solve(A, b, algo=ALG[variant], dinv=dv, x0=x0, **kw)
    x, info = solver.solve(csr_op(A), dev_t(b), None if x0 is None else dev_t(x0), variant=variant,
                           precond=precond, **kw)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
    assert same(host(x), x_or), float(np.nanmax(np.abs(host(x) - x_or)))
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])
    assert same(host(info.history), i_or["history"])


@pytest.mark.parametrize("seed", range(60))
def test_random_system_bitwise(seed):
    require_gpu()
    run_case(seed)


def random_banded_system(rng, spd):
    """A random system of 33,000 to 80,000 rows whose entries lie on a random
    set of diagonals, some of them beyond the int16 block offsets: with up to
    64 diagonals the operator holds diagonal codes, with more it keeps int32
    columns.  Diagonally dominant (symmetric with `spd`)."""
    n = int(rng.integers(33000, 80001))
    ndiag = int(rng.choice([3, 8, 20, 40, 63, 70]))
    half = max(1, ndiag // 2)
    offs = set()
    while len(offs) < half:
        offs.add(int(rng.choice([rng.integers(1, 200), rng.integers(32800, n - 1)])))
    nneg = half if (spd or ndiag >= 63) else max(1, half // 2)  # mirrored offsets
    diags = sorted(offs | {-int(d) for d in rng.choice(sorted(offs), size=nneg, replace=False)} | {0})
    rows, cols, vals = [], [], []
    for d in diags:
        r = np.arange(max(0, -d), min(n, n - d))
        if d != 0:
            r = r[rng.random(r.size) < 0.7]
        rows.append(r)
        cols.append(r + d)
        vals.append(rng.uniform(-1.0, 1.0, r.size))
    r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    M = sp.csr_matrix((v, (r, c)), shape=(n, n))
    if spd:
        M = M + M.T
    rowsum = np.asarray(abs(M).sum(axis=1)).ravel()
    M = (M + sp.diags(rowsum * rng.uniform(1.05, 2.0, n) + rng.uniform(0.1, 1.0, n))).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    return oracle.CSR(M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.astype(np.float64))


def expected_form(A):
    """The column form the library must choose, computed on the host."""
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    off = A.col.astype(np.int64) - (rows & ~63)
    if off.min() >= -32768 and off.max() <= 32767:
        return "block16"
    return "diag16" if np.unique(A.col.astype(np.int64) - rows).size <= 64 else "int32"


@pytest.mark.parametrize("seed", range(16))
def test_random_wide_system_bitwise(seed):
    """Random wide-band systems: the form the operator picks (diagonal codes or
    int32) matches the host's prediction, and solves equal the oracle's bit for
    bit in that form and with ``index32``."""
    require_gpu()
    rng = np.random.default_rng(5000 + seed)
    spd = bool(seed % 4 == 3)
    A = random_banded_system(rng, spd)
    form = expected_form(A)
    variant = str(rng.choice(["cg", "pipe_cg"] if spd else ["bicgstab", "pbicgstab_rr", "ca_bicgstab"]))
    precond = "jacobi" if spd else str(rng.choice(["jacobi_folded", "none"]))
    precond = None if precond == "none" else precond
    tol, maxit, rr = 1e-10, int(rng.choice([7, 60, 400])), int(rng.choice([5, 50]))
    b = rng.standard_normal(A.n)
    say(f"random wide case {seed}: n={A.n} nnz={len(A.val)} form={form} {variant} precond={precond} maxit={maxit}")
    op = csr_op(A)
    assert op.column_form == form
    dv = oracle.jacobi_dinv(A) if precond else None
    kw = dict(tol=tol, maxit=maxit, rr_period=rr, history=True)
    if precond == "jacobi_folded":
        x_or, i_or = oracle.solve_folded(A, b, algo=ALG[variant], dinv=dv, **kw)
    else:
        x_or, i_or = oracle.solve(A, b, algo=ALG[variant], dinv=dv, **kw)
    for index32 in (False, True):
        x, info = solver.solve(op, dev_t(b), variant=variant, precond=precond, index32=index32, **kw)
        assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
        assert same(host(x), x_or), (index32, float(np.nanmax(np.abs(host(x) - x_or))))
        assert same(host(info.history), i_or["history"])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_unsorted_columns_follow_stored_order(seed):
    """Columns need not be ascending within a row: every product sums a row in
    stored order, as the oracle does, so results equal the oracle's on the same
    arrays bit for bit (and differ in rounding from the sorted matrix).  The
    compact column copies keep each entry's column whatever the order."""
    require_gpu()
    rng = np.random.default_rng(400 + seed)
    A = random_system(rng, False)
    col, val = A.col.copy(), A.val.copy()
    for i in range(A.n):  # reverse or shuffle each row's entries
        lo, hi = A.row_ptr[i], A.row_ptr[i + 1]
        perm = rng.permutation(hi - lo) if seed % 2 else np.arange(hi - lo)[::-1]
        col[lo:hi], val[lo:hi] = col[lo:hi][perm], val[lo:hi][perm]
    U = oracle.CSR(A.row_ptr, col, val)
    say(f"unsorted n={U.n} nnz={U.nnz}")
    op = csr_op(U)
    x = inputs.random_vector(U.n, 5)
    assert same(host(solver.spmv(op, dev_t(x))), oracle.spmv(U, x))
    b = oracle.spmv(U, inputs.x_true(U.n))
    kw = dict(tol=1e-10, maxit=500, rr_period=9)
    xg, info = solver.solve(op, dev_t(b), variant="pbicgstab_rr", precond="jacobi_folded", **kw)
    d = oracle.jacobi_dinv(U)
    xo, io = oracle.solve_folded(U, b, algo=oracle.ALG_PBICGSTAB_RR, dinv=d, **kw)
    assert (info.status, info.iters, info.n_rr) == (io["status"], io["iters"], io["n_rr"])
    assert same(host(xg), xo)
    xi, _ = solver.solve(op, dev_t(b), variant="pbicgstab_rr", precond="jacobi_folded", index32=True, **kw)
    assert same(host(xi), xo)
