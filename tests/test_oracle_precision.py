"""Pins of the oracle's precision form (FP32 vectors, SpMV, recurrences and
dot products; FP64 residual replacement, x update and scalars).

The paper runs in one precision; the mixed form is a reading of its residual
replacement (Section 4.2) as the mechanism that restores accuracy lost in
the recurrences.  What mathematics fixes about it, and is checked here:

* binary32 building blocks: the pairwise binary32 sum on a hand-worked
  example whose value differs from both the sequential binary32 sum and the
  binary64 sum; a binary32 SpMV that is exact on small integers;
* a system where every binary32 operation is exact (A = 2I) gives the exact
  solution in one step, as in binary64;
* the first iterates follow the binary64 iterates to binary32 accuracy;
* without replacement the binary32 recurrences stall far above 1e-10
  (unit roundoff 6e-8); with binary64 replacement the true binary64 residual
  reaches 1e-10, and every SUCCESS is confirmed by it;
* a recursive residual that passes tol while the true one does not forces a
  replacement instead of a false SUCCESS.

The exact rounding sequence of the mixed form is pinned separately, operation
by operation, against an exact-rational twin with IEEE 754 rounding
(``test_oracle_precision_exact.py``).
"""

import json
import os

import numpy as np
import pytest

import oracle
from paper_1612_01395_amd import inputs


def test_dot32_pairwise_hand_worked(golden_dir):
    with open(os.path.join(golden_dir, "pairwise32_example.json")) as f:
        g = json.load(f)
    x = np.array(g["x"], dtype=np.float32)
    ones = np.ones_like(x)
    got = oracle.dot32(x, ones)
    assert got == g["pairwise_binary32"]
    assert got != g["sequential_binary32"] and got != g["binary64"]


def test_spmv32_exact_on_integers():
    rng = np.random.default_rng(11)
    D = rng.integers(-4, 5, (9, 9)) * (rng.random((9, 9)) < 0.5)
    import scipy.sparse as sp
    S = sp.csr_matrix(D.astype(np.float64))
    A = oracle.CSR(S.indptr, S.indices, S.data)
    x = rng.integers(-8, 9, 9).astype(np.float32)
    assert np.array_equal(oracle.spmv32(A, x), (D @ x.astype(np.int64)).astype(np.float32))


def test_exact_case_one_step():
    n = 6
    A = oracle.CSR(np.arange(n + 1), np.arange(n), np.full(n, 2.0))
    b = np.array([2.0, -4.0, 6.0, 8.0, -10.0, 12.0])
    x, info = oracle.solve_mp(A, b, tol=1e-12, rr_period=5)
    assert info["status"] == oracle.SUCCESS and info["iters"] == 1
    assert np.array_equal(x, b / 2)


@pytest.mark.parametrize("name,n", [("c1", 32), ("c2", 16)])
def test_first_iterates_follow_binary64(name, n):
    A = oracle.assemble_workload(inputs.workload(name, n=n))
    b = oracle.spmv(A, inputs.x_true(A.n))
    d = oracle.jacobi_dinv(A)
    for k in range(1, 6):
        x64, _ = oracle.solve_folded(A, b, algo=oracle.ALG_PBICGSTAB, dinv=d, tol=0.0, maxit=k)
        x32, i32 = oracle.solve_mp(A, b, dinv=d, tol=0.0, maxit=k, rr_period=0)
        assert i32["status"] == oracle.MAXIT
        assert np.linalg.norm(x32 - x64) <= 1e-5 * np.linalg.norm(x64)


@pytest.mark.parametrize("name,n", [("c1", 64), ("c2", 32)])
def test_replacement_restores_binary64_accuracy(name, n):
    A = oracle.assemble_workload(inputs.workload(name, n=n))
    xt = inputs.x_true(A.n)
    b = oracle.spmv(A, xt)
    d = oracle.jacobi_dinv(A)
    # binary32 recurrences alone stall far above 1e-10
    _, plain = oracle.solve_mp(A, b, dinv=d, tol=1e-10, maxit=600, rr_period=0, history=True)
    assert plain["status"] != oracle.SUCCESS
    assert plain["relres_true"] > 1e-8
    # with binary64 replacement the true residual reaches the tolerance
    x, info = oracle.solve_mp(A, b, dinv=d, tol=1e-10, maxit=4000, rr_period=20)
    assert info["status"] == oracle.SUCCESS
    assert info["relres_true"] <= 1e-10
    x64, i64 = oracle.solve_folded(A, b, algo=oracle.ALG_PBICGSTAB_RR, dinv=d, tol=1e-10, rr_period=20)
    D = A.to_scipy().toarray() if A.n <= 4096 else None
    kappa = np.linalg.cond(D) if D is not None else 1e4
    assert np.linalg.norm(x - x64) <= 10 * kappa * 1e-10 * np.linalg.norm(x64)


def test_recursive_convergence_is_confirmed():
    """Without periodic replacement, a binary32 recursive residual below tol
    is checked against the binary64 true residual; the solve only succeeds
    once the true residual is below tol too."""
    A = oracle.assemble_workload(inputs.workload("c2", n=24))
    b = oracle.spmv(A, inputs.x_true(A.n))
    d = oracle.jacobi_dinv(A)
    for tol in (1e-5, 3e-6):
        x, info = oracle.solve_mp(A, b, dinv=d, tol=tol, maxit=2000, rr_period=0, history=True)
        assert info["status"] == oracle.SUCCESS
        assert info["relres_true"] <= tol
        assert info["n_rr"] == 1  # the first recursive convergence was not confirmed: one forced replacement
    # binary32 p-BiCGStab without any replacement is not stable to tighter tolerances
    _, bad = oracle.solve_mp(A, b, dinv=d, tol=1e-7, maxit=2000, rr_period=0)
    assert bad["status"] != oracle.SUCCESS


def test_precision_form_alpha_eq5_is_less_robust():
    """Section 3.1 reports eq. (3) as the more robust alpha_{i+1}, notably with
    residual replacement.  In the precision form the 2-D problem shows it:
    eq. (3) converges, eq. (5) diverges to a non-finite scalar, and with
    Jacobi eq. (5) needs more than twice the iterations."""
    A = oracle.assemble_workload(inputs.workload("c1"))
    b = oracle.spmv(A, inputs.x_true(A.n))
    kw = dict(tol=1e-10, maxit=3000, rr_period=20)
    _, i3 = oracle.solve_mp(A, b, **kw)
    _, i5 = oracle.solve_mp(A, b, alpha_form=5, **kw)
    assert i3["status"] == oracle.SUCCESS and i5["status"] == oracle.NONFINITE
    dv = oracle.jacobi_dinv(A)
    _, j3 = oracle.solve_mp(A, b, dinv=dv, **kw)
    _, j5 = oracle.solve_mp(A, b, dinv=dv, alpha_form=5, **kw)
    assert j3["status"] == j5["status"] == oracle.SUCCESS and j5["iters"] > 2 * j3["iters"]
