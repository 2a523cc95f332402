"""Pins of the oracle's adjoint pieces: the transpose by its definition, the
entry gradient -lambda x^T, and the adjoint gradient of a loss through
A x = b against dense linear algebra and finite differences."""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1612_01395_amd import inputs


def _mats():
    rng = np.random.default_rng(17)
    D = rng.standard_normal((40, 40)) * (rng.random((40, 40)) < 0.1)
    D[5, :] = 0.0   # an empty row
    D[:, 9] = 0.0   # an empty column
    R = sp.csr_matrix(D)
    R.sort_indices()
    return [oracle.assemble_workload(inputs.workload("c1", n=9)),
            oracle.assemble_workload(inputs.workload("c3", n=4), inputs.kappa_cells(4)),
            oracle.CSR(R.indptr, R.indices, R.data)]


@pytest.mark.parametrize("A", _mats(), ids=["c1_9", "c3_4", "random"])
def test_transpose_definition(A):
    T = oracle.transpose(A)
    S = A.to_scipy().T.tocsr()
    S.sort_indices()
    assert np.array_equal(T.row_ptr, S.indptr) and np.array_equal(T.col, S.indices)
    assert np.array_equal(T.val, S.data)
    assert np.array_equal(T.to_scipy().toarray(), A.to_scipy().toarray().T)
    TT = oracle.transpose(T)
    assert np.array_equal(TT.row_ptr, A.row_ptr) and np.array_equal(TT.col, A.col) and np.array_equal(TT.val, A.val)


def test_outer_grad_is_masked_dense_outer_product():
    A = _mats()[1]
    rng = np.random.default_rng(2)
    lam, x = rng.standard_normal(A.n), rng.standard_normal(A.n)
    g = oracle.outer_grad(A, lam, x)
    G = sp.csr_matrix((g, A.col, A.row_ptr), shape=(A.n, A.n)).toarray()
    mask = A.to_scipy().toarray() != 0
    assert np.array_equal(G[mask], (-np.outer(lam, x))[mask])


def test_adjoint_gradient_against_dense_reference_and_differences():
    A = oracle.assemble_workload(inputs.workload("c1", n=12))
    D = A.to_scipy().toarray()
    b = oracle.spmv(A, inputs.x_true(A.n))
    w = np.random.default_rng(8).standard_normal(A.n)
    x, _ = oracle.solve(A, b, algo=oracle.ALG_PBICGSTAB_RR, tol=1e-13, maxit=500, rr_period=10)
    lam, _ = oracle.solve(oracle.transpose(A), w, algo=oracle.ALG_PBICGSTAB_RR, tol=1e-13, maxit=500, rr_period=10)
    lam_ref = np.linalg.solve(D.T, w)
    assert np.linalg.norm(lam - lam_ref) <= 1e-9 * np.linalg.norm(lam_ref)
    # L = (w, x) is linear in b: central differences along a direction are exact up to rounding
    d = np.random.default_rng(9).standard_normal(A.n)
    eps = 1e-3
    Lp = w @ np.linalg.solve(D, b + eps * d)
    Lm = w @ np.linalg.solve(D, b - eps * d)
    assert abs((Lp - Lm) / (2 * eps) - lam @ d) <= 1e-8 * abs(lam @ d)
    # entry gradient against a dense difference of one stored value
    g = oracle.outer_grad(A, lam, x)
    k = A.row_ptr[40] + 1
    i, j = 40, A.col[k]
    E = np.zeros_like(D)
    E[i, j] = 1.0
    h = 1e-6
    fd = (w @ np.linalg.solve(D + h * E, b) - w @ np.linalg.solve(D - h * E, b)) / (2 * h)
    assert abs(g[k] - fd) <= 1e-6 * abs(fd)
