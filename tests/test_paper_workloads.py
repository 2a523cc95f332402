"""The paper's parallel test problems (Section 5) solved by the oracle.

PTP1: five-point stencil [., -1, .; -1, 4, -eps; ., -eps, .], eps = 0.999;
PTP2: [., -1, .; -1, 1, -1; ., -1, .]; both on a 1000 x 1000 grid with exact
solution all ones, x_0 = 0, no preconditioner, tol 1e-6 on ||r_i||/||r_0||.
The paper reports 205-282 iterations for PTP1 (Figure 3 caption) and
1283-2112 for PTP2 (Table 4); its runs use 1-20 nodes, so rounding differs
from ours and only the range is a pin.  Which neighbour the paper draws north
does not matter: a reflection of the grid is a permutation similarity and
with the all-ones solution the iterates are permuted copies.
"""

import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle


def stencil5(n, center, west, east, south, north):
    """Five-point stencil on an n x n interior grid (rows x fastest, Dirichlet)."""
    N = n * n
    i = np.tile(np.arange(n), n)
    j = np.repeat(np.arange(n), n)
    diags = [np.full(N, center)]
    offs = [0]
    for off, val, ok in ((-1, west, i > 0), (1, east, i < n - 1), (-n, south, j > 0), (n, north, j < n - 1)):
        d = np.where(ok, val, 0.0)
        # scipy.sparse.diags wants the k-th diagonal aligned to its row for k<0
        diags.append(d[-off:] if off < 0 else d[:N - off])
        offs.append(off)
    S = sp.diags(diags, offs, shape=(N, N), format="csr")
    S.eliminate_zeros()
    S.sort_indices()
    return oracle.CSR(S.indptr, S.indices, S.data)


def ptp(which, n=1000):
    if which == "ptp1":
        eps = 1.0 - 0.001
        return stencil5(n, 4.0, -1.0, -eps, -eps, -1.0)
    return stencil5(n, 1.0, -1.0, -1.0, -1.0, -1.0)


@pytest.mark.slow
def test_ptp1_iterations_in_paper_range(golden_dir):
    with open(os.path.join(golden_dir, "paper_workloads.json")) as f:
        g = json.load(f)["ptp1"]
    A = ptp("ptp1")
    b = oracle.spmv(A, np.ones(A.n))
    for algo in (oracle.ALG_BICGSTAB, oracle.ALG_PBICGSTAB, oracle.ALG_PBICGSTAB_RR):
        x, info = oracle.solve(A, b, algo=algo, tol=g["tol"], maxit=2000, rr_period=100, rr_max=10)
        assert info["status"] == oracle.SUCCESS
        assert g["iterations_min"] <= info["iters"] <= g["iterations_max"], info


@pytest.mark.slow
def test_ptp2_iterations_in_paper_range(golden_dir):
    with open(os.path.join(golden_dir, "paper_workloads.json")) as f:
        g = json.load(f)["ptp2"]
    A = ptp("ptp2")
    b = oracle.spmv(A, np.ones(A.n))
    for algo in (oracle.ALG_BICGSTAB, oracle.ALG_PBICGSTAB):
        x, info = oracle.solve(A, b, algo=algo, tol=g["tol"], maxit=4000)
        assert info["status"] == oracle.SUCCESS
        assert g["iterations_min"] <= info["iters"] <= g["iterations_max"], info
        assert np.linalg.norm(b - oracle.spmv(A, x)) <= g["true_residual_max"]
