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
