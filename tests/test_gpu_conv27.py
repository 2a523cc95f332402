"""GPU parity of the matrix-free 27-point variable-coefficient operator
(``pbcgs_op_convdiff27``) against the oracle, through the C ABI.

The operator forms every entry from the cell coefficients in the order the
workload's assembly does and sums each row in ascending column order, so it
must reproduce the oracle's assembled CSR matrix bit for bit in every use:

* products at grid sides 1 to 17 (a single node, all-boundary grids, ragged
  last 64-row blocks), convection in both directions on each axis and with
  zero components, with and without a diagonal shift;
* Jacobi (dinv = 1 / a_ii from the formed diagonal) and the folded operator
  A M^{-1} (each entry scaled by dinv_j as it is formed);
* complete solves of every BiCGStab variant with no, literal and folded
  Jacobi, CA-BiCGStab, the CG family on the symmetric (beta = 0) operator and
  the precision form, against the oracle's solves;
* at the full 256^3 size (16,777,216 rows, 449,455,096 equivalent
  non-zeros): products of sampled row ranges against the oracle's row-range
  assembly, and the complete folded p-BiCGStab+RR solve the benchmark times
  against the oracle's, bit for bit;
* the refused uses (transpose, batched) and bad arguments.
"""

import time

import numpy as np
import pytest
import torch

import oracle
from paper_1612_01395_amd import _lib as L
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR,
       "ca_bicgstab": oracle.ALG_CA_BICGSTAB, "cg": oracle.ALG_CG, "cgcg": oracle.ALG_CGCG,
       "pipe_cg": oracle.ALG_PIPE_CG}

SMALL = [
    (1, (100.0, 0.0, 50.0), 0.1),
    (2, (-30.0, 20.0, -10.0), 0.0),
    (3, (0.0, -75.0, 5.0), 0.25),
    (5, (100.0, 0.0, 50.0), 0.1),
    (10, (100.0, 0.0, 50.0), 0.1),
    (17, (-100.0, 40.0, -0.0), 0.5),
]


def _system(n, beta, shift, seed=2):
    kappa = inputs.kappa_cells(n, 1.0, seed)
    A = oracle.assemble(3, n, 27, beta, kappa, shift)
    op = solver.convdiff27(n, dev_t(kappa), beta, shift)
    return A, kappa, op


@pytest.mark.parametrize("n,beta,shift", SMALL)
def test_products_and_jacobi_bitwise(n, beta, shift):
    require_gpu()
    say(f"conv27 spmv n={n} beta={beta} shift={shift}")
    A, kappa, op = _system(n, beta, shift)
    assert op.column_form == "none" and op.index_bytes == 0
    for seed in (1, 2):
        x = inputs.random_vector(A.n, seed)
        assert same(host(solver.spmv(op, dev_t(x))), oracle.spmv(A, x))
    assert same(host(solver.jacobi_dinv(op)), oracle.jacobi_dinv(A))


SOLVES = [
    ("pbicgstab_rr", "jacobi_folded", 7),
    ("pbicgstab_rr", "jacobi", 5),
    ("pbicgstab", None, 0),
    ("bicgstab", "jacobi_folded", 0),
    ("bicgstab", "jacobi", 0),
    ("ca_bicgstab", "jacobi_folded", 0),
]


@pytest.mark.parametrize("n", [10, 17])
@pytest.mark.parametrize("variant,precond,k", SOLVES)
def test_solves_bitwise(n, variant, precond, k):
    require_gpu()
    beta, shift = (100.0, 0.0, 50.0), 0.1
    A, kappa, op = _system(n, beta, shift)
    xt = inputs.x_true(A.n)
    b = oracle.spmv(A, xt)
    say(f"conv27 solve n={n} {variant} {precond} k={k}")
    kw = dict(tol=1e-10, maxit=400)
    x, info = solver.solve(op, dev_t(b), variant=variant, precond=precond, rr_period=k, history=True, **kw)
    d = oracle.jacobi_dinv(A)
    if precond == "jacobi_folded":
        x_or, i_or = oracle.solve_folded(A, b, algo=ALG[variant], dinv=d, rr_period=k, history=True, **kw)
    else:
        x_or, i_or = oracle.solve(A, b, algo=ALG[variant], dinv=d if precond else None, rr_period=k, history=True,
                                  **kw)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
    assert info.status == 0
    assert same(host(x), x_or)
    assert same(host(info.history), i_or["history"])
    assert info.relres_true == i_or["relres_true"]
    # and the assembled CSR matrix on the GPU gives the same bits
    xc, ic = solver.solve(csr_op(A), dev_t(b), variant=variant, precond=precond, rr_period=k, **kw)
    assert same(host(xc), host(x)) and ic.iters == info.iters


@pytest.mark.parametrize("variant", ["cg", "cgcg", "pipe_cg"])
def test_cg_family_on_the_symmetric_operator(variant):
    require_gpu()
    A, kappa, op = _system(12, (0.0, 0.0, 0.0), 0.1)
    b = oracle.spmv(A, inputs.x_true(A.n))
    say(f"conv27 {variant}")
    x, info = solver.solve(op, dev_t(b), variant=variant, precond="jacobi", tol=1e-10, maxit=500)
    x_or, i_or = oracle.solve(A, b, algo=ALG[variant], dinv=oracle.jacobi_dinv(A), tol=1e-10, maxit=500)
    assert (info.status, info.iters) == (i_or["status"], i_or["iters"]) and info.status == 0
    assert same(host(x), x_or)


def test_precision_form_bitwise():
    require_gpu()
    A, kappa, op = _system(17, (100.0, 0.0, 50.0), 0.1)
    b = oracle.spmv(A, inputs.x_true(A.n))
    say("conv27 precision form")
    d = oracle.jacobi_dinv(A)
    for precond, dv in (("jacobi_folded", d), (None, None)):
        x, info = solver.solve(op, dev_t(b), variant="pbicgstab_rr", precond=precond, precision="fp32_rr64",
                               tol=1e-10, maxit=1000, rr_period=10, history=True)
        x_or, i_or = oracle.solve_mp(A, b, dinv=dv, tol=1e-10, maxit=1000, rr_period=10, history=True)
        assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
        assert same(host(x), x_or)
        assert same(host(info.history), i_or["history"])


def test_refused_uses_and_bad_arguments():
    require_gpu()
    A, kappa, op = _system(5, (1.0, 2.0, 3.0), 0.0)
    with pytest.raises(L.PbcgsError) as e:
        solver.transpose(op)
    assert e.value.code == L.ERR_UNSUPPORTED
    b = dev_t(oracle.spmv(A, inputs.x_true(A.n)))
    with pytest.raises(L.PbcgsError):
        solver.solve_batched([op], [b])
    ctx = op.ctx
    h = L.ctypes.c_void_p()
    beta = (L.ctypes.c_double * 3)(1.0, 2.0, 3.0)
    kd = dev_t(kappa)
    assert L.lib().pbcgs_op_convdiff27(ctx.handle, 0, solver._ptr(kd), beta, 0.0, L.ctypes.byref(h)) == L.ERR_INVALID_ARG
    assert L.lib().pbcgs_op_convdiff27(ctx.handle, 5, None, beta, 0.0, L.ctypes.byref(h)) == L.ERR_INVALID_ARG
    assert L.lib().pbcgs_op_convdiff27(ctx.handle, 1291, solver._ptr(kd), beta, 0.0,
                                       L.ctypes.byref(h)) == L.ERR_UNSUPPORTED  # 1291^3 > 2^31 - 1


@pytest.fixture(scope="module")
def c3_mf():
    require_gpu()
    w = inputs.workload("c3")
    kappa = inputs.kappa_cells(w.n, w.kappa_sigma)
    op = solver.convdiff27(w.n, dev_t(kappa), w.beta, w.shift)
    return w, kappa, op


def test_full_size_sampled_rows(c3_mf):
    w, kappa, op = c3_mf
    N = w.N
    xt = inputs.x_true(N)
    y = host(solver.spmv(op, dev_t(xt)))
    rng = np.random.default_rng(17)
    starts = [0, N // 2 - 5000, N - 3000] + list(rng.integers(0, N - 2000, 5))
    for s0 in starts:
        s0 = int(s0)
        s1 = min(N, s0 + 2000)
        r_or, c_or, v_or = oracle.assemble_rows(3, w.n, 27, w.beta, s0, s1, kappa, w.shift)
        rows = oracle.CSR(r_or, c_or, v_or)  # a row slice: n = s1 - s0 rows over all N columns
        assert same(y[s0:s1], oracle.spmv(rows, xt))


def test_full_size_folded_solve_bitwise(c3_mf):
    """The benchmark's matrix-free 27-point leg: folded Jacobi p-BiCGStab+RR,
    k = 50, tol 1e-8, against the oracle's folded solve on the assembled
    matrix."""
    w, kappa, op = c3_mf
    xt_h = inputs.x_true(w.N)
    t0 = time.time()
    A = oracle.assemble_workload(w, kappa)
    b_or = oracle.spmv(A, xt_h)
    say(f"c3 oracle assembly and rhs {time.time() - t0:.1f}s")
    b = dev_t(b_or)
    assert same(host(solver.spmv(op, dev_t(xt_h))), b_or)
    x, info = solver.solve(op, b, variant="pbicgstab_rr", precond="jacobi_folded", tol=w.tol, maxit=w.maxit,
                           rr_period=w.rr_period)
    say(f"c3 matrix-free folded solve: {info.iters} it, {info.n_rr} RR, {info.ms:.0f} ms")
    t0 = time.time()
    d = oracle.jacobi_dinv(A)
    x_or, i_or = oracle.solve_folded(A, b_or, algo=oracle.ALG_PBICGSTAB_RR, dinv=d, tol=w.tol, maxit=w.maxit,
                                     rr_period=w.rr_period)
    say(f"c3 oracle folded solve {time.time() - t0:.1f}s")
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
    assert info.status == 0
    assert same(host(x), x_or)
    assert info.relres_true == i_or["relres_true"]
    err = torch.linalg.norm(x - dev_t(xt_h)).item() / np.linalg.norm(xt_h)
    assert err < 1e-5
