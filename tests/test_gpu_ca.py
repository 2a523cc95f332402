"""GPU parity of CA-BiCGStab (Algorithm 8, Section 3.1) against the oracle.

The library's CA kernels evaluate every recurrence and dot product in the
oracle's order, so iterates, counts, residuals and histories agree bit for
bit, on CSR and stencil operators, without a preconditioner and with Jacobi
folded into the operator, and with alpha_{i+1} by eq. (3) or eq. (5).
"""

import os

import numpy as np
import pytest

import oracle
from paper_1612_01395_amd import _lib, inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say, stencil_coefs

pytestmark = pytest.mark.gpu

CA = oracle.ALG_CA_BICGSTAB


def _cases():
    c3n = 10
    return {
        "c1": (oracle.assemble_workload(inputs.workload("c1")), 2, 64),
        "c2_24": (oracle.assemble_workload(inputs.workload("c2", n=24)), 3, 24),
        "c3_10": (oracle.assemble_workload(inputs.workload("c3", n=c3n), inputs.kappa_cells(c3n)), 3, c3n),
    }


CASES = _cases()


def _run(name, precond, opkind, alpha_form=3, tol=1e-10, maxit=2000, x0=None, **kw):
    A, dim, n = CASES[name]
    say(f"ca {name} precond={precond} op={opkind} alpha eq.({alpha_form}) tol={tol} maxit={maxit}")
    b = oracle.spmv(A, inputs.x_true(A.n))
    if precond == "jacobi_folded":
        x_or, i_or = oracle.solve_folded(A, b, algo=CA, dinv=oracle.jacobi_dinv(A), x0=x0, tol=tol, maxit=maxit,
                                         history=True, alpha_form=alpha_form)
    else:
        x_or, i_or = oracle.solve(A, b, algo=CA, x0=x0, tol=tol, maxit=maxit, history=True, alpha_form=alpha_form)
    op = csr_op(A) if opkind == "csr" else solver.stencil(n, n, n if dim == 3 else 1, stencil_coefs(A, dim, n))
    x, info = solver.solve(op, dev_t(b), None if x0 is None else dev_t(x0), variant="ca_bicgstab", precond=precond,
                           tol=tol, maxit=maxit, history=True, alpha_form=alpha_form, **kw)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
    assert same(host(x), x_or), float(np.abs(host(x) - x_or).max())
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])
    assert same(host(info.history), i_or["history"])
    assert info.syncs_per_iter == 4
    return host(x), info


@pytest.mark.parametrize("alpha_form", [3, 5])
@pytest.mark.parametrize("precond", [None, "jacobi_folded"])
@pytest.mark.parametrize("name", list(CASES))
def test_ca_bitwise_csr(name, precond, alpha_form):
    require_gpu()
    _, info = _run(name, precond, "csr", alpha_form)
    assert info.status == 0


@pytest.mark.parametrize("precond", [None, "jacobi_folded"])
@pytest.mark.parametrize("name", ["c1", "c2_24"])
def test_ca_bitwise_stencil(name, precond):
    require_gpu()
    _run(name, precond, "stencil")


def test_ca_maxit_x0_and_launch_shapes():
    require_gpu()
    A, _, _, = CASES["c2_24"]
    x0 = inputs.random_vector(A.n, 3)
    _run("c2_24", None, "csr", tol=0.0, maxit=9, x0=x0)
    _run("c2_24", "jacobi_folded", "csr", tol=1e-11, x0=x0)
    ref, iref = _run("c2_24", None, "csr", graph=False)
    saved = {k: os.environ.get(k) for k in ("PBCGS_GTARGET", "PBCGS_R")}
    try:
        for var, val in (("PBCGS_GTARGET", "3"), ("PBCGS_GTARGET", "1024"), ("PBCGS_R", "1"), ("PBCGS_R", "16")):
            for k in saved:
                os.environ.pop(k, None)
            os.environ[var] = val
            x, info = _run("c2_24", None, "csr", check_every=3)
            assert same(x, ref) and info.iters == iref.iters
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_ca_status_cases_match_oracle():
    require_gpu()
    skew = oracle.CSR([0, 1, 2], [1, 0], [1.0, -1.0])
    twoI = oracle.CSR(np.arange(6), np.arange(5), np.full(5, 2.0))
    C = oracle.assemble_workload(inputs.workload("c1", n=8))
    bn = np.ones(C.n)
    bn[5] = np.nan
    cases = [("skew", skew, np.array([1.0, 2.0]), {}), ("2I", twoI, np.array([1.0, -3.0, 0.5, 7.0, 2.0]), {}),
             ("zero-b", C, np.zeros(C.n), {}), ("nan-b", C, bn, {}),
             ("maxit", C, oracle.spmv(C, inputs.x_true(C.n)), dict(tol=1e-14, maxit=3))]
    for name, A, b, kw in cases:
        say(f"ca status {name}")
        x_or, i_or = oracle.solve(A, b, algo=CA, **kw)
        x, info = solver.solve(csr_op(A), dev_t(b), variant="ca_bicgstab", **kw)
        assert (info.status, info.iters) == (i_or["status"], i_or["iters"]), (name, info, i_or)
        assert same(host(x), x_or), name


def test_ca_unsupported_combinations():
    require_gpu()
    A, _, _ = CASES["c1"]
    op = csr_op(A)
    b = dev_t(oracle.spmv(A, inputs.x_true(A.n)))
    for kw in (dict(precond="jacobi"), dict(precision="fp32_rr64")):
        with pytest.raises(_lib.PbcgsError):
            solver.solve(op, b, variant="ca_bicgstab", **kw)
    with pytest.raises(_lib.PbcgsError):
        solver.solve_batched([op], [b], variant="ca_bicgstab")
