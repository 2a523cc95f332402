"""GPU parity of the precision form (binary32 vectors, SpMV, recurrences and
dot products; binary64 residual replacement, x update and scalars) against
the oracle's ``solve_mp``, through the C ABI.  Both sides round the same
operations the same way, so the comparison is bitwise: iterates, iteration
and replacement counts (forced ones included), residuals and histories."""

import numpy as np
import pytest

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say, stencil_coefs

pytestmark = pytest.mark.gpu


def _cases():
    c3n = 10
    return {
        "c1": (oracle.assemble_workload(inputs.workload("c1")), 2, 64),
        "c2_24": (oracle.assemble_workload(inputs.workload("c2", n=24)), 3, 24),
        "c3_10": (oracle.assemble_workload(inputs.workload("c3", n=c3n), inputs.kappa_cells(c3n)), 3, c3n),
    }


CASES = _cases()


def _compare(name, precond, opkind, tol=1e-10, rr=20, maxit=3000, x0=None):
    A, dim, n = CASES[name]
    say(f"fp32_rr64 {name} precond={precond} op={opkind} tol={tol} rr={rr} maxit={maxit}")
    b = oracle.spmv(A, inputs.x_true(A.n))
    dv = oracle.jacobi_dinv(A) if precond else None
    x_or, i_or = oracle.solve_mp(A, b, dinv=dv, x0=x0, tol=tol, maxit=maxit, rr_period=rr, history=True)
    op = csr_op(A) if opkind == "csr" else solver.stencil(n, n, n if dim == 3 else 1, stencil_coefs(A, dim, n))
    x, info = solver.solve(op, dev_t(b), None if x0 is None else dev_t(x0), variant="pbicgstab_rr",
                           precond=precond, precision="fp32_rr64", tol=tol, maxit=maxit, rr_period=rr,
                           history=True)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
    assert same(host(x), x_or), float(np.abs(host(x) - x_or).max())
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])
    assert same(host(info.history), i_or["history"])
    return info, i_or


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precond", [None, "jacobi_folded"])
def test_precision_form_bitwise_csr(name, precond):
    require_gpu()
    info, _ = _compare(name, precond, "csr")
    assert info.status == 0 and info.relres_true <= 1e-10


@pytest.mark.parametrize("name", ["c1", "c2_24"])
def test_precision_form_bitwise_stencil(name):
    require_gpu()
    _compare(name, "jacobi_folded", "stencil")


def test_forced_replacement_and_limits():
    require_gpu()
    # recursive convergence not confirmed by the binary64 residual: one forced replacement
    info, i_or = _compare("c2_24", "jacobi_folded", "csr", tol=1e-5, rr=0)
    assert i_or["n_rr"] == 1
    _compare("c2_24", "jacobi_folded", "csr", tol=3e-6, rr=0)
    # fixed iteration count, frequent replacement, non-zero x0
    _compare("c1", None, "csr", tol=0.0, rr=10, maxit=37)
    _compare("c1", None, "csr", tol=0.0, rr=1, maxit=12)
    _compare("c3_10", "jacobi_folded", "csr", tol=1e-9, rr=7, x0=inputs.random_vector(CASES["c3_10"][0].n, 4))
    # unstable without replacement: same failure on both sides
    _compare("c2_24", "jacobi_folded", "csr", tol=1e-7, rr=0, maxit=2000)


def test_precision_form_errors():
    require_gpu()
    from paper_1612_01395_amd import _lib
    A = CASES["c1"][0]
    op = csr_op(A)
    b = dev_t(oracle.spmv(A, inputs.x_true(A.n)))
    for kw in (dict(variant="bicgstab"), dict(variant="pbicgstab"), dict(precond="jacobi")):
        args = dict(variant="pbicgstab_rr", precision="fp32_rr64")
        args.update(kw)
        with pytest.raises(_lib.PbcgsError):
            solver.solve(op, b, **args)
