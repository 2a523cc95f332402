"""The persistent form (the whole solve in one cooperative launch, grid
barriers in place of kernel boundaries) against the oracle and against the
graph-launched form, bit for bit: every variant and preconditioner, residual
replacement schedules, iteration limits (including the reduction left pending
at maxit) and the status cases."""

import os

import numpy as np
import pytest

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say, stencil_coefs

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR}


class persist:
    def __init__(self, mode):
        self.mode = mode

    def __enter__(self):
        self.old = os.environ.get("PBCGS_PERSIST")
        os.environ["PBCGS_PERSIST"] = self.mode

    def __exit__(self, *exc):
        if self.old is None:
            os.environ.pop("PBCGS_PERSIST", None)
        else:
            os.environ["PBCGS_PERSIST"] = self.old


def _cases():
    return {"c1": (oracle.assemble_workload(inputs.workload("c1")), 2, 64),
            "c2_24": (oracle.assemble_workload(inputs.workload("c2", n=24)), 3, 24),
            "c3_10": (oracle.assemble_workload(inputs.workload("c3", n=10), inputs.kappa_cells(10)), 3, 10)}


CASES = _cases()


@pytest.mark.parametrize("variant", list(ALG))
@pytest.mark.parametrize("precond", [None, "jacobi", "jacobi_folded"])
@pytest.mark.parametrize("name", list(CASES))
def test_persistent_bitwise(name, precond, variant):
    require_gpu()
    A, dim, n = CASES[name]
    b = oracle.spmv(A, inputs.x_true(A.n))
    dv = oracle.jacobi_dinv(A) if precond else None
    solve = oracle.solve_folded if precond == "jacobi_folded" else oracle.solve
    kw = dict(tol=1e-10, maxit=2000, rr_period=20)
    x_or, i_or = solve(A, b, algo=ALG[variant], dinv=dv, history=True, **kw)
    say(f"persistent {name} {variant} {precond}")
    with persist("1"):
        x, info = solver.solve(csr_op(A), dev_t(b), variant=variant, precond=precond, history=True, **kw)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
    assert same(host(x), x_or)
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])
    assert same(host(info.history), i_or["history"])


def test_persistent_limits_schedules_and_statuses():
    require_gpu()
    A, dim, n = CASES["c1"]
    b = oracle.spmv(A, inputs.x_true(A.n))
    st = solver.stencil(n, n, 1, stencil_coefs(A, dim, n))
    for variant in ALG:
        for kw in (dict(tol=0.0, maxit=0), dict(tol=0.0, maxit=1), dict(tol=0.0, maxit=37, rr_period=10),
                   dict(tol=1e-9, maxit=500, rr_period=1), dict(tol=1e-12, maxit=200, rr_period=7, rr_max=3)):
            say(f"persistent limits {variant} {kw}")
            x_or, i_or = oracle.solve(A, b, algo=ALG[variant], **kw)
            with persist("1"):
                x, info = solver.solve(csr_op(A), dev_t(b), variant=variant, **kw)
                xs, infs = solver.solve(st, dev_t(b), variant=variant, **kw)
            with persist("0"):
                xg, infg = solver.solve(csr_op(A), dev_t(b), variant=variant, **kw)
            assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
            assert same(host(x), x_or) and same(host(xs), x_or) and same(host(xg), x_or)
            assert same([info.relres_rec], [infg.relres_rec])
    skew = oracle.CSR([0, 1, 2], [1, 0], [1.0, -1.0])
    C = oracle.assemble_workload(inputs.workload("c1", n=8))
    bn = np.ones(C.n)
    bn[5] = np.nan
    for name, M, rhs in (("skew", skew, np.array([1.0, 2.0])), ("zero-b", C, np.zeros(C.n)), ("nan-b", C, bn)):
        for variant in ALG:
            x_or, i_or = oracle.solve(M, rhs, algo=ALG[variant])
            with persist("1"):
                x, info = solver.solve(csr_op(M), dev_t(rhs), variant=variant)
            assert (info.status, info.iters) == (i_or["status"], i_or["iters"]), (name, variant)
            assert same(host(x), x_or), (name, variant)
