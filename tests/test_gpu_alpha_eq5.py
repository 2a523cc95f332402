"""GPU parity of the eq. (5) alpha_{i+1} (Section 3.1) against the oracle.

Eq. (5) is eq. (3) rearranged into three quotients; in exact arithmetic both
give the same iterates, in binary64 they round differently.  The HIP path and
the oracle evaluate eq. (5) in the same order, so the comparison is bitwise,
as for eq. (3).
"""

import numpy as np
import pytest

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say, stencil_coefs

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR}


def _cases():
    c3n = 10
    return {
        "c1": (oracle.assemble_workload(inputs.workload("c1")), 2, 64),
        "c2_24": (oracle.assemble_workload(inputs.workload("c2", n=24)), 3, 24),
        "c3_10": (oracle.assemble_workload(inputs.workload("c3", n=c3n), inputs.kappa_cells(c3n)), 3, c3n),
    }


CASES = _cases()


def _run(name, variant, precond, opkind, alpha_form, tol=1e-10, rr=20, maxit=2000):
    A, dim, n = CASES[name]
    say(f"alpha eq.({alpha_form}) {name} {variant} precond={precond} op={opkind}")
    b = oracle.spmv(A, inputs.x_true(A.n))
    dv = oracle.jacobi_dinv(A) if precond else None
    solve = oracle.solve_folded if precond == "jacobi_folded" else oracle.solve
    x_or, i_or = solve(A, b, algo=ALG[variant], dinv=dv, tol=tol, maxit=maxit, rr_period=rr, history=True,
                       alpha_form=alpha_form)
    op = csr_op(A) if opkind == "csr" else solver.stencil(n, n, n if dim == 3 else 1, stencil_coefs(A, dim, n))
    x, info = solver.solve(op, dev_t(b), variant=variant, precond=precond, tol=tol, maxit=maxit, rr_period=rr,
                           history=True, alpha_form=alpha_form)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
    assert same(host(x), x_or), float(np.abs(host(x) - x_or).max())
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])
    assert same(host(info.history), i_or["history"])
    return host(x), info


@pytest.mark.parametrize("variant", ["pbicgstab", "pbicgstab_rr"])
@pytest.mark.parametrize("precond", [None, "jacobi", "jacobi_folded"])
@pytest.mark.parametrize("name", list(CASES))
def test_eq5_bitwise_csr(name, variant, precond):
    require_gpu()
    x5, i5 = _run(name, variant, precond, "csr", 5)
    assert i5.status == 0


@pytest.mark.parametrize("name", ["c1", "c2_24"])
def test_eq5_bitwise_stencil(name):
    require_gpu()
    _run(name, "pbicgstab_rr", "jacobi_folded", "stencil", 5)


def test_eq5_is_a_different_rounding_and_bicgstab_ignores_it():
    require_gpu()
    x3, i3 = _run("c1", "pbicgstab_rr", None, "csr", 3)
    x5, i5 = _run("c1", "pbicgstab_rr", None, "csr", 5)
    assert not np.array_equal(x3, x5)
    xb3, _ = _run("c1", "bicgstab", None, "csr", 3)
    xb5, _ = _run("c1", "bicgstab", None, "csr", 5)
    assert np.array_equal(xb3, xb5)


@pytest.mark.parametrize("name", ["c1", "c2_24"])
@pytest.mark.parametrize("precond", [None, "jacobi_folded"])
def test_eq5_precision_form_bitwise(name, precond):
    """In the precision form eq. (5) is the less robust choice: on the 2-D
    problem without a preconditioner it diverges to NONFINITE, with Jacobi it
    needs several times the iterations of eq. (3).  The HIP path reproduces
    those runs bit for bit, divergence included."""
    require_gpu()
    A, dim, n = CASES[name]
    say(f"alpha eq.(5) fp32_rr64 {name} precond={precond}")
    b = oracle.spmv(A, inputs.x_true(A.n))
    dv = oracle.jacobi_dinv(A) if precond else None
    kw = dict(tol=1e-10, maxit=3000, rr_period=20)
    x_or, i_or = oracle.solve_mp(A, b, dinv=dv, history=True, alpha_form=5, **kw)
    x, info = solver.solve(csr_op(A), dev_t(b), variant="pbicgstab_rr", precond=precond, precision="fp32_rr64",
                           history=True, alpha_form=5, **kw)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
    assert same(host(x), x_or)
    assert same(host(info.history), i_or["history"])


def test_eq5_batched_bitwise():
    require_gpu()
    sys = [oracle.assemble(2, n, 5, (30.0 + n, 10.0)) for n in (5, 33, 100)] + [oracle.assemble(3, 12, 7, (20, 5, 1))]
    say(f"alpha eq.(5) batched: N = {[A.n for A in sys]}")
    bs = [oracle.spmv(A, inputs.batch_x_true(k, A.n)) for k, A in enumerate(sys)]
    kw = dict(tol=1e-10, maxit=3000, rr_period=17)
    xs, infos = solver.solve_batched([csr_op(A) for A in sys], [dev_t(b) for b in bs], variant="pbicgstab_rr",
                                     alpha_form=5, **kw)
    for k, (A, b) in enumerate(zip(sys, bs)):
        x_or, i_or = oracle.solve(A, b, algo=oracle.ALG_PBICGSTAB_RR, alpha_form=5, **kw)
        assert (infos[k].status, infos[k].iters, infos[k].n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), k
        assert same(host(xs[k]), x_or), k


def test_alpha_form_argument_checked():
    require_gpu()
    A, _, _ = CASES["c1"]
    with pytest.raises(ValueError):
        solver.solve(csr_op(A), dev_t(np.ones(A.n)), alpha_form=4)
