"""GPU checks of the library's two test hooks, through the C ABI.

Workspace poisoning (opts.flags bit 5): the solve's vectors with their padding,
the partial sums, the diagonal layout's values, A M^{-1} and the binary32
values are filled with NaN bits before the solve writes them.  A solve that
read anything it had not written -- the index -1 vectors of the pipelined
methods, padding rows, a stale partial sum -- would return NaN; every variant,
preconditioner, precision, read path and launch shape must still equal the
oracle bit for bit.

Residual perturbation (pbcgs_debug_perturb): the recursive residual r_{j+1}
is scaled after iteration j, once its reductions are taken.  The oracle has
the same hook, so the perturbed solves are compared bit for bit, and the
replacement of Section 4.2 must close the gap between r and b - A x.
"""

import numpy as np
import pytest

import oracle
from paper_1612_01395_amd import _lib, inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say, stencil_coefs

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR,
       "ca_bicgstab": oracle.ALG_CA_BICGSTAB, "cg": oracle.ALG_CG, "cgcg": oracle.ALG_CGCG,
       "pipe_cg": oracle.ALG_PIPE_CG}


def _cases():
    return {
        # 3-D 7-point, 13,824 rows: many tiles
        "c2_24": (oracle.assemble_workload(inputs.workload("c2", n=24)), 3, 24),
        # 2-D 5-point, 3,721 rows: a ragged last tile
        "c1_61": (oracle.assemble_workload(inputs.workload("c1", n=61)), 2, 61),
        # symmetric positive definite 3-D 7-point (the CG family)
        "c2s_20": (oracle.assemble_workload(inputs.workload("c2s", n=20)), 3, 20),
    }


CASES = _cases()


def _op(name, opkind):
    A, dim, n = CASES[name]
    if opkind == "stencil":
        return solver.stencil(n, n, n if dim == 3 else 1, stencil_coefs(A, dim, n))
    return csr_op(A)


def _oracle(A, b, variant, precond, precision, maxit, rr, perturb=None):
    kw = dict(tol=1e-10, maxit=maxit, rr_period=rr, history=True)
    if precision == "fp32_rr64":
        return oracle.solve_mp(A, b, dinv=oracle.jacobi_dinv(A) if precond else None, **kw)
    if perturb is not None:
        kw["perturb"] = perturb
    if precond == "jacobi_folded":
        return oracle.solve_folded(A, b, algo=ALG[variant], dinv=oracle.jacobi_dinv(A), **kw)
    return oracle.solve(A, b, algo=ALG[variant], dinv=oracle.jacobi_dinv(A) if precond else None, **kw)


def _assert_equal(x, info, x_or, i_or, what):
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (what, info, i_or)
    assert same(host(x), x_or), (what, float(np.nanmax(np.abs(host(x) - x_or))))
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]]), what
    assert same(host(info.history), i_or["history"]), what


def _poisoned(name, variant, precond, opkind="csr", precision="fp64", gtarget=None, monkeypatch=None,
              maxit=3000, rr=20):
    require_gpu()
    if gtarget is not None:
        monkeypatch.setenv("PBCGS_GTARGET", str(gtarget))
    A, _, _ = CASES[name]
    b = oracle.spmv(A, inputs.x_true(A.n))
    what = f"poison {name} {variant} precond={precond} op={opkind} {precision} gtarget={gtarget}"
    say(what)
    x_or, i_or = _oracle(A, b, variant, precond, precision, maxit, rr)
    x, info = solver.solve(_op(name, "stencil" if opkind == "stencil" else "csr"), dev_t(b), variant=variant,
                           precond=precond, precision=precision, tol=1e-10, maxit=maxit, rr_period=rr,
                           history=True, diagonal_layout=(opkind != "csr_nodia"), poison=True)
    _assert_equal(x, info, x_or, i_or, what)
    return info


@pytest.mark.parametrize("opkind", ["csr", "csr_nodia", "stencil"])
@pytest.mark.parametrize("precond", [None, "jacobi", "jacobi_folded"])
@pytest.mark.parametrize("variant", ["bicgstab", "pbicgstab", "pbicgstab_rr"])
@pytest.mark.parametrize("name", ["c2_24", "c1_61"])
def test_poisoned_bicgstab_family(name, variant, precond, opkind):
    info = _poisoned(name, variant, precond, opkind)
    assert info.status == 0


@pytest.mark.parametrize("gtarget", [8, 64])
@pytest.mark.parametrize("variant", ["bicgstab", "pbicgstab_rr"])
def test_poisoned_two_rows_per_lane(variant, gtarget, monkeypatch):
    # few workgroups: every wave owns several 64-row blocks, so the two-row kernels run
    for name in ("c2_24", "c1_61"):
        _poisoned(name, variant, None, "csr", gtarget=gtarget, monkeypatch=monkeypatch)
        _poisoned(name, variant, None, "stencil", gtarget=gtarget, monkeypatch=monkeypatch)


@pytest.mark.parametrize("precond", [None, "jacobi_folded"])
@pytest.mark.parametrize("name", ["c2_24", "c1_61"])
def test_poisoned_ca_bicgstab(name, precond):
    _poisoned(name, "ca_bicgstab", precond)


@pytest.mark.parametrize("opkind", ["csr", "csr_nodia", "stencil"])
@pytest.mark.parametrize("precond", [None, "jacobi"])
@pytest.mark.parametrize("variant", ["cg", "cgcg", "pipe_cg"])
def test_poisoned_cg_family(variant, precond, opkind):
    _poisoned("c2s_20", variant, precond, opkind)


@pytest.mark.parametrize("gtarget", [None, 8])
@pytest.mark.parametrize("opkind", ["csr", "csr_nodia"])
@pytest.mark.parametrize("precond", [None, "jacobi_folded"])
def test_poisoned_precision_form(precond, opkind, gtarget, monkeypatch):
    for name in ("c2_24", "c1_61"):
        _poisoned(name, "pbicgstab_rr", precond, opkind, precision="fp32_rr64", gtarget=gtarget,
                  monkeypatch=monkeypatch, rr=10)


@pytest.mark.parametrize("precond", [None, "jacobi_folded"])
def test_poisoned_noalloc(precond):
    require_gpu()
    A, _, _ = CASES["c1_61"]
    b = oracle.spmv(A, inputs.x_true(A.n))
    say(f"poison noalloc c1_61 precond={precond}")
    x_or, i_or = _oracle(A, b, "pbicgstab_rr", precond, "fp64", 3000, 20)
    x = dev_t(np.zeros(A.n))
    hist = dev_t(np.full(3001, np.nan))
    x, info = solver.solve_noalloc(csr_op(A), dev_t(b), x, variant="pbicgstab_rr", precond=precond, tol=1e-10,
                                   maxit=3000, rr_period=20, history=hist, poison=True)
    _assert_equal(x, info, x_or, i_or, "noalloc")


@pytest.mark.parametrize("layout", [True, False])
@pytest.mark.parametrize("variant", ["bicgstab", "pbicgstab_rr"])
def test_poisoned_batched(variant, layout):
    require_gpu()
    rng = np.random.default_rng(11)
    systems = [oracle.assemble(2, n, 5, tuple(rng.uniform(0.0, 100.0, 2))) for n in (3, 17, 45, 64)]
    systems += [oracle.assemble(3, n, 7, tuple(rng.uniform(0.0, 50.0, 3))) for n in (5, 21)]
    bs = [oracle.spmv(A, inputs.batch_x_true(k, A.n)) for k, A in enumerate(systems)]
    say(f"poison batched {variant} layout={layout} N = {[A.n for A in systems]}")
    kw = dict(tol=1e-10, maxit=3000, rr_period=13)
    xs, infos = solver.solve_batched([csr_op(A) for A in systems], [dev_t(b) for b in bs], variant=variant,
                                     diagonal_layout=layout, poison=True, **kw)
    for k, (A, b) in enumerate(zip(systems, bs)):
        x_or, i_or = oracle.solve(A, b, algo=ALG[variant], **kw)
        info = infos[k]
        assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), k
        assert same(host(xs[k]), x_or), k
        assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]]), k


# ---------------------------------------------------------------------------
# the residual perturbation hook
# ---------------------------------------------------------------------------
J, C, K = 4, 1.25, 10


@pytest.fixture
def hook_ctx():
    require_gpu()
    ctx = solver.Context()  # operators made on it keep it alive until they go
    yield ctx
    ctx.debug_perturb(-1)


def _ctx_op(ctx, name, opkind):
    A, dim, n = CASES[name]
    if opkind == "stencil":
        return solver.stencil(n, n, n if dim == 3 else 1, stencil_coefs(A, dim, n), ctx=ctx)
    return solver.csr(dev_t(A.row_ptr), dev_t(A.col), dev_t(A.val), ctx=ctx)


@pytest.mark.parametrize("opkind", ["csr", "csr_nodia", "stencil"])
@pytest.mark.parametrize("precond", [None, "jacobi", "jacobi_folded"])
@pytest.mark.parametrize("variant", ["pbicgstab", "pbicgstab_rr"])
def test_perturbed_solve_bitwise(hook_ctx, variant, precond, opkind):
    for name in ("c2_24", "c1_61"):
        A, _, _ = CASES[name]
        b = oracle.spmv(A, inputs.x_true(A.n))
        what = f"perturb {name} {variant} precond={precond} op={opkind} j={J} c={C}"
        say(what)
        x_or, i_or = _oracle(A, b, variant, precond, "fp64", 3000, K, perturb=(J, C))
        hook_ctx.debug_perturb(J, C)
        x, info = solver.solve(_ctx_op(hook_ctx, name, opkind), dev_t(b), variant=variant, precond=precond,
                               tol=1e-10, maxit=3000, rr_period=K, history=True,
                               diagonal_layout=(opkind != "csr_nodia"))
        _assert_equal(x, info, x_or, i_or, what)


@pytest.mark.parametrize("precond", [None, "jacobi"])
def test_replacement_closes_the_gap(hook_ctx, precond):
    """Truncated solves: after the perturbation ||b - A x_m|| and ||r_m|| part;
    the replacement of iteration K-1 makes them equal, bit for bit."""
    A, _, _ = CASES["c2_24"]
    b = oracle.spmv(A, inputs.x_true(A.n))
    op = _ctx_op(hook_ctx, "c2_24", "csr")
    hook_ctx.debug_perturb(J, C)
    for m in (J + 1, J + 3, K, K + 3):
        say(f"gap c2_24 precond={precond} maxit={m}")
        x, info = solver.solve(op, dev_t(b), variant="pbicgstab_rr", precond=precond, tol=0.0, maxit=m,
                               rr_period=K, history=True)
        x_or, i_or = _oracle(A, b, "pbicgstab_rr", precond, "fp64", m, K, perturb=(J, C))
        assert same(host(x), x_or)
        h = float(host(info.history)[-1])
        gap = abs(info.relres_true - h) / h
        if m == K:
            assert info.relres_true == h
        elif J + 1 < m < K:
            assert gap > 1e-3
        else:
            assert gap < 1e-10


def test_perturb_hook_errors_and_reset(hook_ctx):
    A, _, _ = CASES["c1_61"]
    b = dev_t(oracle.spmv(A, inputs.x_true(A.n)))
    op = _ctx_op(hook_ctx, "c1_61", "csr")
    with pytest.raises(_lib.PbcgsError) as e:
        hook_ctx.debug_perturb(-2, 1.0)
    assert e.value.code == _lib.ERR_INVALID_ARG
    with pytest.raises(_lib.PbcgsError) as e:
        hook_ctx.debug_perturb(3, float("inf"))
    assert e.value.code == _lib.ERR_INVALID_ARG
    hook_ctx.debug_perturb(3, 0.5)
    for kw in (dict(variant="bicgstab"), dict(variant="cg"), dict(variant="pbicgstab_rr", precision="fp32_rr64")):
        with pytest.raises(_lib.PbcgsError) as e:
            solver.solve(op, b, tol=1e-10, maxit=100, **kw)
        assert e.value.code == _lib.ERR_UNSUPPORTED, kw
    with pytest.raises(_lib.PbcgsError) as e:
        solver.solve_batched([op], [b], variant="pbicgstab_rr", tol=1e-10, maxit=100)
    assert e.value.code == _lib.ERR_UNSUPPORTED
    # switched off, the context solves as before
    hook_ctx.debug_perturb(-1)
    x_or, i_or = _oracle(A, oracle.spmv(A, inputs.x_true(A.n)), "pbicgstab_rr", None, "fp64", 3000, K)
    x, info = solver.solve(op, b, variant="pbicgstab_rr", tol=1e-10, maxit=3000, rr_period=K, history=True)
    _assert_equal(x, info, x_or, i_or, "after reset")
