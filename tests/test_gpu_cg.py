"""GPU parity of the CG family (Section 2: Algorithms 2, 4 and 6) against the oracle.

Bitwise comparison of iterates, counts, residuals and histories on
symmetric positive definite CSR and stencil operators, without a
preconditioner and with Jacobi (a constant or a variable diagonal).  p-CG
alternates its gathered vector between two buffers, so launch shapes, graph
chunking (chunks that start at odd iterations) and direct launches are
checked against each other too.
"""

import os

import numpy as np
import pytest

import oracle
from paper_1612_01395_amd import _lib, inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say, stencil_coefs

pytestmark = pytest.mark.gpu

ALG = {"cg": oracle.ALG_CG, "cgcg": oracle.ALG_CGCG, "pipe_cg": oracle.ALG_PIPE_CG}
SYNCS = {"cg": 3, "cgcg": 2, "pipe_cg": 1}


def _cases():
    c3n = 10
    return {
        "c1s": (oracle.assemble_workload(inputs.workload("c1s")), 2, 64),
        "c2s_24": (oracle.assemble_workload(inputs.workload("c2s", n=24)), 3, 24),
        "c3s_10": (oracle.assemble_workload(inputs.workload("c3s", n=c3n), inputs.kappa_cells(c3n)), 3, c3n),
    }


CASES = _cases()
# an odd row count: the last lane of a two-row block holds one row
ODD = {"c2s_23": (oracle.assemble_workload(inputs.workload("c2s", n=23)), 3, 23)}


def _run(name, variant, precond, opkind="csr", tol=1e-10, maxit=3000, x0=None, **kw):
    A, dim, n = {**CASES, **ODD}[name]
    say(f"{variant} {name} precond={precond} op={opkind} tol={tol} maxit={maxit} {kw}")
    b = oracle.spmv(A, inputs.x_true(A.n))
    dv = oracle.jacobi_dinv(A) if precond else None
    x_or, i_or = oracle.solve(A, b, algo=ALG[variant], dinv=dv, x0=x0, tol=tol, maxit=maxit, history=True)
    op = csr_op(A) if opkind == "csr" else solver.stencil(n, n, n if dim == 3 else 1, stencil_coefs(A, dim, n))
    x, info = solver.solve(op, dev_t(b), None if x0 is None else dev_t(x0), variant=variant, precond=precond,
                           tol=tol, maxit=maxit, history=True, **kw)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
    assert same(host(x), x_or), float(np.abs(host(x) - x_or).max())
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])
    assert same(host(info.history), i_or["history"])
    assert info.syncs_per_iter == SYNCS[variant]
    return host(x), info


@pytest.mark.parametrize("precond", [None, "jacobi"])
@pytest.mark.parametrize("variant", list(ALG))
@pytest.mark.parametrize("name", list(CASES))
def test_cg_family_bitwise_csr(name, variant, precond):
    require_gpu()
    _, info = _run(name, variant, precond)
    assert info.status == 0


@pytest.mark.parametrize("precond", [None, "jacobi"])
@pytest.mark.parametrize("variant", list(ALG))
@pytest.mark.parametrize("name", ["c1s", "c2s_24"])
def test_cg_family_bitwise_stencil(name, variant, precond):
    require_gpu()
    _run(name, variant, precond, opkind="stencil")


@pytest.mark.parametrize("variant", list(ALG))
def test_cg_family_maxit_x0_chunks_and_shapes(variant):
    require_gpu()
    A, _, _ = CASES["c2s_24"]
    x0 = inputs.random_vector(A.n, 4)
    for maxit in (0, 1, 2, 7):
        _run("c2s_24", variant, "jacobi", tol=0.0, maxit=maxit, x0=x0)
    ref, iref = _run("c2s_24", variant, "jacobi", graph=False)
    for kw in (dict(check_every=1), dict(check_every=3), dict(check_every=5), dict(time_kernels=True)):
        x, info = _run("c2s_24", variant, "jacobi", **kw)
        assert same(x, ref) and info.iters == iref.iters, kw
    saved = {k: os.environ.get(k) for k in ("PBCGS_GTARGET", "PBCGS_R")}
    try:
        for var, val in (("PBCGS_GTARGET", "3"), ("PBCGS_GTARGET", "1024"), ("PBCGS_R", "1"), ("PBCGS_R", "16")):
            for k in saved:
                os.environ.pop(k, None)
            os.environ[var] = val
            x, info = _run("c2s_24", variant, "jacobi", check_every=3)
            assert same(x, ref) and info.iters == iref.iters, (var, val)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_cg_family_status_cases():
    require_gpu()
    C = oracle.assemble_workload(inputs.workload("c1s", n=8))
    bn = np.ones(C.n)
    bn[3] = np.inf
    cases = [("zero-b", np.zeros(C.n), {}), ("inf-b", bn, {}),
             ("maxit", oracle.spmv(C, inputs.x_true(C.n)), dict(tol=1e-14, maxit=3))]
    for variant in ALG:
        for name, b, kw in cases:
            say(f"{variant} status {name}")
            x_or, i_or = oracle.solve(C, b, algo=ALG[variant], **kw)
            x, info = solver.solve(csr_op(C), dev_t(b), variant=variant, **kw)
            assert (info.status, info.iters) == (i_or["status"], i_or["iters"]), (variant, name, info, i_or)
            assert same(host(x), x_or), (variant, name)


def test_cg_family_unsupported_combinations():
    require_gpu()
    A, _, _ = CASES["c1s"]
    op = csr_op(A)
    b = dev_t(oracle.spmv(A, inputs.x_true(A.n)))
    for variant in ALG:
        for kw in (dict(precond="jacobi_folded"), dict(precision="fp32_rr64")):
            with pytest.raises(_lib.PbcgsError):
                solver.solve(op, b, variant=variant, **kw)
        with pytest.raises(_lib.PbcgsError):
            solver.solve_batched([op], [b], variant=variant)


@pytest.mark.parametrize("gtarget", [2, 8])
@pytest.mark.parametrize("opkind", ["csr", "stencil"])
@pytest.mark.parametrize("variant", list(ALG))
def test_cg_family_two_rows_per_lane(variant, opkind, gtarget, monkeypatch):
    """Few workgroups, so every wave owns several blocks and the product
    kernels (s = A p, w = A u, p-CG's n = A m) take two rows per lane: on the
    diagonal layout and on stencils with an even x extent.  Same bits."""
    require_gpu()
    monkeypatch.setenv("PBCGS_GTARGET", str(gtarget))
    for name in ("c1s", "c2s_24"):
        for precond in (None, "jacobi"):
            _run(name, variant, precond, opkind)
    if opkind == "csr":
        _run("c3s_10", variant, "jacobi", opkind)


@pytest.mark.parametrize("gtarget", [2, 8])
def test_pipe_cg_two_rows_odd_rows_and_unaligned_x(gtarget, monkeypatch):
    """p-CG's two-row kernel on 23^3 rows (the last pair holds one row), and
    with the caller's x 16-byte aligned (pair updates) or only 8-byte aligned
    (row by row): the oracle's bits, the rest of the buffer untouched."""
    require_gpu()
    monkeypatch.setenv("PBCGS_GTARGET", str(gtarget))
    A, _, _ = ODD["c2s_23"]
    assert A.n % 2 == 1
    for precond in (None, "jacobi"):
        ref, _ = _run("c2s_23", "pipe_cg", precond)
        for shift in (1, 2):
            buf = dev_t(np.full(A.n + 3, 7.0))
            out = buf[shift:shift + A.n]
            assert (out.data_ptr() % 16 == 0) == (shift == 2)
            x, _ = _run("c2s_23", "pipe_cg", precond, out=out)
            assert same(x, ref) and same(host(out), ref)
            hb = host(buf)
            assert (hb[:shift] == 7.0).all() and (hb[shift + A.n:] == 7.0).all()
