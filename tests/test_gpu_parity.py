"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

The library's arithmetic contract (no fused multiply-add, rows summed in
column order, pairwise dot products) is the oracle's, so every comparison
below is bitwise: assembly, SpMV, dot products, Jacobi, and whole solves --
iterates, iteration counts, replacement counts, residuals and histories.
"""

import os

import numpy as np
import pytest
import torch

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say, stencil_coefs

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR}


def small_cases():
    c3n = 10
    return {
        "c1": (oracle.assemble_workload(inputs.workload("c1")), None, 2, 64),
        "c2_24": (oracle.assemble_workload(inputs.workload("c2", n=24)), None, 3, 24),
        "c3_10": (oracle.assemble_workload(inputs.workload("c3", n=c3n), inputs.kappa_cells(c3n)), None, 3, c3n),
    }


CASES = small_cases()


@pytest.mark.parametrize("name", list(CASES))
def test_spmv_bitwise(name):
    require_gpu()
    A, _, dim, n = CASES[name]
    say(f"spmv {name} n={A.n}")
    x = inputs.random_vector(A.n, 1)
    y_or = oracle.spmv(A, x)
    op = csr_op(A)
    y = host(solver.spmv(op, dev_t(x)))
    assert same(y, y_or)
    if name != "c3_10":
        st = solver.stencil(n, n, n if dim == 3 else 1, stencil_coefs(A, dim, n))
        assert same(host(solver.spmv(st, dev_t(x))), y_or)


@pytest.mark.parametrize("n", [1, 7, 255, 256, 257, 4096, 65549, 1 << 21, 3000001])
def test_dot_bitwise_and_shape_independent(n):
    require_gpu()
    say(f"dot n={n}")
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))
    y = rng.standard_normal(n)
    ref = oracle.dot(x, y)
    xd, yd = dev_t(x), dev_t(y)
    old = os.environ.get("PBCGS_GTARGET")
    try:
        for g in ("512", "7", "64", "1024", "1"):
            os.environ["PBCGS_GTARGET"] = g
            assert same(solver.dot(xd, yd), ref), g
    finally:
        if old is None:
            os.environ.pop("PBCGS_GTARGET", None)
        else:
            os.environ["PBCGS_GTARGET"] = old


@pytest.mark.parametrize("name,n", [("c1", 64), ("c1", 5), ("c2", 1), ("c2", 33), ("c3", 2), ("c3", 12)])
def test_device_assembly_bitwise(name, n):
    require_gpu()
    w = inputs.workload(name, n=n)
    kappa = inputs.kappa_cells(n, w.kappa_sigma) if w.npts == 27 else None
    say(f"assembly {name} n={n}")
    A = oracle.assemble_workload(w, kappa)
    rp, col, val = solver.assemble_convdiff(w.dim, n, w.npts, w.beta, None if kappa is None else dev_t(kappa),
                                            w.shift)
    assert np.array_equal(host(rp), A.row_ptr)
    assert np.array_equal(host(col), A.col)
    assert same(host(val), A.val)


@pytest.mark.parametrize("name", list(CASES))
def test_jacobi_dinv_bitwise(name):
    require_gpu()
    A = CASES[name][0]
    assert same(host(solver.jacobi_dinv(csr_op(A))), oracle.jacobi_dinv(A))


def _compare(name, variant, precond, opkind, A, dim, n, dinv_vec=None, tol=1e-10, rr=20, maxit=2000):
    say(f"solve {name} {variant} precond={precond} op={opkind} dinv_vec={dinv_vec is not None}")
    xt = inputs.x_true(A.n)
    b = oracle.spmv(A, xt)
    dv = None
    if precond in ("jacobi", "jacobi_folded"):
        dv = dinv_vec if dinv_vec is not None else oracle.jacobi_dinv(A)
    solve = oracle.solve_folded if precond == "jacobi_folded" else oracle.solve
    x_or, info_or = solve(A, b, algo=ALG[variant], dinv=dv, tol=tol, maxit=maxit, rr_period=rr, history=True)
    if opkind == "csr":
        op = csr_op(A)
    else:
        op = solver.stencil(n, n, n if dim == 3 else 1, stencil_coefs(A, dim, n))
    x, info = solver.solve(op, dev_t(b), variant=variant, precond=precond,
                           dinv=None if dinv_vec is None else dev_t(dinv_vec), tol=tol, maxit=maxit,
                           rr_period=rr, history=True)
    assert info.status == info_or["status"], (info, info_or)
    assert info.iters == info_or["iters"], (info, info_or)
    assert info.n_rr == info_or["n_rr"]
    assert same(host(x), x_or), float(np.abs(host(x) - x_or).max())
    assert same([info.relres_rec, info.relres_true], [info_or["relres_rec"], info_or["relres_true"]])
    assert same(host(info.history), info_or["history"])
    return info


@pytest.mark.parametrize("variant", list(ALG))
@pytest.mark.parametrize("precond", [None, "jacobi", "jacobi_folded"])
@pytest.mark.parametrize("name", list(CASES))
def test_solve_bitwise_csr(name, variant, precond):
    require_gpu()
    A, _, dim, n = CASES[name]
    _compare(name, variant, precond, "csr", A, dim, n)


@pytest.mark.parametrize("variant", list(ALG))
@pytest.mark.parametrize("precond", [None, "jacobi", "jacobi_folded"])
@pytest.mark.parametrize("name", ["c1", "c2_24"])
def test_solve_bitwise_stencil(name, variant, precond):
    require_gpu()
    A, _, dim, n = CASES[name]
    _compare(name, variant, precond, "stencil", A, dim, n)


@pytest.mark.parametrize("variant", list(ALG))
@pytest.mark.parametrize("precond", ["jacobi", "jacobi_folded"])
def test_solve_bitwise_vector_jacobi(variant, precond):
    """A non-constant M^{-1} exercises the vector preconditioner path."""
    require_gpu()
    A, _, dim, n = CASES["c2_24"]
    d = oracle.jacobi_dinv(A) * (1.0 + 0.25 * np.random.default_rng(3).random(A.n))
    _compare("c2_24", variant, precond, "csr", A, dim, n, dinv_vec=d)


def test_folded_with_x0_and_repeated_calls():
    """Folded Jacobi from a non-zero x_0 (y_0 = x_0 / dinv), on a matrix with a
    variable diagonal, twice in a row on one context (the folded values are
    recomputed per call), and a smaller system after a larger one."""
    require_gpu()
    for name in ("c3_10", "c3_10", "c1"):
        A = CASES[name][0]
        b = oracle.spmv(A, inputs.x_true(A.n))
        x0 = inputs.random_vector(A.n, 9)
        dv = oracle.jacobi_dinv(A)
        for variant in ("pbicgstab_rr", "bicgstab"):
            say(f"folded x0 {name} {variant}")
            x_or, i_or = oracle.solve_folded(A, b, algo=ALG[variant], dinv=dv, x0=x0, tol=1e-11, rr_period=6)
            x, info = solver.solve(csr_op(A), dev_t(b), dev_t(x0), variant=variant, precond="jacobi_folded",
                                   tol=1e-11, rr_period=6)
            assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
            assert same(host(x), x_or)
            assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])


def test_launch_modes_and_shapes_identical():
    require_gpu()
    A, _, dim, n = CASES["c2_24"]
    op = csr_op(A)
    b = dev_t(oracle.spmv(A, inputs.x_true(A.n)))
    ref, info_ref = solver.solve(op, b, variant="pbicgstab_rr", precond="jacobi", tol=1e-10, rr_period=7)
    ref = host(ref)
    variants = [dict(graph=False), dict(time_kernels=True), dict(check_every=1), dict(check_every=5),
                dict(check_every=1000)]
    for kw in variants:
        say(f"mode {kw}")
        x, info = solver.solve(op, b, variant="pbicgstab_rr", precond="jacobi", tol=1e-10, rr_period=7, **kw)
        assert same(host(x), ref) and info.iters == info_ref.iters, kw
    saved = {k: os.environ.get(k) for k in ("PBCGS_GTARGET", "PBCGS_R")}
    try:
        for var, val in (("PBCGS_GTARGET", "3"), ("PBCGS_GTARGET", "16"), ("PBCGS_GTARGET", "1024"),
                         ("PBCGS_R", "1"), ("PBCGS_R", "2"), ("PBCGS_R", "8"), ("PBCGS_R", "64")):
            for k in saved:
                os.environ.pop(k, None)
            os.environ[var] = val
            say(f"{var}={val}")
            x, info = solver.solve(op, b, variant="pbicgstab_rr", precond="jacobi", tol=1e-10, rr_period=7)
            assert same(host(x), ref) and info.iters == info_ref.iters, (var, val)
            for variant in ("bicgstab", "pbicgstab"):
                x2, i2 = solver.solve(op, b, variant=variant, precond="jacobi", tol=1e-10)
                x3, i3 = solver.solve(op, b, variant=variant, precond="jacobi", tol=1e-10, graph=False)
                assert same(host(x2), host(x3)) and i2.iters == i3.iters
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_rr_max_and_maxit_and_x0():
    require_gpu()
    A, _, dim, n = CASES["c1"]
    b = oracle.spmv(A, inputs.x_true(A.n))
    x0 = inputs.random_vector(A.n, 5)
    for kw in (dict(rr_period=10, rr_max=2, tol=1e-12, maxit=200), dict(rr_period=1, rr_max=-1, tol=1e-9, maxit=500),
               dict(rr_period=10, rr_max=-1, tol=0.0, maxit=37)):
        say(f"rr case {kw}")
        x_or, i_or = oracle.solve(A, b, algo=oracle.ALG_PBICGSTAB_RR, x0=x0, **kw)
        x, info = solver.solve(csr_op(A), dev_t(b), dev_t(x0), variant="pbicgstab_rr", **kw)
        assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
        assert same(host(x), x_or)


def test_status_cases_match_oracle():
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
        for variant in ALG:
            say(f"status {name} {variant}")
            x_or, i_or = oracle.solve(A, b, algo=ALG[variant], **kw)
            x, info = solver.solve(csr_op(A), dev_t(b), variant=variant, **kw)
            assert (info.status, info.iters) == (i_or["status"], i_or["iters"]), (name, variant, info, i_or)
            assert same(host(x), x_or), (name, variant)


def test_api_errors():
    require_gpu()
    from paper_1612_01395_amd import _lib
    bad = oracle.CSR([0, 2, 1], [0, 1], [1.0, 1.0])  # decreasing row pointer
    with pytest.raises(_lib.PbcgsError):
        csr_op(bad)
    badcol = oracle.CSR([0, 1, 2], [0, 5], [1.0, 1.0])
    with pytest.raises(_lib.PbcgsError):
        csr_op(badcol)
    nodiag = oracle.CSR([0, 1, 2], [1, 0], [1.0, 1.0])
    op = csr_op(nodiag)
    with pytest.raises(_lib.PbcgsError):
        solver.solve(op, dev_t(np.ones(2)), precond="jacobi")
    with pytest.raises(_lib.PbcgsError):
        solver.solve(op, dev_t(np.ones(2)), tol=-1.0)
    with pytest.raises(_lib.PbcgsError):
        solver.solve(op, dev_t(np.ones(2)), precond="jacobi_folded")
    st = solver.stencil(4, 4, 1, [-1.0, -1.0, 4.5, -1.0, -1.0])
    with pytest.raises(_lib.PbcgsError):
        solver.solve(st, dev_t(np.ones(16)), precond="jacobi_folded", dinv=dev_t(np.linspace(0.2, 0.3, 16)))


def test_size_limits():
    """An empty operator is refused; the largest system one launch covers is
    1024 workgroups x 4 waves x 1024 blocks x 64 rows = 268,435,456 rows
    (about 645^3), and an operator one row larger is refused as unsupported
    rather than mis-launched.  The maximum-size solve (2 I x = 1, one
    iteration, about 40 GB of device memory) runs every reduction through the
    deepest per-wave tree."""
    require_gpu()
    from paper_1612_01395_amd import _lib
    dev = torch.device("cuda", 0)
    with pytest.raises(_lib.PbcgsError):
        solver.csr(torch.zeros(1, dtype=torch.int32, device=dev), torch.zeros(0, dtype=torch.int32, device=dev),
                   torch.zeros(0, dtype=torch.float64, device=dev))
    n = 268435456 + 1
    rp = torch.arange(n + 1, dtype=torch.int32, device=dev)
    col = torch.arange(n, dtype=torch.int32, device=dev)
    val = torch.full((n,), 2.0, dtype=torch.float64, device=dev)
    with pytest.raises(_lib.PbcgsError) as e:
        solver.csr(rp, col, val)
    assert e.value.code == _lib.ERR_UNSUPPORTED
    b = torch.ones(n, dtype=torch.float64, device=dev)
    # exactly the maximum: 2I x = 1 converges in one step
    n = 268435456
    op = solver.csr(rp[: n + 1].contiguous(), col[:n].contiguous(), val[:n].contiguous())
    x, info = solver.solve(op, b[:n].contiguous(), tol=1e-12)
    assert info.status == 0 and info.iters == 1
    assert bool(torch.all(x == 0.5))
