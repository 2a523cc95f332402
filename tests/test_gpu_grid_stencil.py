"""GPU parity of the matrix-free stencils with 27 points or per-row coefficients.

``pbcgs_op_stencil`` takes 5-, 7- or 27-point stencils with one set of
constant coefficients or with coefficients per row (a device array, term d
of row r at coef[d * n + r]).  Its products and solves must equal, bit for
bit, the oracle's on the equivalent CSR matrix, which the tests build on the
host from the same coefficients (entries that leave the grid dropped, each
row's terms in ascending column order).  Grids with sides of 1 and 2, odd and
even x extents; every solver, Jacobi form, the precision form, the
allocation-free entry point, poisoned workspaces, and the refused uses.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1612_01395_amd import _lib, inputs, solver
from gpu_util import dev_t, host, require_gpu, same, say

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR,
       "ca_bicgstab": oracle.ALG_CA_BICGSTAB, "cg": oracle.ALG_CG, "cgcg": oracle.ALG_CGCG,
       "pipe_cg": oracle.ALG_PIPE_CG}


def offsets(npts):
    """(dx, dy, dz) of each term, in ascending column order."""
    if npts == 5:
        return [(0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0)]
    if npts == 7:
        return [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    return [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def pattern(nx, ny, nz, npts):
    """present[r, d] and col[r, d] of every row and term."""
    n = nx * ny * nz
    r = np.arange(n)
    i, j, k = r % nx, (r // nx) % ny, r // (nx * ny)
    present = np.zeros((n, npts), bool)
    col = np.zeros((n, npts), np.int64)
    for d, (dx, dy, dz) in enumerate(offsets(npts)):
        present[:, d] = (0 <= i + dx) & (i + dx < nx) & (0 <= j + dy) & (j + dy < ny) & (0 <= k + dz) & (k + dz < nz)
        col[:, d] = r + dz * nx * ny + dy * nx + dx
    return present, col


def to_csr(nx, ny, nz, npts, coef_rows):
    """The equivalent CSR matrix of per-row coefficients coef_rows[d, r]."""
    present, col = pattern(nx, ny, nz, npts)
    vals = coef_rows.T  # [r, d]
    rp = np.zeros(present.shape[0] + 1, np.int64)
    rp[1:] = np.cumsum(present.sum(1))
    return oracle.CSR(rp.astype(np.int32), col[present].astype(np.int32), np.ascontiguousarray(vals[present]))


def random_coefs(nx, ny, nz, npts, seed, symmetric=False):
    """Per-row coefficients [npts, n]: off-diagonal in [-1, 0) (symmetric on
    request), the centre the sum of the row's |off-diagonals| plus 0.5..1.5,
    so the matrix is diagonally dominant (positive definite when symmetric)."""
    rng = np.random.default_rng(seed)
    n = nx * ny * nz
    present, col = pattern(nx, ny, nz, npts)
    c = np.zeros((npts, n))
    centre = npts // 2
    if symmetric:
        # one weight per edge, shared by both rows it joins
        w = {}
        for d in range(npts):
            if d == centre:
                continue
            for r in np.nonzero(present[:, d])[0]:
                key = (min(r, col[r, d]), max(r, col[r, d]))
                if key not in w:
                    w[key] = -rng.uniform(0.1, 1.0)
                c[d, r] = w[key]
    else:
        c[:] = -rng.uniform(0.1, 1.0, (npts, n))
    c[centre] = 0.0
    c[centre] = np.abs(np.where(present.T, c, 0.0)).sum(0) + rng.uniform(0.5, 1.5, n)
    c[~present.T] = np.nan  # slots of terms that leave the grid: never read
    return c


GRIDS = [(1, 1, 1), (1, 5, 3), (3, 1, 7), (2, 2, 2), (7, 9, 1), (65, 3, 2), (12, 11, 10), (64, 5, 4)]


@pytest.mark.parametrize("nx,ny,nz", GRIDS)
@pytest.mark.parametrize("npts", [5, 7, 27])
@pytest.mark.parametrize("per_row", [False, True])
def test_spmv_bitwise(nx, ny, nz, npts, per_row):
    require_gpu()
    if npts == 5 and nz != 1:
        pytest.skip("5-point stencils are 2-D")
    n = nx * ny * nz
    rng = np.random.default_rng(n + npts)
    if per_row:
        c = rng.standard_normal((npts, n))
        c[~pattern(nx, ny, nz, npts)[0].T] = np.nan  # never read
        op = solver.stencil(nx, ny, nz, dev_t(c.reshape(-1)))
    else:
        const = rng.standard_normal(npts)
        c = np.repeat(const[:, None], n, axis=1)
        op = solver.stencil(nx, ny, nz, list(const))
    A = to_csr(nx, ny, nz, npts, c)
    x = rng.standard_normal(n) * np.exp(rng.uniform(-5, 5, n))
    say(f"grid stencil spmv {nx}x{ny}x{nz} npts={npts} per_row={per_row} nnz={A.nnz}")
    assert same(host(solver.spmv(op, dev_t(x))), oracle.spmv(A, x))


def _case(kind, seed=1):
    """(nx, ny, nz, npts, coef[npts, n], per_row, symmetric)"""
    if kind == "27_per_row":
        return (12, 11, 10, 27, random_coefs(12, 11, 10, 27, seed), True)
    if kind == "7_per_row":
        return (13, 11, 9, 7, random_coefs(13, 11, 9, 7, seed), True)
    if kind == "5_per_row":
        return (40, 37, 1, 5, random_coefs(40, 37, 1, 5, seed), True)
    if kind == "27_const":
        nx, ny, nz = 14, 12, 10
        const = np.array([-0.3 - 0.01 * d for d in range(27)])
        const[13] = 12.0  # the off-diagonal magnitudes sum to 11.18
        return (nx, ny, nz, 27, np.repeat(const[:, None], nx * ny * nz, axis=1), False)
    raise ValueError(kind)


def _op(nx, ny, nz, npts, c, per_row, ctx=None):
    if per_row:
        return solver.stencil(nx, ny, nz, dev_t(np.ascontiguousarray(c).reshape(-1)), ctx=ctx)
    return solver.stencil(nx, ny, nz, list(c[:, 0]), ctx=ctx)


def _compare(kind, variant, precond, precision="fp64", poison=False, seed=1):
    nx, ny, nz, npts, c, per_row = _case(kind, seed)
    A = to_csr(nx, ny, nz, npts, c)
    b = oracle.spmv(A, inputs.x_true(A.n))
    d = oracle.jacobi_dinv(A) if precond else None
    kw = dict(tol=1e-10, maxit=2000, rr_period=20)
    if precision == "fp32_rr64":
        x_or, i_or = oracle.solve_mp(A, b, dinv=d, history=True, **kw)
    elif precond == "jacobi_folded":
        x_or, i_or = oracle.solve_folded(A, b, algo=ALG[variant], dinv=d, history=True, **kw)
    else:
        x_or, i_or = oracle.solve(A, b, algo=ALG[variant], dinv=d, history=True, **kw)
    say(f"grid stencil solve {kind} {variant} precond={precond} {precision} poison={poison}")
    op = _op(nx, ny, nz, npts, c, per_row)
    x, info = solver.solve(op, dev_t(b), variant=variant, precond=precond, precision=precision, history=True,
                           poison=poison, **kw)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
    assert same(host(x), x_or), float(np.abs(host(x) - x_or).max())
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])
    assert same(host(info.history), i_or["history"])
    return info


@pytest.mark.parametrize("kind", ["27_per_row", "7_per_row", "5_per_row", "27_const"])
@pytest.mark.parametrize("precond", [None, "jacobi", "jacobi_folded"])
@pytest.mark.parametrize("variant", ["bicgstab", "pbicgstab", "pbicgstab_rr"])
def test_bicgstab_family_bitwise(kind, variant, precond):
    require_gpu()
    assert _compare(kind, variant, precond).status == 0


@pytest.mark.parametrize("kind", ["27_per_row", "27_const"])
@pytest.mark.parametrize("precond", [None, "jacobi_folded"])
def test_ca_bicgstab_and_precision_form(kind, precond):
    require_gpu()
    _compare(kind, "ca_bicgstab", precond)
    _compare(kind, "pbicgstab_rr", precond, precision="fp32_rr64")


@pytest.mark.parametrize("variant", ["cg", "cgcg", "pipe_cg"])
@pytest.mark.parametrize("precond", [None, "jacobi"])
def test_cg_family_on_symmetric_per_row_coefficients(variant, precond):
    require_gpu()
    nx, ny, nz, npts = 9, 8, 7, 27
    c = random_coefs(nx, ny, nz, npts, 5, symmetric=True)
    A = to_csr(nx, ny, nz, npts, c)
    dense = np.zeros((A.n, A.n))
    for r in range(A.n):
        dense[r, A.col[A.row_ptr[r]:A.row_ptr[r + 1]]] = A.val[A.row_ptr[r]:A.row_ptr[r + 1]]
    assert np.array_equal(dense, dense.T)
    b = oracle.spmv(A, inputs.x_true(A.n))
    d = oracle.jacobi_dinv(A) if precond else None
    x_or, i_or = oracle.solve(A, b, algo=ALG[variant], dinv=d, tol=1e-10, maxit=2000, history=True)
    say(f"grid stencil {variant} precond={precond}")
    x, info = solver.solve(_op(nx, ny, nz, npts, c, True), dev_t(b), variant=variant, precond=precond, tol=1e-10,
                           maxit=2000, history=True)
    assert (info.status, info.iters) == (i_or["status"], i_or["iters"]) and info.status == 0
    assert same(host(x), x_or) and same(host(info.history), i_or["history"])


@pytest.mark.parametrize("kind", ["27_per_row", "7_per_row"])
def test_poisoned_workspace(kind):
    require_gpu()
    _compare(kind, "pbicgstab_rr", "jacobi_folded", poison=True)
    _compare(kind, "pbicgstab_rr", "jacobi_folded", precision="fp32_rr64", poison=True)


def test_noalloc_folded_per_row():
    require_gpu()
    nx, ny, nz, npts, c, per_row = _case("27_per_row")
    A = to_csr(nx, ny, nz, npts, c)
    b = oracle.spmv(A, inputs.x_true(A.n))
    kw = dict(tol=1e-10, maxit=2000, rr_period=20)
    x_or, i_or = oracle.solve_folded(A, b, algo=oracle.ALG_PBICGSTAB_RR, dinv=oracle.jacobi_dinv(A), **kw)
    op = _op(nx, ny, nz, npts, c, per_row)
    for _ in range(2):
        x = dev_t(np.zeros(A.n))
        x, info = solver.solve_noalloc(op, dev_t(b), x, variant="pbicgstab_rr", precond="jacobi_folded", **kw)
        assert info.iters == i_or["iters"] and same(host(x), x_or)


def test_coefficients_change_in_place():
    """Per-row coefficients are borrowed: a change between solves is seen."""
    require_gpu()
    nx, ny, nz, npts, c, _ = _case("7_per_row")
    cd = dev_t(np.ascontiguousarray(c).reshape(-1))
    op = solver.stencil(nx, ny, nz, cd)
    x = inputs.random_vector(nx * ny * nz, 2)
    assert same(host(solver.spmv(op, dev_t(x))), oracle.spmv(to_csr(nx, ny, nz, npts, c), x))
    c2 = c * 0.5  # absent slots stay NaN
    cd.copy_(dev_t(np.ascontiguousarray(c2).reshape(-1)))
    assert same(host(solver.spmv(op, dev_t(x))), oracle.spmv(to_csr(nx, ny, nz, npts, c2), x))


def test_refused_uses():
    require_gpu()
    ctx = solver.default_context()
    L = _lib.lib()
    h = _lib.ctypes.c_void_p()
    arr = (_lib.ctypes.c_double * 27)(*([1.0] * 27))
    p = _lib.ctypes.cast(arr, _lib.ctypes.c_void_p)
    for args in ((4, 4, 4, 9, 0), (4, 4, 2, 5, 0), (4, 4, 4, 7, 2), (0, 4, 4, 7, 0)):
        assert L.pbcgs_op_stencil(ctx.handle, *args[:4], p, args[4], _lib.ctypes.byref(h)) == _lib.ERR_INVALID_ARG
    # a zero centre coefficient with Jacobi
    nx, ny, nz, npts, c, _ = _case("7_per_row")
    c = c.copy()
    c[3, 17] = 0.0
    op = _op(nx, ny, nz, npts, c, True)
    b = dev_t(np.ones(nx * ny * nz))
    with pytest.raises(_lib.PbcgsError) as e:
        solver.solve(op, b, precond="jacobi")
    assert e.value.code == _lib.ERR_INVALID_ARG
    with pytest.raises(_lib.PbcgsError) as e:
        solver.transpose(op)
    assert e.value.code == _lib.ERR_UNSUPPORTED
    with pytest.raises(_lib.PbcgsError) as e:
        solver.solve_batched([op], [b])
    assert e.value.code == _lib.ERR_UNSUPPORTED
    # folded Jacobi with a non-constant dinv on constant coefficients
    nx, ny, nz, npts, c, _ = _case("27_const")
    op = _op(nx, ny, nz, npts, c, False)
    dv = dev_t(np.linspace(0.1, 0.2, nx * ny * nz))
    with pytest.raises(_lib.PbcgsError) as e:
        solver.solve(op, dev_t(np.ones(nx * ny * nz)), precond="jacobi_folded", dinv=dv)
    assert e.value.code == _lib.ERR_UNSUPPORTED


@pytest.mark.parametrize("kind", ["27_per_row", "7_per_row", "5_per_row", "27_const"])
@pytest.mark.parametrize("variant,precision", [("bicgstab", "fp64"), ("pbicgstab_rr", "fp64"),
                                               ("pbicgstab_rr", "fp32_rr64")])
@pytest.mark.parametrize("precond", [None, "jacobi_folded"])
def test_two_rows_per_lane(kind, variant, precision, precond, monkeypatch):
    """Few workgroups, so every wave owns several blocks and the kernels take
    two rows per lane: with an even x extent (27_per_row, 5_per_row,
    27_const) through aligned pairs shared by the lane's two rows, with an odd
    one (7_per_row) row by row; the same bits either way."""
    require_gpu()
    monkeypatch.setenv("PBCGS_GTARGET", "2")
    info = _compare(kind, variant, precond, precision=precision)
    assert info.shape[0] >= 2
