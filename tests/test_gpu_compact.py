"""GPU parity of the compact int16 column copy of a CSR operator.

The copy changes only how a product finds its columns (each stored as the
offset from the first row of its row's 64-row block), never the arithmetic:
every solve and product must equal the oracle bit for bit whether the kernels
read the compact copy or the caller's int32 columns (solve flag ``index32``).
The solves here read the CSR stream (``diagonal_layout=False``) even where an
operator also has a diagonal layout, which ``test_gpu_dia.py`` covers.
The edge matrices put columns exactly at the int16 limits -32768 and +32767
around their block start, and one past them (then the operator keeps int32).
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR,
       "ca_bicgstab": oracle.ALG_CA_BICGSTAB, "cg": oracle.ALG_CG, "cgcg": oracle.ALG_CGCG,
       "pipe_cg": oracle.ALG_PIPE_CG}


def edge_matrix(n, fits, seed=7):
    """Unsymmetric, diagonally dominant: 4 on the diagonal, -1 - U[0, 0.2) at
    i +- 1, and far entries U[0.01, 0.1) at base - 32768 and base + 32767
    (base = i & ~63) in every 97th row where they exist; with fits False one
    row also holds base + 32768, which int16 offsets cannot reach."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    far_row = None
    for i in range(n):
        base = i & ~63
        ent = {i: 4.0}
        if i > 0:
            ent[i - 1] = -1.0 - 0.2 * rng.random()
        if i < n - 1:
            ent[i + 1] = -1.0 - 0.2 * rng.random()
        if i % 97 == 5:
            for j in (base - 32768, base + 32767):
                if 0 <= j < n and j not in ent:
                    ent[j] = 0.01 + 0.09 * rng.random()
        if not fits and far_row is None and base + 32768 < n and i % 64 == 3:
            ent[base + 32768] = 0.05
            far_row = i
        for j in sorted(ent):
            rows.append(i)
            cols.append(j)
            vals.append(ent[j])
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, np.asarray(rows) + 1, 1)
    return oracle.CSR(np.cumsum(rp), np.asarray(cols), np.asarray(vals))


def _cases():
    return {
        "edge_fit": edge_matrix(70001, True),     # 70001 = 1093 * 64 + 49: ragged last block
        "edge_nofit": edge_matrix(70001, False),
        "c2_24": oracle.assemble_workload(inputs.workload("c2", n=24)),
        "c2s_24": oracle.assemble_workload(inputs.workload("c2s", n=24)),
    }


CASES = _cases()


def test_edge_matrices_reach_the_limits():
    """The fitting matrix holds offsets -32768 and +32767 exactly; the other
    one offset +32768 (host check of the test inputs themselves)."""
    for name, lo, hi in (("edge_fit", -32768, 32767), ("edge_nofit", -32768, 32768)):
        A = CASES[name]
        rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
        off = A.col.astype(np.int64) - (rows & ~63)
        assert off.min() == lo and off.max() == hi, (name, off.min(), off.max())


def test_index_bytes():
    require_gpu()
    assert csr_op(CASES["edge_fit"]).index_bytes == 2
    assert csr_op(CASES["edge_nofit"]).index_bytes == 4
    assert csr_op(CASES["c2_24"]).index_bytes == 2
    assert solver.stencil(8, 8, 8, [-1, -1, -1, 6, -1, -1, -1]).index_bytes == 0
    assert solver.transpose(csr_op(CASES["c2_24"])).index_bytes == 2


@pytest.mark.parametrize("name", ["edge_fit", "edge_nofit", "c2_24"])
def test_spmv_bitwise(name):
    require_gpu()
    A = CASES[name]
    x = inputs.random_vector(A.n, 11)
    y = host(solver.spmv(csr_op(A), dev_t(x)))
    assert same(y, oracle.spmv(A, x)), float(np.abs(y - oracle.spmv(A, x)).max())


def _solve_both(A, variant, precond, tol, maxit, rr=20, precision="fp64"):
    b = oracle.spmv(A, inputs.x_true(A.n))
    op = csr_op(A)
    out = []
    for index32 in (False, True):
        say(f"compact: n={A.n} {variant} precond={precond} precision={precision} index32={index32}")
        x, info = solver.solve(op, dev_t(b), variant=variant, precond=precond, tol=tol, maxit=maxit,
                               rr_period=rr, history=True, precision=precision, index32=index32,
                               diagonal_layout=False)
        out.append((host(x), info))
    return b, out


def _oracle(A, b, variant, precond, tol, maxit, rr=20):
    dv = oracle.jacobi_dinv(A) if precond else None
    solve = oracle.solve_folded if precond == "jacobi_folded" else oracle.solve
    return solve(A, b, algo=ALG[variant], dinv=dv, tol=tol, maxit=maxit, rr_period=rr, history=True)


def _check(out, x_or, i_or):
    for x, info in out:
        assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
        assert same(x, x_or), float(np.abs(x - x_or).max())
        assert same(host(info.history), i_or["history"])
        assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])


@pytest.mark.parametrize("variant,precond", [
    ("bicgstab", None), ("bicgstab", "jacobi"), ("bicgstab", "jacobi_folded"),
    ("pbicgstab", None), ("pbicgstab_rr", "jacobi"), ("pbicgstab_rr", "jacobi_folded"),
    ("ca_bicgstab", None), ("ca_bicgstab", "jacobi_folded")])
@pytest.mark.parametrize("name", ["edge_fit", "c2_24"])
def test_solve_bitwise_both_index_forms(name, variant, precond):
    require_gpu()
    A = CASES[name]
    b, out = _solve_both(A, variant, precond, 1e-10, 400)
    x_or, i_or = _oracle(A, b, variant, precond, 1e-10, 400)
    _check(out, x_or, i_or)
    assert out[0][1].status == 0


@pytest.mark.parametrize("variant", ["cg", "cgcg", "pipe_cg"])
def test_cg_family_bitwise_both_index_forms(variant):
    require_gpu()
    A = CASES["c2s_24"]
    b, out = _solve_both(A, variant, "jacobi", 1e-10, 400)
    x_or, i_or = _oracle(A, b, variant, "jacobi", 1e-10, 400)
    _check(out, x_or, i_or)


@pytest.mark.parametrize("name", ["edge_fit", "c2_24"])
def test_precision_form_bitwise_both_index_forms(name):
    require_gpu()
    A = CASES[name]
    b, out = _solve_both(A, "pbicgstab_rr", "jacobi_folded", 1e-10, 800, precision="fp32_rr64")
    x_or, i_or = oracle.solve_mp(A, b, dinv=oracle.jacobi_dinv(A), tol=1e-10, maxit=800, rr_period=20,
                                 history=True)
    _check(out, x_or, i_or)


def test_values_may_change_between_solves():
    """The compact copy holds only columns: new values in val are used."""
    require_gpu()
    A = CASES["edge_fit"]
    rp, col, val = dev_t(A.row_ptr), dev_t(A.col), dev_t(A.val)
    op = solver.csr(rp, col, val)
    assert op.index_bytes == 2
    A2 = oracle.CSR(A.row_ptr, A.col, A.val * 1.5)
    val.mul_(1.5)
    torch.cuda.synchronize()
    b = oracle.spmv(A2, inputs.x_true(A.n))
    x, info = solver.solve(op, dev_t(b), variant="pbicgstab_rr", precond="jacobi_folded", tol=1e-10, maxit=400,
                           rr_period=20, diagonal_layout=False)
    x_or, i_or = oracle.solve_folded(A2, b, algo=oracle.ALG_PBICGSTAB_RR, dinv=oracle.jacobi_dinv(A2), tol=1e-10,
                                     maxit=400, rr_period=20)
    assert info.iters == i_or["iters"] and same(host(x), x_or)


def tail_matrix(n, odd_nnz, empty_tail, seed):
    """Banded random matrix (0 to 5 entries per row within +-40 of the
    diagonal, whole empty 64-row blocks in the middle, the last `empty_tail`
    rows empty) with nnz of the requested parity: exercises the pair loads'
    odd starts, empty blocks and the end of the non-zero array."""
    rng = np.random.default_rng([seed, n, int(odd_nnz), empty_tail])
    rows, cols = [], []
    for i in range(n - empty_tail):
        if (i // 64) % 7 == 3:
            continue  # an empty block
        cnt = int(rng.integers(0, 6))
        lo, hi = max(0, i - 40), min(n, i + 41)
        for j in sorted(rng.choice(np.arange(lo, hi), size=min(cnt, hi - lo), replace=False)):
            rows.append(i)
            cols.append(int(j))
    if (len(cols) % 2 == 1) != odd_nnz:
        rows.pop(0)
        cols.pop(0)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, np.asarray(rows, dtype=np.int64) + 1, 1)
    vals = rng.uniform(-1.0, 1.0, len(cols))
    return oracle.CSR(np.cumsum(rp), np.asarray(cols), vals)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 5001])
@pytest.mark.parametrize("odd_nnz", [False, True])
@pytest.mark.parametrize("empty_tail", [0, 70])
def test_spmv_pair_loads_at_the_edges(n, odd_nnz, empty_tail):
    require_gpu()
    empty_tail = min(empty_tail, n - 1)
    A = tail_matrix(n, odd_nnz, empty_tail, 5)
    if A.nnz == 0:
        pytest.skip("no non-zeros at this size")
    assert (A.nnz % 2 == 1) == odd_nnz
    say(f"pair loads: n={n} nnz={A.nnz} empty_tail={empty_tail}")
    op = csr_op(A)
    assert op.index_bytes == 2
    x = inputs.random_vector(A.n, 13)
    y = host(solver.spmv(op, dev_t(x)))
    assert same(y, oracle.spmv(A, x))


# ---- the diagonal-coded form: at most 64 distinct diagonals, offsets beyond int16

def grid7(nx, ny, nz, seed, symmetric=False):
    """3-D 7-point operator on an nx x ny x nz grid (x fastest): diagonally
    dominant, unsymmetric U[0.5, 1.5) couplings unless `symmetric`; with
    nx * ny > 32767 the +-nx*ny diagonals do not fit the int16 block offsets."""
    rng = np.random.default_rng([seed, nx, ny, nz])
    n = nx * ny * nz
    i = np.arange(n)
    x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
    offs = [(-nx * ny, z > 0), (-nx, y > 0), (-1, x > 0), (0, np.ones(n, bool)),
            (1, x < nx - 1), (nx, y < ny - 1), (nx * ny, z < nz - 1)]
    rows, cols, vals = [], [], []
    for d, ok in offs:
        r = i[ok]
        rows.append(r)
        cols.append(r + d)
        if d == 0:
            vals.append(np.full(r.size, 8.0))
        elif symmetric:
            vals.append(-np.ones(r.size))
        else:
            vals.append(-rng.uniform(0.5, 1.5, r.size))
    r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    o = np.lexsort((c, r))
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    return oracle.CSR(np.cumsum(rp), c[o], v[o])


def diag_set_matrix(n, diags, seed, odd_nnz=None, empty_tail=0):
    """Random matrix whose entries lie on the given diagonals only (each
    present with probability 0.6, the main diagonal always, 0 to be dominant)."""
    rng = np.random.default_rng([seed, n, len(diags)])
    rows, cols = [], []
    for d in diags:
        r = np.arange(max(0, -d), min(n, n - d))
        r = r[r < n - empty_tail]
        if d != 0:
            r = r[rng.random(r.size) < 0.6]
        rows.append(r)
        cols.append(r + d)
    r, c = np.concatenate(rows), np.concatenate(cols)
    if odd_nnz is not None and (r.size % 2 == 1) != odd_nnz:
        keep = np.ones(r.size, bool)
        keep[np.flatnonzero(c != r)[0]] = False
        r, c = r[keep], c[keep]
    v = np.where(c == r, float(len(diags)) + 1.0, rng.uniform(-1.0, 1.0, r.size))
    o = np.lexsort((c, r))
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    return oracle.CSR(np.cumsum(rp), c[o], v[o])


WIDE = [-40000, -33000, -200, -1, 0, 1, 200, 33000, 40000]
DCASES = {
    "grid_200x200x3": grid7(200, 200, 3, 1),
    "grid_200x200x3_sym": grid7(200, 200, 3, 2, symmetric=True),
    "diag64": diag_set_matrix(70001, sorted(set([0] + [s * (33000 + 7 * k) for k in range(32) for s in (1, -1)][:63])), 3),
    "diag65": diag_set_matrix(70001, sorted(set([0] + [s * (33000 + 7 * k) for k in range(33) for s in (1, -1)][:64])), 3),
}


def test_diag_inputs():
    """Host check of the test inputs: 64 and 65 distinct diagonals, offsets beyond int16."""
    for name, want in (("diag64", 64), ("diag65", 65), ("grid_200x200x3", 7)):
        A = DCASES[name]
        rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
        assert np.unique(A.col - rows).size == want, name
        assert np.abs(A.col - (rows & ~63)).max() > 32767, name


def test_column_forms():
    require_gpu()
    assert csr_op(CASES["c2_24"]).column_form == "block16"
    assert csr_op(DCASES["grid_200x200x3"]).column_form == "diag16"
    assert csr_op(DCASES["diag64"]).column_form == "diag16"
    assert csr_op(DCASES["diag65"]).column_form == "int32"
    assert csr_op(DCASES["diag65"]).index_bytes == 4
    assert csr_op(DCASES["diag64"]).index_bytes == 2
    assert solver.stencil(8, 8, 8, [-1, -1, -1, 6, -1, -1, -1]).column_form == "none"
    assert solver.transpose(csr_op(DCASES["grid_200x200x3"])).column_form == "diag16"


@pytest.mark.parametrize("name", list(DCASES))
def test_diag_spmv_bitwise(name):
    require_gpu()
    A = DCASES[name]
    x = inputs.random_vector(A.n, 17)
    y = host(solver.spmv(csr_op(A), dev_t(x)))
    assert same(y, oracle.spmv(A, x))


@pytest.mark.parametrize("n", [65, 1000, 70001])
@pytest.mark.parametrize("odd_nnz", [False, True])
@pytest.mark.parametrize("empty_tail", [0, 70])
def test_diag_spmv_at_the_edges(n, odd_nnz, empty_tail):
    """Odd and even nnz, empty trailing rows and ragged blocks in the coded form."""
    require_gpu()
    empty_tail = min(empty_tail, n // 2)
    diags = [d for d in WIDE if abs(d) < n] + [n - 1, -(n - 1)] if n > 40000 else [-(n - 1), -3, 0, 5, n - 1]
    A = diag_set_matrix(n, sorted(set(diags)), 9, odd_nnz=odd_nnz, empty_tail=empty_tail)
    assert (A.nnz % 2 == 1) == odd_nnz
    op = csr_op(A)
    want = "diag16" if n > 32767 + 64 else "block16"
    assert op.column_form == want
    say(f"diag edges: n={n} nnz={A.nnz} form={want}")
    x = inputs.random_vector(A.n, 19)
    assert same(host(solver.spmv(op, dev_t(x))), oracle.spmv(A, x))


@pytest.mark.parametrize("variant,precond", [
    ("bicgstab", None), ("bicgstab", "jacobi_folded"), ("pbicgstab", "jacobi"),
    ("pbicgstab_rr", None), ("pbicgstab_rr", "jacobi"), ("pbicgstab_rr", "jacobi_folded"),
    ("ca_bicgstab", "jacobi_folded")])
def test_diag_solves_bitwise_both_index_forms(variant, precond):
    require_gpu()
    A = DCASES["grid_200x200x3"]
    b, out = _solve_both(A, variant, precond, 1e-10, 300)
    x_or, i_or = _oracle(A, b, variant, precond, 1e-10, 300)
    _check(out, x_or, i_or)
    assert out[0][1].status == 0


@pytest.mark.parametrize("variant", ["cg", "pipe_cg"])
def test_diag_cg_family_bitwise(variant):
    require_gpu()
    A = DCASES["grid_200x200x3_sym"]
    b, out = _solve_both(A, variant, "jacobi", 1e-10, 300)
    x_or, i_or = _oracle(A, b, variant, "jacobi", 1e-10, 300)
    _check(out, x_or, i_or)


def test_diag_precision_form_bitwise():
    require_gpu()
    A = DCASES["grid_200x200x3"]
    b, out = _solve_both(A, "pbicgstab_rr", "jacobi_folded", 1e-10, 600, precision="fp32_rr64")
    x_or, i_or = oracle.solve_mp(A, b, dinv=oracle.jacobi_dinv(A), tol=1e-10, maxit=600, rr_period=20, history=True)
    _check(out, x_or, i_or)


def test_alternating_forms_reuse_cached_graphs():
    """Solves alternate between the compact and the int32 columns of one
    operator: each form replays its own cached graphs (the cache is keyed on
    the operator's bytes) and every solve equals the oracle bit for bit."""
    require_gpu()
    A = CASES["c2_24"]
    b = oracle.spmv(A, inputs.x_true(A.n))
    x_or, i_or = oracle.solve_folded(A, b, algo=oracle.ALG_PBICGSTAB_RR, dinv=oracle.jacobi_dinv(A), tol=1e-10,
                                     maxit=400, rr_period=20)
    op = csr_op(A)
    for rep in range(3):
        for index32 in (False, True, False):
            x, info = solver.solve(op, dev_t(b), variant="pbicgstab_rr", precond="jacobi_folded", tol=1e-10,
                                   maxit=400, rr_period=20, index32=index32, diagonal_layout=False)
            assert info.iters == i_or["iters"] and same(host(x), x_or), (rep, index32)
