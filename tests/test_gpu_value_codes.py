"""GPU parity of value indexing in the diagonal layout (``SolveInfo.value_codes``).

When a CSR operator's layout has at most 8 diagonals, none of which holds more
than 16 distinct values (after folding Jacobi in; binary64, or binary32 and
binary64 for the precision form), and no Jacobi vector is applied (none,
folded, or Jacobi by a constant diagonal), a solve reads each entry's value
as a one-byte code into its diagonal's table of values (one 8-byte word of
codes per row).
The products use the same binary64 values in the same order, so every solve
must equal the oracle bit for bit, and equal the same solve with the codes
switched off (``PBCGS_VALUE_CODES=0``):

* which solves use codes: constant-coefficient workloads without, with
  folded and with literal Jacobi by a constant diagonal do, and so do 8
  constant diagonals and a diagonal of two values folded; variable
  coefficients (27-point, random bands), 9 diagonals, literal Jacobi by a
  vector and the switch do not; without the switch only from 2^18 rows up (the
  other tests force them with ``PBCGS_VALUE_CODES=1``);
* a table's capacity: 16 distinct values on a diagonal (among them +0 and -0,
  distinct bit patterns) use codes, 17 do not;
* every BiCGStab variant and the CG family, with one and two rows per lane,
  on an odd row count;
* the binary32 form with binary32 and binary64 tables, with one, two and
  four rows per lane, offsets of every residue modulo 4 and ragged fours;
* values changed between solves: the codes are made again for each solve,
  and a solve whose values no longer fit falls back to the values.
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


def _solve(A, op, variant, precond, codes, monkeypatch, **kw):
    monkeypatch.setenv("PBCGS_VALUE_CODES", "1" if codes else "0")
    b = oracle.spmv(A, inputs.x_true(A.n))
    x, info = solver.solve(op, dev_t(b), variant=variant, precond=precond, history=True, **kw)
    d = oracle.jacobi_dinv(A)
    if precond == "jacobi_folded":
        x_or, i_or = oracle.solve_folded(A, b, algo=ALG[variant], dinv=d, history=True, **kw)
    else:
        x_or, i_or = oracle.solve(A, b, algo=ALG[variant], dinv=d if precond else None, history=True, **kw)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
    assert same(host(x), x_or), float(np.abs(host(x) - x_or).max())
    assert same(host(info.history), i_or["history"])
    return host(x), info


def coded_band(n, per_diag, seed, extra=None):
    """A banded matrix on diagonal 0 and the offsets d of per_diag whose
    off-diagonal entries take per_diag[d] distinct values (cycled by row;
    diagonal -2 holds +0 and -0 among them), with a constant dominant
    diagonal, so that folding Jacobi keeps the counts.  ``extra`` =
    (offset, row, value) sets one entry."""
    offs = sorted(set(per_diag) | {0})
    rows, cols, vals = [], [], []
    for i in range(n):
        for o in offs:
            j = i + o
            if not 0 <= j < n:
                continue
            if o == 0:
                v = 0.0  # set below
            else:
                k = per_diag[o]
                pool = np.linspace(-1.0, 1.0, k) + 0.01 * o
                if o == -2:
                    pool[0], pool[1] = 0.0, -0.0
                v = pool[(i * 7 + seed) % k]
            rows.append(i)
            cols.append(j)
            vals.append(v)
    vals = np.asarray(vals)
    vals[np.asarray(rows) == np.asarray(cols)] = 1.0 + 2.0 * sum(1 for o in offs if o != 0)
    if extra is not None:
        o, r, v = extra
        hit = [k for k in range(len(rows)) if rows[k] == r and cols[k] == r + o]
        vals[hit[0]] = v
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, np.asarray(rows) + 1, 1)
    return oracle.CSR(np.cumsum(rp).astype(np.int32), np.asarray(cols, np.int32), vals)


def test_which_solves_use_codes(monkeypatch):
    require_gpu()
    c2 = oracle.assemble_workload(inputs.workload("c2", n=24))
    c3 = oracle.assemble_workload(inputs.workload("c3", n=10), inputs.kappa_cells(10))
    kw = dict(tol=1e-10, maxit=600, rr_period=13)
    # a Jacobi vector: a banded matrix whose diagonal takes two values
    V = coded_band(2000, {-9: 2, -1: 3, 1: 3, 9: 2}, seed=4)
    dg = np.repeat(np.arange(V.n), np.diff(V.row_ptr)) == V.col
    V.val[dg] = np.where(np.arange(V.n) % 2 == 0, 9.0, 11.0)
    for A, precond, codes, want in ((c2, "jacobi_folded", True, True), (c2, None, True, True),
                                    (c2, "jacobi", True, True), (c2, "jacobi_folded", False, False),
                                    (V, "jacobi", True, False), (V, "jacobi_folded", True, True),
                                    (c3, "jacobi_folded", True, False), (c3, None, True, False)):
        op = csr_op(A)
        assert op.diagonals > 0
        say(f"value codes: n={A.n} precond={precond} switch={codes}")
        _, info = _solve(A, op, "pbicgstab_rr", precond, codes, monkeypatch, **kw)
        assert info.value_codes == want, (A.n, precond, codes)
    for nd, want in ((8, True), (9, False)):
        offs = [-40, -17, -3, -1, 1, 2, 5, 33][: nd - 1]
        A = coded_band(2500, {o: 2 for o in offs}, seed=nd)
        op = csr_op(A)
        assert op.diagonals == nd
        say(f"value codes: {nd} diagonals")
        _, info = _solve(A, op, "pbicgstab_rr", "jacobi_folded", True, monkeypatch, **kw)
        assert info.value_codes == want, nd


def test_default_from_2_to_the_18_rows(monkeypatch):
    """Without the switch, codes are taken from 2^18 rows up (below that a
    solve is latency-bound); the results are the oracle's either way."""
    require_gpu()
    monkeypatch.delenv("PBCGS_VALUE_CODES", raising=False)
    kw = dict(tol=1e-10, maxit=600, rr_period=50)
    for n, want in ((24, False), (63, False), (64, True)):
        A = oracle.assemble_workload(inputs.workload("c2", n=n))
        b = oracle.spmv(A, inputs.x_true(A.n))
        say(f"value codes by default: c2 n={n} rows={A.n}")
        x, info = solver.solve(csr_op(A), dev_t(b), variant="pbicgstab_rr", precond="jacobi_folded", **kw)
        x_or, i_or = oracle.solve_folded(A, b, algo=oracle.ALG_PBICGSTAB_RR, dinv=oracle.jacobi_dinv(A), **kw)
        assert info.value_codes == want, n
        assert info.iters == i_or["iters"] and same(host(x), x_or)


@pytest.mark.parametrize("k,want", [(16, True), (17, False)])
@pytest.mark.parametrize("precond", ["jacobi_folded", None])
def test_table_capacity(k, want, precond, monkeypatch):
    require_gpu()
    A = coded_band(3001, {-9: 3, -2: 16, 1: k, 9: 1}, seed=5)
    op = csr_op(A)
    assert op.diagonals == 5
    say(f"value codes: {k} values on a diagonal, precond={precond}")
    x, info = _solve(A, op, "pbicgstab_rr", precond, True, monkeypatch, tol=1e-10, maxit=800, rr_period=9)
    assert info.value_codes == want
    x0, info0 = _solve(A, op, "pbicgstab_rr", precond, False, monkeypatch, tol=1e-10, maxit=800, rr_period=9)
    assert not info0.value_codes and same(x, x0)


@pytest.mark.parametrize("gtarget", [1, 8])
@pytest.mark.parametrize("variant,precond", [
    ("pbicgstab_rr", "jacobi_folded"), ("pbicgstab_rr", None), ("pbicgstab_rr", "jacobi"),
    ("pbicgstab", "jacobi_folded"), ("bicgstab", "jacobi_folded"), ("bicgstab", None), ("bicgstab", "jacobi"),
    ("ca_bicgstab", "jacobi_folded"), ("cg", None), ("cgcg", None), ("pipe_cg", None), ("cg", "jacobi"),
    ("cgcg", "jacobi"), ("pipe_cg", "jacobi")])
def test_variants_bitwise(variant, precond, gtarget, monkeypatch):
    require_gpu()
    monkeypatch.setenv("PBCGS_GTARGET", str(gtarget))
    name = "c2s" if variant in ("cg", "cgcg", "pipe_cg") else "c2"
    A = oracle.assemble_workload(inputs.workload(name, n=23))
    assert A.n % 2 == 1
    op = csr_op(A)
    say(f"value codes: {variant} {precond} {name} n=23 gtarget={gtarget}")
    x, info = _solve(A, op, variant, precond, True, monkeypatch, tol=1e-10, maxit=800, rr_period=17)
    assert info.value_codes
    if gtarget == 1:
        assert info.shape[0] >= 2  # every wave owns several blocks: two rows per lane


def test_values_changed_between_solves(monkeypatch):
    require_gpu()
    monkeypatch.setenv("PBCGS_VALUE_CODES", "1")
    A = coded_band(2000, {-9: 2, -2: 4, 1: 16, 9: 1}, seed=3)
    rp, col, val = dev_t(A.row_ptr), dev_t(A.col), dev_t(A.val)
    op = solver.csr(rp, col, val)
    kw = dict(variant="pbicgstab_rr", precond="jacobi_folded", tol=1e-10, maxit=500, rr_period=20)

    def run(M, want):
        b = oracle.spmv(M, inputs.x_true(M.n))
        x, info = solver.solve(op, dev_t(b), **kw)
        x_or, i_or = oracle.solve_folded(M, b, algo=oracle.ALG_PBICGSTAB_RR, dinv=oracle.jacobi_dinv(M), tol=1e-10,
                                         maxit=500, rr_period=20)
        assert info.value_codes == want
        assert info.iters == i_or["iters"] and same(host(x), x_or)

    run(A, True)
    # one more distinct value on diagonal +1: 17, no codes
    B = coded_band(2000, {-9: 2, -2: 4, 1: 16, 9: 1}, seed=3, extra=(1, 1000, 0.123))
    val.copy_(dev_t(B.val))
    torch.cuda.synchronize()
    run(B, False)
    # scaled back to 16 per diagonal: codes again, with the new values
    C = oracle.CSR(A.row_ptr, A.col, A.val * 1.5)
    val.copy_(dev_t(C.val))
    torch.cuda.synchronize()
    run(C, True)


@pytest.mark.parametrize("gtarget", [1, 2, 8])
@pytest.mark.parametrize("case", ["c2_23", "c1", "band"])
def test_precision_form_bitwise(case, gtarget, monkeypatch):
    """The binary32 form with both layouts value-indexed (binary32 tables for
    the iteration's four- and two-row products, binary64 ones for the
    replacement steps): the oracle's bits, and the same bits as on the
    layouts' values.  The band has offsets of every residue modulo 4 (aligned
    fours, aligned pairs, single loads) and 16 values with +0 and -0 on one
    diagonal; 1003 rows leave a last four with three rows."""
    require_gpu()
    monkeypatch.setenv("PBCGS_GTARGET", str(gtarget))
    if case == "c2_23":
        A = oracle.assemble_workload(inputs.workload("c2", n=23))
    elif case == "c1":
        A = oracle.assemble_workload(inputs.workload("c1"))
    else:
        A = coded_band(1003, {-9: 3, -4: 2, -2: 16, 1: 5, 8: 1}, seed=11)
    op = csr_op(A)
    b = oracle.spmv(A, inputs.x_true(A.n))
    kw = dict(tol=1e-9, maxit=1500, rr_period=10)
    for folded in (True, False):
        d = oracle.jacobi_dinv(A) if folded else None
        x_or, i_or = oracle.solve_mp(A, b, dinv=d, history=True, **kw)
        got = []
        for codes in ("1", "0"):
            monkeypatch.setenv("PBCGS_VALUE_CODES", codes)
            say(f"value codes {codes}: precision form {case} folded={folded} gtarget={gtarget}")
            x, info = solver.solve(op, dev_t(b), variant="pbicgstab_rr", precond="jacobi_folded" if folded else None,
                                   precision="fp32_rr64", history=True, **kw)
            assert info.value_codes == (codes == "1")
            assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (info, i_or)
            assert same(host(x), x_or), float(np.abs(host(x) - x_or).max())
            assert same(host(info.history), i_or["history"])
            got.append(info.shape[0])
        if gtarget == 1:
            assert got[0] >= 4  # every wave owns at least four blocks: four rows per lane
