"""GPU parity of batched solves: independent systems of uneven size in one
batched call, each against its own oracle solve, bit for bit (iterates,
iteration and replacement counts, statuses, residuals).  Systems converge at
different iterations; a stopped system must leave the later launches alone."""

import numpy as np
import pytest
import torch

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR}


def small_batch():
    """2-D and 3-D systems from 1 to ~40K unknowns, uneven convection."""
    sys = []
    rng = np.random.default_rng(5)
    for k, n in enumerate([1, 2, 5, 16, 33, 64, 100, 150, 200]):
        beta = tuple(rng.uniform(0.0, 200.0, 2))
        sys.append(oracle.assemble(2, n, 5, beta))
    for n in (3, 12, 24, 34):
        sys.append(oracle.assemble(3, n, 7, tuple(rng.uniform(0.0, 100.0, 3))))
    return sys


BATCH = small_batch()


@pytest.mark.parametrize("variant", list(ALG))
def test_batched_equals_individual_oracle_solves(variant):
    require_gpu()
    say(f"batched {variant}: {len(BATCH)} systems, N = {[A.n for A in BATCH]}")
    bs = [oracle.spmv(A, inputs.batch_x_true(k, A.n)) for k, A in enumerate(BATCH)]
    ops = [csr_op(A) for A in BATCH]
    kw = dict(tol=1e-10, maxit=3000, rr_period=17)
    xs, infos = solver.solve_batched(ops, [dev_t(b) for b in bs], variant=variant, **kw)
    for k, (A, b) in enumerate(zip(BATCH, bs)):
        x_or, i_or = oracle.solve(A, b, algo=ALG[variant], **kw)
        info = infos[k]
        assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (k, info, i_or)
        assert same(host(xs[k]), x_or), k
        assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]]), k
    # statuses differ in general: the loop above covers successes and the tiny systems' early exits


def test_batched_x0_maxit_and_shapes():
    require_gpu()
    import os
    sub = BATCH[3:8]
    bs = [oracle.spmv(A, inputs.batch_x_true(k, A.n)) for k, A in enumerate(sub)]
    x0s = [inputs.random_vector(A.n, 30 + k) for k, A in enumerate(sub)]
    ops = [csr_op(A) for A in sub]
    for kw in (dict(tol=0.0, maxit=23, rr_period=5), dict(tol=1e-9, maxit=40, rr_period=0)):
        ref = [oracle.solve(A, b, algo=oracle.ALG_PBICGSTAB_RR, x0=x0, **kw) for A, b, x0 in zip(sub, bs, x0s)]
        old = os.environ.get("PBCGS_BATCH_GCAP")
        try:
            for gcap in ("1", "4", "64"):
                os.environ["PBCGS_BATCH_GCAP"] = gcap
                for graph in (True, False):
                    say(f"batched x0 {kw} gcap={gcap} graph={graph}")
                    xs, infos = solver.solve_batched(ops, [dev_t(b) for b in bs], [dev_t(x0) for x0 in x0s],
                                                     variant="pbicgstab_rr", graph=graph, **kw)
                    for k, (x_or, i_or) in enumerate(ref):
                        assert (infos[k].status, infos[k].iters) == (i_or["status"], i_or["iters"])
                        assert same(host(xs[k]), x_or)
        finally:
            if old is None:
                os.environ.pop("PBCGS_BATCH_GCAP", None)
            else:
                os.environ["PBCGS_BATCH_GCAP"] = old


def test_batched_errors():
    require_gpu()
    from paper_1612_01395_amd import _lib
    A = BATCH[5]
    op = csr_op(A)
    b = dev_t(oracle.spmv(A, inputs.x_true(A.n)))
    st = solver.stencil(8, 8, 1, [-1.0, -1.0, 4.5, -1.0, -1.0])
    with pytest.raises(_lib.PbcgsError):
        solver.solve_batched([op, st], [b, dev_t(np.ones(64))])
    with pytest.raises(ValueError):
        solver.solve_batched([], [])


@pytest.mark.parametrize("variant", ["bicgstab", "pbicgstab_rr"])
def test_batched_compact_and_int32_columns(variant):
    """Every system holds the compact int16 columns, so the batch reads them;
    ``index32`` makes it read the int32 columns.  Both equal each system's own
    oracle solve bit for bit."""
    require_gpu()
    bs = [oracle.spmv(A, inputs.batch_x_true(k, A.n)) for k, A in enumerate(BATCH)]
    ops = [csr_op(A) for A in BATCH]
    assert all(op.column_form == "block16" for op in ops)
    kw = dict(tol=1e-10, maxit=3000, rr_period=17)
    ref = [oracle.solve(A, b, algo=ALG[variant], **kw) for A, b in zip(BATCH, bs)]
    for index32 in (False, True):
        say(f"batched {variant} index32={index32}")
        xs, infos = solver.solve_batched(ops, [dev_t(b) for b in bs], variant=variant, index32=index32, **kw)
        for k, (x_or, i_or) in enumerate(ref):
            assert (infos[k].status, infos[k].iters, infos[k].n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
            assert same(host(xs[k]), x_or), (index32, k)


def test_batched_mixed_column_forms():
    """One system whose columns do not fit the int16 block offsets (it holds
    diagonal codes instead) keeps the whole batch on int32 columns; results
    still equal the oracle's."""
    require_gpu()
    n = 40000
    rows = np.arange(n)
    far = (rows + 33000) % n  # offsets beyond int16 from the block start
    r = np.concatenate([rows, rows])
    c = np.concatenate([rows, far])
    v = np.concatenate([np.full(n, 4.0), np.full(n, 0.5)])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, r + 1, 1)
    wide = oracle.CSR(np.cumsum(rp), c, v)
    sysl = [BATCH[4], wide, BATCH[6]]
    ops = [csr_op(A) for A in sysl]
    assert [op.column_form for op in ops] == ["block16", "diag16", "block16"]
    bs = [oracle.spmv(A, inputs.batch_x_true(k, A.n)) for k, A in enumerate(sysl)]
    kw = dict(tol=1e-10, maxit=500, rr_period=17)
    say("batched mixed column forms")
    xs, infos = solver.solve_batched(ops, [dev_t(b) for b in bs], variant="pbicgstab_rr", **kw)
    for k, (A, b) in enumerate(zip(sysl, bs)):
        x_or, i_or = oracle.solve(A, b, algo=oracle.ALG_PBICGSTAB_RR, **kw)
        assert (infos[k].status, infos[k].iters) == (i_or["status"], i_or["iters"]), k
        assert same(host(xs[k]), x_or), k


def dia_batch():
    """Systems that all have a diagonal layout (2-D 5-point from a single node
    to 257^2, 3-D 7-point up to 34^3), so the batch reads every one of them
    through it, two rows per lane."""
    rng = np.random.default_rng(11)
    sys = [oracle.assemble(2, n, 5, tuple(rng.uniform(0.0, 200.0, 2))) for n in (1, 5, 16, 33, 64, 100, 150, 257)]
    sys += [oracle.assemble(3, n, 7, tuple(rng.uniform(0.0, 100.0, 3))) for n in (12, 24, 34)]
    return sys


DIA_BATCH = dia_batch()


@pytest.mark.parametrize("variant", list(ALG))
def test_batched_diagonal_layout(variant):
    require_gpu()
    ops = [csr_op(A) for A in DIA_BATCH]
    assert all(op.diagonals > 0 for op in ops)
    bs = [oracle.spmv(A, inputs.batch_x_true(k, A.n)) for k, A in enumerate(DIA_BATCH)]
    kw = dict(tol=1e-10, maxit=3000, rr_period=17)
    ref = [oracle.solve(A, b, algo=ALG[variant], **kw) for A, b in zip(DIA_BATCH, bs)]
    for layout in (True, False):
        say(f"batched {variant} diagonal_layout={layout}: N = {[A.n for A in DIA_BATCH]}")
        xs, infos = solver.solve_batched(ops, [dev_t(b) for b in bs], variant=variant, diagonal_layout=layout, **kw)
        for k, (x_or, i_or) in enumerate(ref):
            info = infos[k]
            assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), (layout, k)
            assert same(host(xs[k]), x_or), (layout, k)
            assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]]), (layout, k)


@pytest.mark.parametrize("variant", ["bicgstab", "pbicgstab_rr"])
def test_batched_diagonal_layout_shapes_and_x0(variant, monkeypatch):
    """Per-system workgroup caps from 1 (many blocks per wave) to 64, graph
    replay and direct launches, a non-zero x_0 and a fixed iteration count,
    values changed in place between two batches (the layout's values are laid
    out for each batch)."""
    require_gpu()
    sub = DIA_BATCH[1:8]
    ops = [csr_op(A) for A in sub]
    bs = [oracle.spmv(A, inputs.batch_x_true(k, A.n)) for k, A in enumerate(sub)]
    x0s = [inputs.random_vector(A.n, 40 + k) for k, A in enumerate(sub)]
    kw = dict(tol=0.0, maxit=37, rr_period=5)
    ref = [oracle.solve(A, b, algo=ALG[variant], x0=x0, **kw) for A, b, x0 in zip(sub, bs, x0s)]
    for gcap in ("1", "4", "64"):
        monkeypatch.setenv("PBCGS_BATCH_GCAP", gcap)
        for graph in (True, False):
            say(f"batched diagonal layout {variant} gcap={gcap} graph={graph}")
            xs, infos = solver.solve_batched(ops, [dev_t(b) for b in bs], [dev_t(x0) for x0 in x0s],
                                             variant=variant, graph=graph, **kw)
            for k, (x_or, i_or) in enumerate(ref):
                assert (infos[k].status, infos[k].iters) == (i_or["status"], i_or["iters"]), (gcap, graph, k)
                assert same(host(xs[k]), x_or), (gcap, graph, k)
    monkeypatch.delenv("PBCGS_BATCH_GCAP")
    # values scaled in place: the next batch lays out the new values
    A0 = sub[2]
    rp, col, val = dev_t(A0.row_ptr), dev_t(A0.col), dev_t(A0.val)
    op0 = solver.csr(rp, col, val)
    ops2 = [ops[0], ops[1], op0] + ops[3:]
    solver.solve_batched(ops2, [dev_t(b) for b in bs], variant=variant, tol=1e-10, maxit=500)
    val.mul_(1.5)
    torch.cuda.synchronize()
    A2 = oracle.CSR(A0.row_ptr, A0.col, A0.val * 1.5)
    xs, infos = solver.solve_batched(ops2, [dev_t(b) for b in bs], variant=variant, tol=1e-10, maxit=500)
    x_or, i_or = oracle.solve(A2, bs[2], algo=ALG[variant], tol=1e-10, maxit=500)
    assert infos[2].iters == i_or["iters"] and same(host(xs[2]), x_or)
    x_or, i_or = oracle.solve(sub[3], bs[3], algo=ALG[variant], tol=1e-10, maxit=500)
    assert infos[3].iters == i_or["iters"] and same(host(xs[3]), x_or)


def test_batched_one_system_without_layout_keeps_csr():
    """One system with no diagonal layout (a 2 x 2 grid: 5 diagonals for 12
    entries) puts the whole batch on the CSR arrays; results still equal the
    oracle's."""
    require_gpu()
    sysl = [DIA_BATCH[2], oracle.assemble(2, 2, 5, (10.0, 20.0)), DIA_BATCH[4]]
    ops = [csr_op(A) for A in sysl]
    assert [op.diagonals > 0 for op in ops] == [True, False, True]
    bs = [oracle.spmv(A, inputs.batch_x_true(k, A.n)) for k, A in enumerate(sysl)]
    kw = dict(tol=1e-10, maxit=500, rr_period=17)
    say("batched, one system without a diagonal layout")
    xs, infos = solver.solve_batched(ops, [dev_t(b) for b in bs], variant="pbicgstab_rr", **kw)
    for k, (A, b) in enumerate(zip(sysl, bs)):
        x_or, i_or = oracle.solve(A, b, algo=oracle.ALG_PBICGSTAB_RR, **kw)
        assert (infos[k].status, infos[k].iters) == (i_or["status"], i_or["iters"]), k
        assert same(host(xs[k]), x_or), k
