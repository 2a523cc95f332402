"""GPU parity at the full benchmark sizes, in the launch configuration the
benchmark uses.

* 3-D 7-point 128^3 (2,097,152 unknowns): device assembly, b = A x_true and
  complete p-BiCGStab+RR / BiCGStab / p-BiCGStab solves (Jacobi, tol 1e-8)
  against the oracle, bit for bit; the matrix-free stencil gives the same x.
* the same grid for CA-BiCGStab and the eq. (5) alpha (folded Jacobi), and its
  symmetric counterpart (Poisson) for CG, Chronopoulos & Gear CG and p-CG
  (Jacobi), each complete solve against the oracle bit for bit.
* 3-D 27-point variable-coefficient 256^3 (16,777,216 unknowns, 449,455,096
  non-zeros): assembled rows sampled across the grid against the oracle's
  row-by-row assembly, then the whole matrix, the first iterations and the
  complete RR solve (k = 50, tol 1e-8) against the oracle bit for bit, plus
  properties that hold at any size (true residual, error against x_true).
* 3-D 7-point 256^3 precision form (binary32 + binary64 replacement, folded
  Jacobi, tol 1e-10, k = 20) and its all-binary64 counterpart, each against
  the oracle bit for bit; the binary64 true residual below 1e-10.
* the batched workload, 512 2-D systems (22,324,961 unknowns) in one batched
  call: sampled systems (the smallest, the largest and six others) against
  their oracle solves bit for bit, every system converged with its true
  residual at tol, and the batched adjoint likewise.
"""

import time

import numpy as np
import pytest
import torch

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import dev_t, host, require_gpu, same, say

pytestmark = pytest.mark.gpu

ALG = {"bicgstab": oracle.ALG_BICGSTAB, "pbicgstab": oracle.ALG_PBICGSTAB, "pbicgstab_rr": oracle.ALG_PBICGSTAB_RR}


@pytest.fixture(scope="module")
def c2():
    require_gpu()
    w = inputs.workload("c2")
    t0 = time.time()
    A = oracle.assemble_workload(w)
    rp, col, val = solver.assemble_convdiff(w.dim, w.n, w.npts, w.beta)
    say(f"c2 assembled in {time.time() - t0:.1f}s")
    xt = inputs.x_true(A.n)
    b_or = oracle.spmv(A, xt)
    op = solver.csr(rp, col, val)
    b = solver.spmv(op, dev_t(xt))
    return w, A, (rp, col, val), op, b, b_or


def test_c2_assembly_and_rhs_bitwise(c2):
    w, A, (rp, col, val), op, b, b_or = c2
    assert np.array_equal(host(rp), A.row_ptr)
    assert np.array_equal(host(col), A.col)
    assert same(host(val), A.val)
    assert same(host(b), b_or)


@pytest.mark.parametrize("precond", ["jacobi", "jacobi_folded"])
@pytest.mark.parametrize("variant", ["pbicgstab_rr", "bicgstab", "pbicgstab"])
def test_c2_full_solve_bitwise(c2, variant, precond):
    w, A, _, op, b, b_or = c2
    dinv = oracle.jacobi_dinv(A)
    t0 = time.time()
    solve = oracle.solve_folded if precond == "jacobi_folded" else oracle.solve
    x_or, i_or = solve(A, b_or, algo=ALG[variant], dinv=dinv, tol=w.tol, maxit=w.maxit,
                       rr_period=w.rr_period, history=True)
    say(f"c2 {variant} {precond}: oracle {i_or['iters']} it in {time.time() - t0:.1f}s")
    x, info = solver.solve(op, b, variant=variant, precond=precond, tol=w.tol, maxit=w.maxit,
                           rr_period=w.rr_period, history=True)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
    assert same(host(x), x_or)
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])
    assert same(host(info.history), i_or["history"])
    # the stated accuracy bound ||x - x_oracle|| <= 1e-8 ||x_oracle||, met trivially by bitwise equality
    assert np.linalg.norm(host(x) - x_or) <= 1e-8 * np.linalg.norm(x_or)


@pytest.mark.parametrize("variant,alpha_form", [("ca_bicgstab", 3), ("pbicgstab_rr", 5)])
def test_c2_other_algorithms_bitwise(c2, variant, alpha_form):
    """CA-BiCGStab (Algorithm 8) and the eq. (5) alpha at the benchmark's size
    and launch configuration (folded Jacobi)."""
    w, A, _, op, b, b_or = c2
    algo = oracle.ALG_CA_BICGSTAB if variant == "ca_bicgstab" else ALG[variant]
    t0 = time.time()
    x_or, i_or = oracle.solve_folded(A, b_or, algo=algo, dinv=oracle.jacobi_dinv(A), tol=w.tol, maxit=w.maxit,
                                     rr_period=w.rr_period, history=True, alpha_form=alpha_form)
    say(f"c2 {variant} eq.({alpha_form}): oracle {i_or['iters']} it in {time.time() - t0:.1f}s")
    x, info = solver.solve(op, b, variant=variant, precond="jacobi_folded", tol=w.tol, maxit=w.maxit,
                           rr_period=w.rr_period, history=True, alpha_form=alpha_form)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
    assert info.status == 0
    assert same(host(x), x_or)
    assert same(host(info.history), i_or["history"])


@pytest.fixture(scope="module")
def c2s():
    require_gpu()
    w = inputs.workload("c2s")
    A = oracle.assemble_workload(w)
    rp, col, val = solver.assemble_convdiff(w.dim, w.n, w.npts, w.beta)
    assert np.array_equal(host(rp), A.row_ptr) and same(host(val), A.val)
    xt = inputs.x_true(A.n)
    return w, A, solver.csr(rp, col, val), solver.spmv(solver.csr(rp, col, val), dev_t(xt)), oracle.spmv(A, xt)


@pytest.mark.parametrize("variant,algo", [("cg", oracle.ALG_CG), ("cgcg", oracle.ALG_CGCG),
                                          ("pipe_cg", oracle.ALG_PIPE_CG)])
def test_c2s_cg_family_full_solve_bitwise(c2s, variant, algo):
    """The CG family on the 128^3 Poisson operator with Jacobi, as the benchmark runs it."""
    w, A, op, b, b_or = c2s
    assert same(host(b), b_or)
    t0 = time.time()
    x_or, i_or = oracle.solve(A, b_or, algo=algo, dinv=oracle.jacobi_dinv(A), tol=w.tol, maxit=w.maxit,
                              history=True)
    say(f"c2s {variant}: oracle {i_or['iters']} it in {time.time() - t0:.1f}s")
    x, info = solver.solve(op, b, variant=variant, precond="jacobi", tol=w.tol, maxit=w.maxit, history=True)
    assert (info.status, info.iters) == (i_or["status"], i_or["iters"]) and info.status == 0
    assert same(host(x), x_or)
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])
    assert same(host(info.history), i_or["history"])


def test_c2_stencil_equals_csr(c2):
    w, A, (rp, col, val), op, b, _ = c2
    mid = w.n // 2
    row = mid + w.n * mid + w.n * w.n * mid
    coef = list(A.val[A.row_ptr[row]:A.row_ptr[row + 1]])
    st = solver.stencil(w.n, w.n, w.n, coef)
    for precond in ("jacobi", "jacobi_folded"):
        x1, i1 = solver.solve(op, b, variant="pbicgstab_rr", precond=precond, tol=w.tol, rr_period=w.rr_period)
        x2, i2 = solver.solve(st, b, variant="pbicgstab_rr", precond=precond, tol=w.tol, rr_period=w.rr_period)
        assert i1.iters == i2.iters and same(host(x1), host(x2))


@pytest.fixture(scope="module")
def c3():
    require_gpu()
    w = inputs.workload("c3")
    kappa = inputs.kappa_cells(w.n, w.kappa_sigma)
    t0 = time.time()
    rp, col, val = solver.assemble_convdiff(w.dim, w.n, w.npts, w.beta, dev_t(kappa), w.shift)
    torch.cuda.synchronize()
    say(f"c3 device assembly {time.time() - t0:.1f}s nnz={val.numel()}")
    op = solver.csr(rp, col, val)
    return w, kappa, (rp, col, val), op


def test_c3_sampled_rows_bitwise(c3):
    w, kappa, (rp, col, val), op = c3
    N = w.N
    assert val.numel() == oracle.assemble_nnz(3, w.n, 27) == 449455096
    rng = np.random.default_rng(7)
    starts = [0, N // 2 - 5000, N - 3000] + list(rng.integers(0, N - 2000, 5))
    rp_h = host(rp)
    for s0 in starts:
        s0 = int(s0)
        s1 = min(N, s0 + 2000)
        r_or, c_or, v_or = oracle.assemble_rows(3, w.n, 27, w.beta, s0, s1, kappa, w.shift)
        lo, hi = int(rp_h[s0]), int(rp_h[s1])
        assert np.array_equal(rp_h[s0:s1 + 1] - lo, r_or)
        assert np.array_equal(host(col[lo:hi]), c_or)
        assert same(host(val[lo:hi]), v_or)


def test_c3_first_iterations_bitwise_and_full_solve(c3):
    w, kappa, (rp, col, val), op = c3
    xt_h = inputs.x_true(w.N)
    xt = dev_t(xt_h)
    b = solver.spmv(op, xt)
    t0 = time.time()
    A = oracle.assemble_workload(w, kappa)
    say(f"c3 oracle assembly {time.time() - t0:.1f}s")
    # the whole device matrix, bit for bit
    assert np.array_equal(host(rp), A.row_ptr)
    assert np.array_equal(host(col), A.col)
    assert same(host(val), A.val)
    t0 = time.time()
    b_or = oracle.spmv(A, xt_h)
    assert same(host(b), b_or)
    dinv = oracle.jacobi_dinv(A)
    x_or, i_or = oracle.solve(A, b_or, algo=oracle.ALG_PBICGSTAB_RR, dinv=dinv, tol=0.0, maxit=4, rr_period=2)
    say(f"c3 oracle 4 iterations {time.time() - t0:.1f}s")
    x, info = solver.solve(op, b, variant="pbicgstab_rr", precond="jacobi", tol=0.0, maxit=4, rr_period=2)
    assert (info.iters, info.n_rr) == (i_or["iters"], i_or["n_rr"]) == (4, 2)
    assert same(host(x), x_or)
    # complete solve at the configuration's tolerance and replacement period
    x, info = solver.solve(op, b, variant="pbicgstab_rr", precond="jacobi", tol=w.tol, maxit=w.maxit,
                           rr_period=w.rr_period)
    say(f"c3 full solve: {info.iters} it, {info.n_rr} RR, relres_true {info.relres_true:.2e}, {info.ms:.0f} ms")
    t0 = time.time()
    x_or, i_or = oracle.solve(A, b_or, algo=oracle.ALG_PBICGSTAB_RR, dinv=dinv, tol=w.tol, maxit=w.maxit,
                              rr_period=w.rr_period)
    say(f"c3 oracle full solve {time.time() - t0:.1f}s")
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
    assert same(host(x), x_or)
    del A
    # and properties that hold at any size
    assert info.status == 0
    assert info.relres_rec <= w.tol
    assert info.relres_true <= 1.5 * w.tol
    assert info.n_rr == info.iters // w.rr_period
    err = torch.linalg.norm(x - xt).item() / torch.linalg.norm(xt).item()
    assert err < 1e-5


def test_c4_precision_form_bitwise():
    require_gpu()
    w = inputs.workload("c4")
    t0 = time.time()
    A = oracle.assemble_workload(w)
    rp, col, val = solver.assemble_convdiff(w.dim, w.n, w.npts, w.beta)
    assert np.array_equal(host(rp), A.row_ptr) and np.array_equal(host(col), A.col) and same(host(val), A.val)
    op = solver.csr(rp, col, val)
    xt = inputs.x_true(A.n)
    b_or = oracle.spmv(A, xt)
    b = solver.spmv(op, dev_t(xt))
    assert same(host(b), b_or)
    dinv = oracle.jacobi_dinv(A)
    say(f"c4 assembled {time.time() - t0:.1f}s")
    t0 = time.time()
    x_or, i_or = oracle.solve_mp(A, b_or, dinv=dinv, tol=w.tol, maxit=w.maxit, rr_period=w.rr_period)
    say(f"c4 oracle binary32 form: {i_or['iters']} it, {i_or['n_rr']} RR, {time.time() - t0:.1f}s")
    x, info = solver.solve(op, b, variant="pbicgstab_rr", precond="jacobi_folded", precision="fp32_rr64",
                           tol=w.tol, maxit=w.maxit, rr_period=w.rr_period)
    assert (info.status, info.iters, info.n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"])
    assert same(host(x), x_or)
    assert same([info.relres_rec, info.relres_true], [i_or["relres_rec"], i_or["relres_true"]])
    assert info.status == 0 and info.relres_true <= w.tol
    t0 = time.time()
    x64_or, i64 = oracle.solve_folded(A, b_or, algo=oracle.ALG_PBICGSTAB_RR, dinv=dinv, tol=w.tol, maxit=w.maxit,
                                      rr_period=50)
    say(f"c4 oracle binary64: {i64['iters']} it, {time.time() - t0:.1f}s")
    x64, info64 = solver.solve(op, b, variant="pbicgstab_rr", precond="jacobi_folded", tol=w.tol, maxit=w.maxit,
                               rr_period=50)
    assert (info64.status, info64.iters) == (i64["status"], i64["iters"]) and same(host(x64), x64_or)
    err = np.linalg.norm(x_or - x64_or) / np.linalg.norm(x64_or)
    say(f"c4 binary32 form vs binary64 solution: {err:.2e}")
    assert err < 1e-6


def test_c5_batched_full_workload():
    require_gpu()
    systems = inputs.batch_systems()
    ops, bs, Ns = [], [], []
    for sy in systems:
        rp, col, val = solver.assemble_convdiff(2, sy.n, 5, sy.beta)
        A = solver.csr(rp, col, val)
        ops.append(A)
        bs.append(solver.spmv(A, dev_t(inputs.batch_x_true(sy.k, sy.n * sy.n))))
        Ns.append(sy.n * sy.n)
    assert sum(Ns) == 22324961
    kw = dict(variant="pbicgstab_rr", tol=1e-8, maxit=20000, rr_period=50)
    t0 = time.time()
    xs, infos = solver.solve_batched(ops, bs, **kw)
    torch.cuda.synchronize()
    say(f"c5 batched: {time.time() - t0:.2f}s, iterations {min(i.iters for i in infos)}..{max(i.iters for i in infos)}")
    assert all(i.status == 0 for i in infos)
    assert all(i.relres_rec <= 1e-8 and i.relres_true <= 2e-8 for i in infos)
    order = np.argsort(Ns)
    sample = [int(order[0]), int(order[-1])] + [int(k) for k in np.random.default_rng(3).choice(len(systems), 6, replace=False)]
    for k in sample:
        sy = systems[k]
        A = oracle.assemble(2, sy.n, 5, sy.beta)
        b = oracle.spmv(A, inputs.batch_x_true(sy.k, A.n))
        assert same(host(bs[k]), b)
        x_or, i_or = oracle.solve(A, b, algo=oracle.ALG_PBICGSTAB_RR, tol=1e-8, maxit=20000, rr_period=50)
        assert (infos[k].status, infos[k].iters, infos[k].n_rr) == (i_or["status"], i_or["iters"], i_or["n_rr"]), k
        assert same(host(xs[k]), x_or), k
        say(f"c5 system {k} (n={sy.n}): {i_or['iters']} iterations, bitwise")
    ws = [dev_t(inputs.batch_loss_weights(sy.k, sy.n * sy.n)) for sy in systems]
    lams, ainfos, _ = solver.solve_adjoint_batched(ops, ws, **kw)
    assert all(i.status == 0 for i in ainfos)
    for k in sample[:3]:
        sy = systems[k]
        A = oracle.assemble(2, sy.n, 5, sy.beta)
        lam_or, li = oracle.solve(oracle.transpose(A), inputs.batch_loss_weights(sy.k, A.n),
                                  algo=oracle.ALG_PBICGSTAB_RR, tol=1e-8, maxit=20000, rr_period=50)
        assert ainfos[k].iters == li["iters"] and same(host(lams[k]), lam_or), k
