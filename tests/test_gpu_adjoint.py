"""GPU parity and checks of the adjoint path: the device transpose and the
entry gradient bit for bit against the oracle, the adjoint solve through
the autograd Function, and the batched workload's dL/dbeta against central
finite differences of direct solves (step 1e-6 relative to beta, b frozen at
the nominal beta; an absolute step of 1e-6 on beta ~ 100 would leave the
differences dominated by the direct solves' rounding, u kappa |L| / step)."""

import numpy as np
import pytest
import scipy.sparse.linalg as spl
import torch

import oracle
from paper_1612_01395_amd import inputs, solver
from gpu_util import csr_op, dev_t, host, require_gpu, same, say

pytestmark = pytest.mark.gpu


def _mats():
    rng = np.random.default_rng(17)
    import scipy.sparse as sp
    D = rng.standard_normal((300, 300)) * (rng.random((300, 300)) < 0.03) + 4 * np.eye(300)
    D[7, :] = 0.0
    D[7, 7] = 1.0
    D[:, 11] = 0.0
    D[11, 11] = 2.0
    R = sp.csr_matrix(D)
    R.sort_indices()
    return {"c1": oracle.assemble_workload(inputs.workload("c1")),
            "c2_24": oracle.assemble_workload(inputs.workload("c2", n=24)),
            "c3_10": oracle.assemble_workload(inputs.workload("c3", n=10), inputs.kappa_cells(10)),
            "random": oracle.CSR(R.indptr, R.indices, R.data)}


MATS = _mats()


def _arrowhead(n, extra_long=()):
    """Dense first row and first column plus the diagonal (column 0 of A, so
    row 0 of A^T, holds n entries), and further columns with the given numbers
    of entries at random rows; values random of both signs."""
    import scipy.sparse as sp
    rng = np.random.default_rng(n)
    rows = [np.zeros(n, np.int64), np.arange(n), np.arange(n)]
    cols = [np.arange(n), np.zeros(n, np.int64), np.arange(n)]
    for c, m in extra_long:
        rows.append(rng.choice(n, size=m, replace=False))
        cols.append(np.full(m, c))
    r, c = np.concatenate(rows), np.concatenate(cols)
    v = rng.standard_normal(len(r))
    M = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()  # duplicates summed
    M.sort_indices()
    M = M + sp.diags(np.full(n, 50.0))
    M = M.tocsr()
    M.sort_indices()
    return oracle.CSR(M.indptr, M.indices, M.data)


@pytest.mark.parametrize("n,extra", [(20000, ()), (3000, ((5, 65), (6, 64), (7, 1000), (8, 2049), (9, 2999))),
                                     (70, ((3, 65),))])
def test_transpose_long_columns_bitwise(n, extra):
    """Columns longer than one thread's share are ordered by a workgroup each;
    the product with A^T sums every row in ascending column order like the
    oracle's transpose."""
    require_gpu()
    A = _arrowhead(n, extra)
    say(f"transpose arrowhead n={n} longest column {int(np.bincount(A.col).max())}")
    T_or = oracle.transpose(A)
    T = solver.transpose(csr_op(A))
    for seed in (3, 4):
        x = inputs.random_vector(A.n, seed)
        assert same(host(solver.spmv(T, dev_t(x))), oracle.spmv(T_or, x))


@pytest.mark.parametrize("name", list(MATS))
def test_transpose_bitwise(name):
    require_gpu()
    A = MATS[name]
    say(f"transpose {name}")
    T_or = oracle.transpose(A)
    op = csr_op(A)
    T = solver.transpose(op)
    # read the transposed arrays back through products with unit vectors is slow;
    # compare y = A^T x bitwise instead, and the solve on A^T below
    x = inputs.random_vector(A.n, 3)
    assert same(host(solver.spmv(T, dev_t(x))), oracle.spmv(T_or, x))


@pytest.mark.parametrize("variant", ["pbicgstab_rr", "bicgstab"])
@pytest.mark.parametrize("name", ["c1", "c3_10"])
def test_adjoint_solve_and_gradient_bitwise(name, variant):
    require_gpu()
    A = MATS[name]
    alg = oracle.ALG_PBICGSTAB_RR if variant == "pbicgstab_rr" else oracle.ALG_BICGSTAB
    b = oracle.spmv(A, inputs.x_true(A.n))
    g = inputs.random_vector(A.n, 12)
    kw = dict(tol=1e-11, maxit=3000, rr_period=25)
    x_or, _ = oracle.solve(A, b, algo=alg, **kw)
    lam_or, li = oracle.solve(oracle.transpose(A), g, algo=alg, **kw)
    gv_or = oracle.outer_grad(A, lam_or, x_or)
    rp, col, vals = dev_t(A.row_ptr), dev_t(A.col), dev_t(A.val).requires_grad_(True)
    bt = dev_t(b).requires_grad_(True)
    x = solver.SolveFn.apply(vals, bt, rp, col, dict(variant=variant, **kw))
    assert same(host(x.detach()), x_or)
    loss = (x * dev_t(g)).sum()
    loss.backward()
    assert same(host(bt.grad), lam_or)
    assert same(host(vals.grad), gv_or)


def test_dense_reference_gradient():
    require_gpu()
    A = oracle.assemble_workload(inputs.workload("c1", n=10))
    D = A.to_scipy().toarray()
    b = oracle.spmv(A, inputs.x_true(A.n))
    w = inputs.random_vector(A.n, 5)
    vals = dev_t(A.val).requires_grad_(True)
    x = solver.SolveFn.apply(vals, dev_t(b), dev_t(A.row_ptr), dev_t(A.col), dict(tol=1e-13, maxit=2000, rr_period=10))
    (x * dev_t(w)).sum().backward()
    lam = np.linalg.solve(D.T, w)
    xr = np.linalg.solve(D, b)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    ref = -(lam[rows] * xr[A.col])
    assert np.linalg.norm(host(vals.grad) - ref) <= 1e-9 * np.linalg.norm(ref)


def test_batched_loss_gradient_against_finite_differences():
    """L = sum_k (w_k, x_k) over the first 8 systems of the batched workload;
    dL/dbeta_k from one batched forward and one batched adjoint solve, against
    central differences of SuperLU solves with b_k frozen at the nominal beta."""
    require_gpu()
    systems = inputs.batch_systems()[:8]
    ops, bs, ws, Ahost = [], [], [], []
    for s in systems:
        A = oracle.assemble(2, s.n, 5, s.beta)
        Ahost.append(A)
        ops.append(csr_op(A))
        bs.append(oracle.spmv(A, inputs.batch_x_true(s.k, A.n)))
        ws.append(inputs.batch_loss_weights(s.k, A.n))
    kw = dict(variant="pbicgstab_rr", tol=1e-12, maxit=20000, rr_period=50)
    xs, infos = solver.solve_batched(ops, [dev_t(b) for b in bs], **kw)
    assert all(i.status == 0 for i in infos)
    lams, ainfos, _ = solver.solve_adjoint_batched(ops, [dev_t(w) for w in ws], **kw)
    assert all(i.status == 0 for i in ainfos)
    eps = 1e-6
    worst = 0.0
    for k, s in enumerate(systems):
        gv = host(solver.csr_outer_grad(ops[k], lams[k], xs[k]))
        for a in range(2):
            e = np.zeros(2)
            e[a] = 1.0
            # d vals / d beta_a: the operator is affine in beta_a (> 1 here), so a unit central difference is exact
            dv = (oracle.assemble(2, s.n, 5, tuple(np.array(s.beta) + e)).val
                  - oracle.assemble(2, s.n, 5, tuple(np.array(s.beta) - e)).val) / 2.0
            grad = float(gv @ dv)

            def L(beta):
                Ab = oracle.assemble(2, s.n, 5, tuple(beta)).to_scipy().tocsc()
                return float(ws[k] @ spl.splu(Ab).solve(bs[k]))

            h = eps * abs(s.beta[a])  # the step is relative to beta_a (about 1e-4 here)
            fd = (L(np.array(s.beta) + h * e) - L(np.array(s.beta) - h * e)) / (2 * h)
            rel = abs(grad - fd) / abs(fd)
            say(f"system {k} (n={s.n}) beta_{a}: adjoint {grad:.10e} fd {fd:.10e} rel {rel:.2e}")
            worst = max(worst, rel)
    assert worst <= 1e-5


def test_unconverged_solves_raise():
    """A forward or adjoint solve that stops at its iteration budget raises
    instead of feeding an unconverged x or lambda into the gradient."""
    require_gpu()
    A = oracle.assemble_workload(inputs.workload("c1", n=12))
    b = oracle.spmv(A, inputs.x_true(A.n))
    rp, col = dev_t(A.row_ptr), dev_t(A.col)
    vals = dev_t(A.val).requires_grad_(True)
    with pytest.raises(solver.NotConvergedError) as e:
        solver.SolveFn.apply(vals, dev_t(b), rp, col, dict(tol=1e-12, maxit=1))
    assert e.value.info.status == 1 and e.value.info.iters == 1
    x = solver.SolveFn.apply(vals, dev_t(b), rp, col, dict(tol=1e-12, maxit=2000, adjoint_maxit=1))
    with pytest.raises(solver.NotConvergedError) as e:
        (x * dev_t(inputs.random_vector(A.n, 3))).sum().backward()
    assert "adjoint" in str(e.value)
    vals.grad = None
    x = solver.SolveFn.apply(vals, dev_t(b), rp, col, dict(tol=1e-12, maxit=2000, adjoint_maxit=1,
                                                            allow_unconverged=True))
    (x * dev_t(inputs.random_vector(A.n, 3))).sum().backward()
    assert vals.grad is not None
