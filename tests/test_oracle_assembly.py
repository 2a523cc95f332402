"""Pins of the oracle's operator assembly (the workloads' matrices).

The assembly rule is the workload definition: h^2-scaled first-order upwind
convection-diffusion on the interior nodes, Dirichlet boundaries dropped, rows
x fastest.  These tests check the oracle's C assembler against independent
constructions: a Kronecker-sum build of the 5/7-point operators, a vectorised
numpy build of the 27-point operator, closed forms and structural invariants.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1612_01395_amd import inputs


def _tri(n, hb, beta_sign_nonneg):
    """1-D h^2-scaled upwind operator: -u'' + b u' -> [-1-|hb|, 2+|hb|, -1] (b >= 0)."""
    up = -1.0 - abs(hb)
    lower = np.full(n - 1, up if beta_sign_nonneg else -1.0)
    upper = np.full(n - 1, -1.0 if beta_sign_nonneg else up)
    diag = np.full(n, 2.0 + abs(hb))
    return sp.diags([lower, diag, upper], [-1, 0, 1], format="csr")


def kron_operator(dim, n, beta):
    hb = [b / (n + 1) for b in beta]
    I = sp.identity(n, format="csr")
    T = [_tri(n, hb[a], beta[a] >= 0) for a in range(dim)]
    if dim == 2:
        A = sp.kron(I, T[0]) + sp.kron(T[1], I)
    else:
        A = (sp.kron(sp.kron(I, I), T[0]) + sp.kron(sp.kron(I, T[1]), I)
             + sp.kron(sp.kron(T[2], I), I))
    A = A.tocsr()
    A.sort_indices()
    return A


@pytest.mark.parametrize("dim,n,beta", [
    (2, 1, (20.0, 10.0)), (2, 7, (20.0, 10.0)), (2, 16, (-3.0, 7.5)), (2, 64, (20.0, 10.0)),
    (3, 1, (1.0, 2.0, 3.0)), (3, 6, (50.0, 30.0, 10.0)), (3, 9, (-50.0, 0.0, 13.0)),
])
def test_5_7_point_matches_kronecker_sum(dim, n, beta):
    npts = 5 if dim == 2 else 7
    A = oracle.assemble(dim, n, npts, beta)
    K = kron_operator(dim, n, beta)
    assert A.nnz == K.nnz == oracle.assemble_nnz(dim, n, npts)
    np.testing.assert_array_equal(A.row_ptr, K.indptr)
    np.testing.assert_array_equal(A.col, K.indices)
    # the Kronecker sum adds the diagonal in another order: equal to rounding
    np.testing.assert_allclose(A.val, K.data, rtol=4e-16, atol=0)
    off = A.col != np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    np.testing.assert_array_equal(A.val[off], K.data[off])


@pytest.mark.parametrize("dim,npts,formula", [
    (2, 5, lambda n: 5 * n * n - 4 * n),
    (3, 7, lambda n: 7 * n ** 3 - 6 * n * n),
    (3, 27, lambda n: (3 * n - 2) ** 3),
])
def test_nnz_closed_forms(dim, npts, formula):
    for n in (1, 2, 3, 5, 8):
        kappa = np.ones((n + 1) ** 3) if npts == 27 else None
        A = oracle.assemble(dim, n, npts, (1.0,) * dim, kappa)
        assert A.nnz == formula(n)
        # and every row has the count of in-grid neighbours + 1
        if npts == 27:
            idx = np.arange(n)
            per_axis = 3 - (idx == 0) - (idx == n - 1)
            expect = np.einsum("k,j,i->kji", per_axis, per_axis, per_axis).ravel()
            np.testing.assert_array_equal(np.diff(A.row_ptr), expect)


def test_c1_entries_closed_form():
    """C1: 64 x 64, beta = (20, 10): hb = beta/65, interior row [-1-hby, -1-hbx, d, -1, -1]."""
    A = oracle.assemble(2, 64, 5, (20.0, 10.0))
    hbx, hby = 20.0 / 65.0, 10.0 / 65.0
    row = 64 * 10 + 10
    lo, hi = A.row_ptr[row], A.row_ptr[row + 1]
    np.testing.assert_array_equal(A.col[lo:hi], [row - 64, row - 1, row, row + 1, row + 64])
    np.testing.assert_array_equal(A.val[lo:hi], [-1.0 - hby, -1.0 - hbx, (4.0 + hbx) + hby, -1.0, -1.0])
    # interior row sums vanish (the operator annihilates constants away from the boundary)
    S = A.to_scipy()
    ones = np.ones(A.n)
    rs = (S @ ones).reshape(64, 64)
    assert np.abs(rs[1:-1, 1:-1]).max() < 1e-14


def numpy_27pt(n, beta, kappa, shift):
    """Independent vectorised 27-point build (dense per-offset arrays)."""
    cn = n + 1
    K = kappa.reshape(cn, cn, cn)  # [ck, cj, ci]
    hb = [b / (n + 1) for b in beta]
    N = n ** 3
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    entries = {}
    diag_sum = np.zeros((n, n, n))
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if dx == dy == dz == 0:
                    continue
                rng = lambda d: [0] if d < 0 else ([1] if d > 0 else [0, 1])
                ks = np.zeros((n, n, n))
                cnt = 0
                for c in rng(dz):
                    for b in rng(dy):
                        for a in rng(dx):
                            ks = ks + K[c:c + n, b:b + n, a:a + n]
                            cnt += 1
                kbar = ks * (1.0 / cnt)
                diag_sum = diag_sum + kbar
                v = -kbar
                if abs(dx) + abs(dy) + abs(dz) == 1:
                    ax = 0 if dx else (1 if dy else 2)
                    side = dx or dy or dz
                    upwind = (side < 0) if beta[ax] >= 0 else (side > 0)
                    if upwind:
                        v = -kbar - abs(hb[ax])
                entries[(dz, dy, dx)] = v
    diag = (diag_sum + ((abs(hb[0]) + abs(hb[1])) + abs(hb[2]))) + shift
    entries[(0, 0, 0)] = diag
    rows, cols, vals = [], [], []
    for (dz, dy, dx), v in entries.items():
        ok = ((ii + dx >= 0) & (ii + dx < n) & (jj + dy >= 0) & (jj + dy < n)
              & (kk + dz >= 0) & (kk + dz < n))
        r = (ii + n * jj + n * n * kk)[ok]
        c = ((ii + dx) + n * (jj + dy) + n * n * (kk + dz))[ok]
        rows.append(r)
        cols.append(c)
        vals.append(v[ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    order = np.lexsort((cols, rows))
    rp = np.zeros(N + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols[order], vals[order]


@pytest.mark.parametrize("n,beta", [(3, (100.0, 0.0, 50.0)), (6, (100.0, 0.0, 50.0)),
                                    (5, (-7.0, 3.0, -2.0))])
def test_27_point_matches_vectorised_build(n, beta):
    kappa = inputs.kappa_cells(n, 1.0)
    A = oracle.assemble(3, n, 27, beta, kappa, 0.1)
    rp, col, val = numpy_27pt(n, beta, kappa, 0.1)
    np.testing.assert_array_equal(A.row_ptr, rp)
    np.testing.assert_array_equal(A.col, col)
    np.testing.assert_array_equal(A.val, val)  # same evaluation order: bit-exact


def test_27_point_constant_kappa_closed_form():
    """kappa = 1: every diffusion coupling is -1 and the diagonal is 26 + sum|hb| + shift."""
    n = 4
    beta = (100.0, 0.0, 50.0)
    A = oracle.assemble(3, n, 27, beta, np.ones((n + 1) ** 3), 0.1)
    S = A.to_scipy().toarray()
    hb = [b / (n + 1) for b in beta]
    diag_expect = (26.0 + ((abs(hb[0]) + abs(hb[1])) + abs(hb[2]))) + 0.1
    np.testing.assert_array_equal(np.diag(S), np.full(n ** 3, diag_expect))
    p = 1 + n * 1 + n * n * 1  # interior node (1,1,1)
    assert S[p, p - 1] == -1.0 - hb[0]      # upwind x face (beta_x > 0)
    assert S[p, p + 1] == -1.0
    assert S[p, p - n] == -1.0               # beta_y = 0: no upwind term
    assert S[p, p - n * n] == -1.0 - hb[2]
    assert S[p, p + n * n + n + 1] == -1.0   # corner


def test_27_point_diffusion_part_symmetric_and_dominant():
    n = 6
    kappa = inputs.kappa_cells(n, 1.0)
    A0 = oracle.assemble(3, n, 27, (0.0, 0.0, 0.0), kappa, 0.1).to_scipy()
    D = (A0 - A0.T)
    assert abs(D).max() == 0.0  # bitwise symmetric without convection
    A = oracle.assemble(3, n, 27, (100.0, 0.0, 50.0), kappa, 0.1).to_scipy().toarray()
    off = A - np.diag(np.diag(A))
    assert (off <= 0).all()
    assert (np.diag(A) > np.abs(off).sum(axis=1)).all()  # strictly diagonally dominant
    # interior rows sum to the shift: diffusion and upwind terms cancel
    rs = A.sum(axis=1).reshape(n, n, n)[1:-1, 1:-1, 1:-1]
    np.testing.assert_allclose(rs, 0.1, rtol=0, atol=1e-12)


def test_ptp_stencils_via_beta_free_operator():
    """The paper's PTP2 stencil [-1; -1 1 -1; -1] is the 5-point Laplacian minus 3 I."""
    n = 10
    L = oracle.assemble(2, n, 5, (0.0, 0.0))
    S = L.to_scipy().toarray()
    assert (np.diag(S) == 4.0).all()
    assert sorted(set(S[np.nonzero(S - np.diag(np.diag(S)))])) == [-1.0]


def test_row_range_assembly_is_a_slice_of_the_whole():
    n = 9
    kappa = inputs.kappa_cells(n, 1.0)
    A = oracle.assemble(3, n, 27, (100.0, 0.0, 50.0), kappa, 0.1)
    for r0, r1 in ((0, 1), (100, 300), (700, n ** 3)):
        rp, col, val = oracle.assemble_rows(3, n, 27, (100.0, 0.0, 50.0), r0, r1, kappa, 0.1)
        lo, hi = A.row_ptr[r0], A.row_ptr[r1]
        np.testing.assert_array_equal(rp, A.row_ptr[r0:r1 + 1] - lo)
        np.testing.assert_array_equal(col, A.col[lo:hi])
        np.testing.assert_array_equal(val, A.val[lo:hi])
