"""Pins of the oracle's building blocks: SpMV, the pairwise dot product, Jacobi."""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1612_01395_amd import inputs


def test_spmv_brute_force_integer_matrix():
    """Integer entries and vector: every sum is exact, so the SpMV is the dense product."""
    rng = np.random.default_rng(5)
    n = 37
    D = rng.integers(-9, 10, (n, n)) * (rng.random((n, n)) < 0.2)
    S = sp.csr_matrix(D.astype(np.float64))
    S.sort_indices()
    A = oracle.CSR(S.indptr, S.indices, S.data)
    x = rng.integers(-50, 50, n).astype(np.float64)
    np.testing.assert_array_equal(oracle.spmv(A, x), D @ x.astype(np.int64))


def test_spmv_matches_row_order_sum():
    A = oracle.assemble_workload(inputs.workload("c1"))
    x = inputs.x_true(A.n)
    y = oracle.spmv(A, x)
    # independent: per-row left-to-right sum of rounded products in stored order
    for row in (0, 1, 63, 64, 2000, A.n - 1):
        acc = 0.0
        for k in range(A.row_ptr[row], A.row_ptr[row + 1]):
            acc = acc + A.val[k] * x[A.col[k]]
        assert y[row] == acc
    np.testing.assert_allclose(y, A.to_scipy() @ x, rtol=1e-15, atol=1e-15)


def _tree_bottom_up(a):
    """Pairwise sum by levels: pad to a power of two, then add adjacent pairs."""
    n = 1
    while n < len(a):
        n *= 2
    v = np.zeros(n)
    v[: len(a)] = a
    while len(v) > 1:
        v = v[0::2] + v[1::2]
    return float(v[0]) + 0.0


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 100, 4096, 65536, 65537, 300001])
def test_pairwise_sum_is_the_balanced_tree(n):
    a = np.random.default_rng(n).standard_normal(n) * np.exp(np.random.default_rng(n + 1).uniform(-20, 20, n))
    assert oracle.pairwise_sum(a) == _tree_bottom_up(a)


def test_pairwise_hand_worked_examples(golden_dir):
    with open(os.path.join(golden_dir, "pairwise_example.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        terms = np.array(case["terms"])
        assert oracle.pairwise_sum(terms) == case["pairwise"]
        ltr = 0.0
        for t in terms:
            ltr = ltr + t
        assert ltr == case["left_to_right"]
        # the dot with a ones vector is the same sum (products are exact)
        assert oracle.dot(terms, np.ones_like(terms)) == case["pairwise"]


def test_dot_error_bound_against_exact():
    """|pairwise - exact| <= gamma_{ceil(log2 n)+1} sum |x_i y_i| (products rounded once)."""
    rng = np.random.default_rng(11)
    for n in (10, 1000, 77777):
        x = rng.standard_normal(n)
        y = rng.standard_normal(n) * np.exp(rng.uniform(-5, 5, n))
        d = oracle.dot(x, y)
        exact = math.fsum(float(Fraction(a) * Fraction(b)) for a, b in zip(x[:2000], y[:2000])) \
            if n <= 2000 else None
        prods = x * y
        ref = math.fsum(prods)  # correctly rounded sum of the rounded products
        u = 2.0 ** -53
        k = math.ceil(math.log2(n)) + 1
        bound = (k * u / (1 - k * u)) * np.abs(prods).sum()
        assert abs(d - ref) <= bound
        if exact is not None:
            assert abs(d - exact) <= bound


def test_dot_exact_for_integers_and_zero_sign():
    rng = np.random.default_rng(2)
    x = rng.integers(-1000, 1000, 12345).astype(np.float64)
    y = rng.integers(-1000, 1000, 12345).astype(np.float64)
    assert oracle.dot(x, y) == float(int(np.dot(x.astype(np.int64), y.astype(np.int64))))
    z = oracle.dot(np.array([-0.0, -0.0]), np.array([1.0, 1.0]))
    assert z == 0.0 and math.copysign(1.0, z) == 1.0  # a zero sum is +0


def test_jacobi_dinv():
    A = oracle.assemble_workload(inputs.workload("c2", n=6))
    d = oracle.jacobi_dinv(A)
    np.testing.assert_array_equal(d, 1.0 / A.to_scipy().diagonal())
    bad = oracle.CSR([0, 1, 2], [1, 0], [1.0, 1.0])  # no diagonal
    with pytest.raises(ValueError):
        oracle.jacobi_dinv(bad)
