"""The precision form's rounding sequence, pinned by an exact twin.

``oracle/ieee.py`` rounds exact rationals to binary32 / binary64 from the
standard's definition; it is pinned here against the machine's own IEEE
arithmetic (CPython's correctly rounded int/int division, numpy's binary32
operations, libm's correctly rounded sqrt), including ties and subnormals.
``oracle.exact.pbicgstab_mp`` follows the precision form's reading
(binary32 vectors, operator, recurrences and pairwise dots; binary64 scalars
rounded to binary32 for the vector updates; binary64 x update and
replacement steps rounded once when stored; rho_0 from the binary32 dot;
binary64 confirmation of a recursive stop) with exact arithmetic and one
rounding per operation.  The C oracle must equal it bit for bit: x, the
residual history, iteration and replacement counts, status and the true
residual, on tiny systems with periodic and with forced replacements.  The
stored cases (``tests/golden/mp_rounding_cases.json``, written by
``make_mp_golden.py`` from the oracle alone) are also reproduced by the twin,
and each plausible misreading -- unrounded scalars in the binary32 updates,
w formed from the rounded r in a replacement, rho_0 from the binary64
residual -- gives different bits on them.
"""

import json
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact
from oracle.ieee import round32, round64, sqrt64
from paper_1612_01395_amd import inputs


# --------------------------------------------------------------------------
# IEEE rounding of rationals
# --------------------------------------------------------------------------

def test_round64_equals_correctly_rounded_division():
    rnd = random.Random(5)
    for _ in range(4000):
        num = rnd.getrandbits(rnd.randint(1, 160)) or 1
        den = rnd.getrandbits(rnd.randint(1, 160)) or 1
        q = Fraction(num, den) * Fraction(2) ** rnd.randint(-1100, 1000)
        q = -q if rnd.random() < 0.5 else q
        try:
            f = float(q)  # CPython divides the integers with one correct rounding
        except OverflowError:
            with pytest.raises(OverflowError):
                round64(q)
            continue
        assert round64(q) == Fraction(f)


def test_round64_ties_and_subnormals():
    two = Fraction(2)
    assert round64(two ** 53 + 1) == two ** 53                # tie, to even (down)
    assert round64(two ** 53 + 3) == two ** 53 + 4            # tie, to even (up)
    assert round64(two ** -1075) == 0                         # half the smallest subnormal: to even zero
    assert round64(3 * two ** -1075) == two ** -1073          # tie between subnormals 1 and 2 ulps: to 2
    assert round64(two ** -1074 * Fraction(5, 4)) == two ** -1074
    with pytest.raises(OverflowError):
        round64(two ** 1024)


def test_round32_equals_binary32_machine_arithmetic():
    rnd = random.Random(7)
    ops = (lambda a, b: a + b, lambda a, b: a - b, lambda a, b: a * b, lambda a, b: a / b)
    for _ in range(3000):
        a = np.float32(rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-140, 60))
        b = np.float32(rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-140, 60))
        if b == 0:
            continue
        for op in ops:
            with np.errstate(all="ignore"):
                c = op(a, b)
            if np.isfinite(c):
                assert round32(op(Fraction(float(a)), Fraction(float(b)))) == Fraction(float(c))
    two = Fraction(2)
    assert round32(two ** 24 + 1) == two ** 24 and round32(two ** 24 + 3) == two ** 24 + 4
    assert round32(two ** -150) == 0 and round32(3 * two ** -150) == two ** -148


def test_sqrt64_equals_libm():
    rnd = random.Random(9)
    for _ in range(4000):
        v = rnd.random() * 2.0 ** rnd.randint(-1070, 1020)
        if v > 0:
            assert sqrt64(Fraction(v)) == Fraction(math.sqrt(v))
    assert sqrt64(Fraction(49, 4)) == Fraction(7, 2)


# --------------------------------------------------------------------------
# The precision form: C oracle == exact twin
# --------------------------------------------------------------------------

def _rows(A):
    return [[(int(A.col[k]), Fraction(float(A.val[k]))) for k in range(A.row_ptr[i], A.row_ptr[i + 1])]
            for i in range(A.n)]


def _twin(A, b, **kw):
    x, info = exact.pbicgstab_mp(_rows(A), [Fraction(float(v)) for v in b], [Fraction(0)] * A.n, **kw)
    return np.array([float(v) for v in x]), info


STATUS = {"success": oracle.SUCCESS, "maxit": oracle.MAXIT, "breakdown": oracle.BREAKDOWN}


@pytest.mark.parametrize("name,n,kw,periodic,forced", [
    ("c1", 3, dict(tol=0.0, maxit=8, rr_period=3), 2, 0),
    ("c2", 2, dict(tol=0.0, maxit=8, rr_period=3), 2, 0),
    ("c2", 3, dict(tol=0.0, maxit=9, rr_period=3), 3, 0),
    ("c2", 3, dict(tol=1e-6, maxit=30, rr_period=0), 0, 1),
    ("c1", 5, dict(tol=3e-6, maxit=30, rr_period=0), 0, 1),
    ("c1", 5, dict(tol=3e-7, maxit=12, rr_period=4, rr_max=1), 1, 1),
])
def test_oracle_equals_exact_twin(name, n, kw, periodic, forced):
    A = oracle.assemble_workload(inputs.workload(name, n=n))
    b = oracle.spmv(A, inputs.x_true(A.n))
    x_or, i_or = oracle.solve_mp(A, b, history=True, **kw)
    x_ex, i_ex = _twin(A, b, **kw)
    assert i_or["iters"] >= 6
    assert i_or["iters"] == i_ex["iters"] and i_or["n_rr"] == i_ex["n_rr"] == periodic + forced
    assert i_or["status"] == STATUS[i_ex["status"]]
    assert np.array_equal(x_or, x_ex)
    assert np.array_equal(i_or["history"], np.array([float(v) for v in i_ex["history"]]))
    assert i_or["relres_true"] == float(i_ex["relres_true"])


def test_oracle_equals_exact_twin_random_sparse():
    """An unsymmetric random sparse system (diagonally dominant, values of
    both signs) from a non-zero x_0, with a periodic replacement."""
    rng = np.random.default_rng(31)
    n = 7
    D = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.45)
    D += np.diag(np.abs(D).sum(axis=1) + 1.5)
    import scipy.sparse as sp
    S = sp.csr_matrix(D)
    A = oracle.CSR(S.indptr, S.indices, S.data)
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    kw = dict(tol=0.0, maxit=7, rr_period=3)
    x_or, i_or = oracle.solve_mp(A, b, x0=x0, history=True, **kw)
    x_ex, i_ex = exact.pbicgstab_mp(_rows(A), [Fraction(float(v)) for v in b], [Fraction(float(v)) for v in x0],
                                    **kw)
    assert i_or["iters"] == i_ex["iters"] == 7 and i_or["n_rr"] == i_ex["n_rr"] == 2
    assert np.array_equal(x_or, np.array([float(v) for v in x_ex]))
    assert np.array_equal(i_or["history"], np.array([float(v) for v in i_ex["history"]]))


def _golden(golden_dir):
    with open(os.path.join(golden_dir, "mp_rounding_cases.json")) as f:
        g = json.load(f)
    s = g["system"]
    A = oracle.CSR(np.array(s["row_ptr"], np.int32), np.array(s["col"], np.int32),
                   np.array([float.fromhex(v) for v in s["val"]]))
    b = np.array([float.fromhex(v) for v in s["b"]])
    return A, b, g["cases"]


def _bits(info, x):
    return ([float(v) for v in x], [float(v) for v in info["history"]], info["iters"], info["n_rr"])


@pytest.mark.parametrize("case", ["periodic", "forced"])
def test_golden_cases_and_misreadings(golden_dir, case):
    A, b, cases = _golden(golden_dir)
    c = cases[case]
    want = ([float.fromhex(v) for v in c["x"]], [float.fromhex(v) for v in c["history"]], c["iters"], c["n_rr"])
    x_or, i_or = oracle.solve_mp(A, b, history=True, **c["opts"])
    assert _bits(i_or, x_or) == want
    assert i_or["relres_true"] == float.fromhex(c["relres_true"])
    x_ex, i_ex = _twin(A, b, **c["opts"])
    assert _bits(i_ex, x_ex) == want and i_ex["status"] == c["status"]
    for misreading in ("scalars64", "w_of_rounded_r", "rho0_64"):
        x_m, i_m = _twin(A, b, reading=(misreading,), **c["opts"])
        assert _bits(i_m, x_m) != want, misreading
