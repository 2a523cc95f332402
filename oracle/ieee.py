"""IEEE 754 rounding of exact rationals -- TEST INFRASTRUCTURE ONLY.

Rounding to nearest, ties to even, into the binary32 and binary64 formats,
written from the standard's definition of a binary format (precision p
significand bits, exponent range [emin, emax], subnormals at the fixed
quantum 2^(emin - p + 1)).  Every arithmetic operation of an IEEE machine is
"compute exactly, then round once", so applying :func:`round32` or
:func:`round64` to the exact ``fractions.Fraction`` result of each +, -, *, /
reproduces the machine's result bit for bit; :func:`sqrt64` does the same for
the correctly rounded square root.  Signed zeros are not represented (both
zeros are Fraction(0)); no operation of the solvers that use this module
depends on the sign of a zero.
"""

from __future__ import annotations

from fractions import Fraction
from math import isqrt

__all__ = ["BINARY32", "BINARY64", "round_to", "round32", "round64", "sqrt64", "exponent"]

# (precision p including the hidden bit, emin, emax)
BINARY32 = (24, -126, 127)
BINARY64 = (53, -1022, 1023)


def exponent(a: Fraction) -> int:
    """floor(log2(a)) of a positive rational a."""
    e = a.numerator.bit_length() - a.denominator.bit_length()
    # 2^e <= a < 2^(e+1) after at most one correction either way
    lo = Fraction(1 << e) if e >= 0 else Fraction(1, 1 << -e)
    if a < lo:
        e -= 1
    elif a >= 2 * lo:
        e += 1
    return e


def round_to(q, fmt) -> Fraction:
    """The value of the format nearest to the rational q (ties to the even
    significand).  Raises OverflowError when the result would be infinite."""
    q = Fraction(q)
    if q == 0:
        return Fraction(0)
    p, emin, emax = fmt
    neg = q < 0
    a = -q if neg else q
    e = max(exponent(a), emin)  # below the normal range the quantum stays fixed
    sh = e - p + 1              # quantum = 2^sh
    m = a / (1 << sh) if sh >= 0 else a * (1 << -sh)
    lo = m.numerator // m.denominator
    rem = m - lo
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and (lo & 1)):
        lo += 1
    r = lo * (Fraction(1 << sh) if sh >= 0 else Fraction(1, 1 << -sh))
    largest = (2 - Fraction(1, 1 << (p - 1))) * (1 << emax)
    if r > largest:
        raise OverflowError("result overflows the format")
    return -r if neg else r


def round32(q) -> Fraction:
    return round_to(q, BINARY32)


def round64(q) -> Fraction:
    return round_to(q, BINARY64)


def sqrt64(q) -> Fraction:
    """Correctly rounded binary64 square root of a non-negative rational."""
    q = Fraction(q)
    if q < 0:
        raise ValueError("sqrt of a negative number")
    if q == 0:
        return Fraction(0)
    p = BINARY64[0]
    # scale so that s = floor(sqrt(q) 2^k) has at least p + 2 bits
    k = p + 3 - exponent(q) // 2
    scaled = q * (1 << (2 * k)) if k >= 0 else q / (1 << (-2 * k))
    s = isqrt(scaled.numerator // scaled.denominator)
    exact = Fraction(s * s) == scaled
    unit = Fraction(1, 1 << k) if k >= 0 else Fraction(1 << -k)  # 2^-k
    # the root lies in [s, s + 1) units; when it is not exact it lies strictly
    # inside, and no rounding boundary of the target (a multiple of 2 units)
    # falls there, so s + 1/2 rounds the same way as the root itself
    val = Fraction(s) if exact else Fraction(2 * s + 1, 2)
    return round64(val * unit)
