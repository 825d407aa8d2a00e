"""Exact (rational / big-integer) evaluation of radial Zernike polynomials from
the paper's closed forms, used to pin the oracle.

Nothing here shares code with the oracle or the GPU library.

* Eq. (radial-part-eq): R_n^m(r) = sum_s (-1)^s (n-s)! / (s! ((n+m)/2-s)! ((n-m)/2-s)!) r^(n-2s)
* Eq. (radial-part-eq-binom): the same coefficients as (-1)^s C(n-s, s) C(n-2s, (n-m)/2 - s),
  integers for every valid mode.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb, factorial


@lru_cache(maxsize=None)
def coefficients(n: int, m: int):
    """[(power, integer coefficient)] of R_n^{|m|} from Eq. (radial-part-eq)."""
    m = abs(m)
    out = []
    for s in range((n - m) // 2 + 1):
        num = (-1) ** s * factorial(n - s)
        den = factorial(s) * factorial((n + m) // 2 - s) * factorial((n - m) // 2 - s)
        assert num % den == 0
        out.append((n - 2 * s, num // den))
    return tuple(out)


@lru_cache(maxsize=None)
def coefficients_binom(n: int, m: int):
    """Same coefficients from Eq. (radial-part-eq-binom)."""
    m = abs(m)
    return tuple((n - 2 * s, (-1) ** s * comb(n - s, s) * comb(n - 2 * s, (n - m) // 2 - s))
                 for s in range((n - m) // 2 + 1))


def _falling(e: int, j: int) -> int:
    v = 1
    for t in range(j):
        v *= e - t
    return v


def radial_exact(n: int, m: int, r, j: int = 0) -> Fraction:
    """d^j/dr^j R_n^{|m|} at r (a float is taken at its exact binary value)."""
    r = Fraction(r)
    tot = Fraction(0)
    for e, c in coefficients(n, m):
        if e >= j:
            tot += c * _falling(e, j) * r ** (e - j)
    return tot


def radial_at_one(n: int, m: int, j: int) -> int:
    """d^j/dr^j R at r = 1: an exact integer."""
    return sum(c * _falling(e, j) for e, c in coefficients(n, m) if e >= j)


def radial_at_zero(n: int, m: int, j: int) -> int:
    """d^j/dr^j R at r = 0 = j! * [r^j] R: an exact integer."""
    for e, c in coefficients(n, m):
        if e == j:
            return factorial(j) * c
    return 0


def as_fraction(hi: float, lo: float) -> Fraction:
    return Fraction(hi) + Fraction(lo)
