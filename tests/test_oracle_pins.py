"""Pins for the quad-precision oracle (CPU only).

Each test fixes the oracle against something other than itself: the paper's
closed forms and printed values, exact integer and rational arithmetic,
identities the polynomials satisfy, and independent library routines.  A
dropped term, a wrong sign or index, or a transposed argument anywhere in the
oracle (Jacobi seeds, recurrence, derivative identity, chain rule, Leibniz
rule, the (-1)^K factor, the angular factor) breaks at least one of them.
"""
from __future__ import annotations

import os
from fractions import Fraction
from math import comb

import mpmath
import numpy as np
import pytest
from scipy.special import roots_jacobi

from tests import exact_ref as X
import zp_workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line)
    return rows


def _poly_deriv(coefs, r, j):
    """d^j/dr^j of sum_i coefs[i] r^i, exactly."""
    tot = Fraction(0)
    for i, c in enumerate(coefs):
        if i >= j and c:
            f = 1
            for t in range(j):
                f *= i - t
            tot += c * f * Fraction(r) ** (i - j)
    return tot


R_POINTS = [0.0, 1.0, 0.5, 0.25, 0.125, 2.0 ** -30, 1.0 - 2.0 ** -30, 0.7071067811865475,
            0.7071067811865476, 0.3, 0.6180339887498949, 0.9, 0.99, 0.123456789, 0.987654321]


def test_golden_low_order_polynomials(oracle_mod):
    """Hand-expanded closed forms (incl. R_2^0 = 2r^2-1, R_4^0 = 6r^4-6r^2+1), all
    four derivative orders, both signs of m."""
    rows = _read_golden("radial_low_order.txt")
    ns, ms, polys = [], [], []
    for row in rows:
        head, coefs = row.split(":")
        n, m = map(int, head.split())
        ns += [n, n]
        ms += [m, -m]
        polys += [[int(c) for c in coefs.split()]] * 2
    assert ns[4:6] == [2, 2] and polys[4] == [-1, 0, 2]
    hi, lo = oracle_mod.radial(ns, ms, R_POINTS, 3, with_lo=True)
    for i, poly in enumerate(polys):
        for j in range(4):
            for p, r in enumerate(R_POINTS):
                ref = _poly_deriv(poly, r, j)
                got = X.as_fraction(hi[j, i, p], lo[j, i, p])
                assert abs(float(got - ref)) <= 1e-30 * max(1.0, abs(float(ref))), (ns[i], ms[i], j, r)


def test_golden_center_values(oracle_mod):
    """Eq. (zernike-at0): value at r = 0."""
    rows = [list(map(int, r.split())) for r in _read_golden("center_values.txt")]
    n = [r[0] for r in rows]
    m = [r[1] for r in rows]
    hi = oracle_mod.radial(n, m, [0.0], 0)
    for i, row in enumerate(rows):
        assert hi[0, i, 0] == row[2], row


def test_closed_form_coefficients_agree():
    """Eq. (radial-part-eq) and Eq. (radial-part-eq-binom) give the same integers
    (so the exact reference below is itself consistent)."""
    for n in range(0, 61):
        for m in range(n % 2, n + 1, 2):
            assert X.coefficients(n, m) == X.coefficients_binom(n, m)


def test_exact_rational_small_n(oracle_mod):
    """All modes n <= 20, derivative orders 0..3, against exact rational
    evaluation of Eq. (radial-part-eq) at the exact binary value of each r."""
    n, m = W.radial_pairs(20)
    rng = np.random.default_rng(11)
    pts = R_POINTS + list(rng.random(10))
    hi, lo = oracle_mod.radial(n, m, pts, 3, with_lo=True)
    worst = 0.0
    for i in range(n.size):
        for j in range(4):
            scale = float(n[i] + 1) ** (2 * j)
            for p, r in enumerate(pts):
                ref = X.radial_exact(int(n[i]), int(m[i]), r, j)
                got = X.as_fraction(hi[j, i, p], lo[j, i, p])
                worst = max(worst, abs(float(got - ref)) / scale)
    assert worst <= 1e-28, worst


def _sparse_high_modes():
    """A sparse set of modes up to the largest degree the library accepts
    (n = 1000): every 25th m at n = 1000, 999, 998, 750 and 401, plus a few
    small, middle and near-diagonal m (the modes the GPU parity test at
    n = 1000 uses are among them)."""
    ms = list(range(0, 1001, 25)) + [1, 2, 3, 250, 499, 500, 501, 997, 999]
    modes = [(N, mm) for N in (1000, 999, 998, 750, 401) for mm in ms if mm <= N and (N - mm) % 2 == 0]
    return np.array([a for a, _ in modes]), np.array([b for _, b in modes])


def _mode_set(which):
    return W.radial_pairs(200) if which == "n<=200" else _sparse_high_modes()


@pytest.mark.parametrize("which", ["n<=200", "sparse n<=1000"])
def test_exact_integers_at_edge(oracle_mod, which):
    """r = 1: R = 1 for every mode (P_K^{(alpha,0)}(-1) = (-1)^K), and each
    derivative is the exact integer sum_s coef_s (n-2s)_j (falling factorial)."""
    n, m = _mode_set(which)
    hi, lo = oracle_mod.radial(n, m, [1.0], 3, with_lo=True)
    assert np.all(hi[0, :, 0] == 1.0)
    for i in range(n.size):
        for j in range(1, 4):
            ref = X.radial_at_one(int(n[i]), int(m[i]), j)
            got = X.as_fraction(hi[j, i, 0], lo[j, i, 0])
            assert abs(float(got - ref)) <= 1e-26 * max(1.0, abs(ref)), (n[i], m[i], j)
    # R'(1) = (n(n+2) - m^2)/2
    for i in range(0, n.size, 37 if n.size > 1000 else 1):
        assert hi[1, i, 0] == (n[i] * (n[i] + 2) - m[i] ** 2) / 2


@pytest.mark.parametrize("which", ["n<=200", "sparse n<=1000"])
def test_exact_integers_at_centre(oracle_mod, which):
    """r = 0: d^j R = j! [r^j] R, nonzero only for j >= m, j = m mod 2."""
    n, m = _mode_set(which)
    hi, lo = oracle_mod.radial(n, m, [0.0], 3, with_lo=True)
    for i in range(n.size):
        for j in range(4):
            ref = X.radial_at_zero(int(n[i]), int(m[i]), j)
            got = X.as_fraction(hi[j, i, 0], lo[j, i, 0])
            assert got == ref, (n[i], m[i], j, got, ref)


def test_parity_negative_r(oracle_mod):
    """R has only powers n - 2s: d^j R(-r) = (-1)^(n-j) d^j R(r)."""
    n, m = W.radial_pairs(60)
    r = np.array([0.1, 0.35, 0.5, 0.77, 0.95])
    a_hi, a_lo = oracle_mod.radial(n, m, r, 3, with_lo=True)
    b_hi, b_lo = oracle_mod.radial(n, m, -r, 3, with_lo=True)
    for j in range(4):
        sgn = (-1.0) ** ((n - j) % 2)
        d = (a_hi[j] + a_lo[j]) * sgn[:, None] - (b_hi[j] + b_lo[j])
        scale = (n + 1.0)[:, None] ** (2 * j)
        assert np.all(np.abs(d) <= 1e-28 * scale)


def test_zernike_radial_ode(oracle_mod):
    """The radial ODE r^2(1-r^2)R'' + r(1-3r^2)R' + (n(n+2)r^2 - m^2)R = 0 and its
    r-derivative (which brings in R'''), evaluated in exact arithmetic on the
    oracle's binary128 outputs."""
    n, m = W.radial_pairs(200)
    sel = np.arange(0, n.size, 97)
    n, m = n[sel], m[sel]
    rng = np.random.default_rng(5)
    pts = list(rng.random(4)) + [0.5, 0.999]
    hi, lo = oracle_mod.radial(n, m, pts, 3, with_lo=True)
    for i in range(n.size):
        N, Mm = int(n[i]), int(m[i])
        for p, rf in enumerate(pts):
            r = Fraction(rf)
            R = [X.as_fraction(hi[j, i, p], lo[j, i, p]) for j in range(4)]
            t = [r * r * (1 - r * r) * R[2], r * (1 - 3 * r * r) * R[1], (N * (N + 2) * r * r - Mm * Mm) * R[0]]
            res = sum(t)
            scale = sum(abs(x) for x in t) + 1
            assert abs(float(res / scale)) <= 1e-27, (N, Mm, rf)
            t3 = [(2 * r - 4 * r ** 3) * R[2], r * r * (1 - r * r) * R[3], (1 - 9 * r * r) * R[1],
                  r * (1 - 3 * r * r) * R[2], 2 * N * (N + 2) * r * R[0], (N * (N + 2) * r * r - Mm * Mm) * R[1]]
            res3 = sum(t3)
            scale3 = sum(abs(x) for x in t3) + 1
            assert abs(float(res3 / scale3)) <= 1e-27, (N, Mm, rf)


def test_zernike_recursion_identity(oracle_mod):
    """Eq. (zernike-recursion), which ties chains of different |m| together:
    R_n^m = r [R_{n-1}^{|m-1|} + R_{n-1}^{m+1}] - R_{n-2}^m, for m + 1 <= n - 1."""
    n, m = W.radial_pairs(200)
    index = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(n, m))}
    pts = np.array([0.05, 0.4, 0.7071, 0.93, 0.9999])
    hi, lo = oracle_mod.radial(n, m, pts, 0, with_lo=True)
    R = hi[0] + lo[0]  # float64 view is enough for a relative test at 1e-13
    checked = 0
    for (a, b), i in index.items():
        if b + 1 > a - 1:
            continue
        i1 = index[(a - 1, abs(b - 1))]
        i2 = index[(a - 1, b + 1)]
        i3 = index[(a - 2, b)]
        rhs = pts * (R[i1] + R[i2]) - R[i3]
        assert np.all(np.abs(R[i] - rhs) <= 1e-13), (a, b)
        checked += 1
    assert checked > 9000


@pytest.mark.parametrize("mm,nmax,tol", [(0, 200, 1e-11), (1, 200, 1e-11), (7, 200, 1e-11), (50, 200, 1e-11),
                                         (120, 200, 1e-11), (199, 200, 1e-11), (0, 1000, 1e-9), (1, 1000, 1e-9),
                                         (333, 1000, 1e-9), (998, 1000, 1e-9)])
def test_orthogonality_gauss_jacobi(oracle_mod, mm, nmax, tol):
    """int_0^1 R_n^m R_n'^m r dr = delta_nn' / (2(n+1)) for every n <= nmax of one
    m.  With x = 1 - 2r^2 the integral is 2^-(m+2) int (1-x)^m F(x) dx,
    F = R_n R_n' / r^(2m) a polynomial, done exactly by Gauss-Jacobi
    quadrature (alpha = m, beta = 0) from scipy."""
    ns = np.arange(mm, nmax + 1, 2)
    K = (ns - mm) // 2
    N = int(K.max()) + 2
    x, w = roots_jacobi(N, mm, 0)
    r = np.sqrt((1 - x) / 2)
    R = oracle_mod.radial(ns, np.full_like(ns, mm), r, 0)[0]
    F = R / r[None, :] ** mm
    G = (F * w) @ F.T * 2.0 ** (-mm - 2)
    target = np.diag(1 / (2 * (ns + 1.0)))
    # The Gram matrix is summed in float64 over N ~ K_max nodes: rounding grows with N (about 1e-10 of the
    # smallest diagonal entry at n <= 1000); a wrong term gives O(1) deviations.
    assert np.abs(G - target).max() <= tol * (1 / (2 * (ns.max() + 1.0)))


def test_jacobi_chain_vs_mpmath(oracle_mod):
    """The oracle's Jacobi chain (Eq. jacobi seeds + Eq. jacobi-recursion) against
    mpmath.jacobi at 50 digits, for beta = 0 and beta = j != 0 chains."""
    mpmath.mp.dps = 50
    for (a, b) in [(0, 0), (3, 1), (50, 2), (150, 3), (0, 3), (7, 0)]:
        for x in [-0.999999, -0.5, 0.001, 0.3141592653589793, 0.9, 0.99999999, -0.9999999999]:
            hi, lo = oracle_mod.jacobi_chain(100, a, b, x)
            for k in range(0, 101, 7):
                ref = mpmath.jacobi(k, a, b, mpmath.mpf(x))
                scale = comb(k + max(a, b), k)
                got = mpmath.mpf(hi[k]) + mpmath.mpf(lo[k])
                assert abs(got - ref) <= 1e-28 * scale, (a, b, x, k)
    mpmath.mp.dps = 15


def test_jacobi_explicit_sum_vs_chain(oracle_mod):
    """Eq. (jacobi) summed directly equals the recurrence for small degree."""
    for (a, b) in [(0, 0), (4, 2), (11, 3)]:
        for x in [-0.8, 0.1, 0.77]:
            hi, lo = oracle_mod.jacobi_chain(12, a, b, x)
            for k in range(13):
                e_hi, e_lo = oracle_mod.jacobi_explicit(k, a, b, x)
                assert abs((hi[k] - e_hi) + (lo[k] - e_lo)) <= 1e-28 * comb(k + max(a, b), k)


@pytest.mark.parametrize("nm", [(200, 0), (200, 2), (199, 1), (200, 50), (200, 150), (201, 201), (180, 96),
                                (1000, 0), (1000, 250), (1000, 500), (999, 1), (1000, 1000)])
def test_high_n_derivatives_vs_mpmath(oracle_mod, nm):
    """n ~ 200 and n ~ 1000 (the largest degree the library accepts), derivative
    orders 0..3, against mpmath: (-1)^K r^m jacobi(K,m,0,1-2r^2) differentiated
    numerically by mpmath.diff at 60 digits (80 above n = 200)."""
    n, m = nm
    K = (n - m) // 2
    mpmath.mp.dps = 60 if n <= 200 else 80
    pts = [0.0312, 0.3, 0.70710678, 0.8123, 0.9999]
    hi, lo = oracle_mod.radial([n], [m], pts, 3, with_lo=True)

    def f(t):
        return (-1) ** K * t ** m * mpmath.jacobi(K, m, 0, 1 - 2 * t * t)

    for p, r in enumerate(pts):
        for j in range(4):
            ref = mpmath.diff(f, mpmath.mpf(r), j)
            got = mpmath.mpf(hi[j, 0, p]) + mpmath.mpf(lo[j, 0, p])
            assert abs(got - ref) <= 1e-27 * (n + 1.0) ** (2 * j), (n, m, r, j)
    mpmath.mp.dps = 15


def test_basis_angular_factor_vs_mpmath(oracle_mod):
    """Eq. (zernike-poly): cos for m >= 0, sin(|m| theta) for m < 0, on every
    radial derivative; dZ/dtheta by mpmath.diff in theta."""
    mpmath.mp.dps = 40
    n, m = W.ansi_modes(8)
    r = np.array([0.0, 0.3, 0.81, 1.0])
    th = np.array([0.0, 1.1, 3.3, 6.0])
    hi, lo = oracle_mod.basis(n, m, r, th, 31, with_lo=True)
    for i in range(n.size):
        N, Mm = int(n[i]), int(m[i])
        a = abs(Mm)
        for p in range(r.size):
            ang = mpmath.sin if Mm < 0 else mpmath.cos
            for j in range(4):
                ref = mpmath.mpf(X.radial_exact(N, a, r[p], j).numerator) / X.radial_exact(N, a, r[p], j).denominator
                ref = ref * ang(a * mpmath.mpf(th[p]))
                got = mpmath.mpf(hi[j, i, p]) + mpmath.mpf(lo[j, i, p])
                assert abs(got - ref) <= 1e-28 * (N + 1) ** (2 * j), (N, Mm, j, p)
            R0 = X.radial_exact(N, a, r[p], 0)
            R0 = mpmath.mpf(R0.numerator) / R0.denominator
            dth = mpmath.diff(lambda t: R0 * ang(a * t), mpmath.mpf(th[p]))
            got = mpmath.mpf(hi[4, i, p]) + mpmath.mpf(lo[4, i, p])
            assert abs(got - dth) <= 1e-28 * (N + 1), (N, Mm, p)
    mpmath.mp.dps = 15


def test_basis_centre_is_theta_independent(oracle_mod):
    n, m = W.ansi_modes(30)
    th = np.linspace(0, 2 * np.pi, 9)
    Z = oracle_mod.basis(n, m, np.zeros_like(th), th, 1 | 16)
    assert np.all(Z[0] == Z[0][:, :1])
    assert np.all(Z[1] == 0.0)


def test_oracle_rejects_invalid_modes(oracle_mod):
    for n, m in [(-1, 0), (3, 0), (2, 4), (5, -6)]:
        with pytest.raises(ValueError):
            oracle_mod.radial([n], [m], [0.5], 0)
