"""Pins for the oracle's Zernike series and its adjoint (CPU only).

The series f[p, b] = sum_k c[k, b] Z_k(r_p, theta_p) is linear in c, and each
point's (r, theta) enters only that point's row, so:
* dL/dc is exactly the change of L = sum(g * f) for a unit step in c;
* dL/dr_p and dL/dtheta_p are the limits of central differences of L in r_p
  and theta_p (re-evaluating the oracle basis at the moved point);
* at r = 0 the series does not depend on theta.
"""
from __future__ import annotations

import numpy as np

import zp_workloads as W


def _setup(oracle_mod, nmax=10, npts=12, nb=3, seed=21):
    rng = np.random.default_rng(seed)
    n, m = W.ansi_modes(nmax)
    r = np.sqrt(rng.random(npts))
    th = 2 * np.pi * rng.random(npts)
    c = rng.standard_normal((n.size, nb)) / (n + 1.0)[:, None]
    g = rng.standard_normal((npts, nb))
    return n, m, r, th, c, g


def _loss(oracle_mod, n, m, r, th, c, g):
    Z = oracle_mod.basis(n, m, r, th, 1)[0]
    return float(np.sum(g * oracle_mod.series_fwd(Z, c)))


def test_grad_c_is_exact_linear_increment(oracle_mod):
    n, m, r, th, c, g = _setup(oracle_mod)
    Z, Zr, Zt = oracle_mod.series_basis(n, m, r, th)
    gc, _, _ = oracle_mod.series_bwd(Z, Zr, Zt, c, g)
    L0 = _loss(oracle_mod, n, m, r, th, c, g)
    for k, b in [(0, 0), (5, 1), (n.size - 1, 2), (17, 0)]:
        c2 = c.copy()
        c2[k, b] += 1.0
        assert abs((_loss(oracle_mod, n, m, r, th, c2, g) - L0) - gc[k, b]) <= 1e-12 * (1 + abs(gc[k, b]))


def test_grad_r_theta_central_differences(oracle_mod):
    n, m, r, th, c, g = _setup(oracle_mod)
    Z, Zr, Zt = oracle_mod.series_basis(n, m, r, th)
    _, gr, gt = oracle_mod.series_bwd(Z, Zr, Zt, c, g)
    h = 1e-6
    for p in range(r.size):
        for vec, grad in ((r, gr), (th, gt)):
            a, b = vec.copy(), vec.copy()
            a[p] += h
            b[p] -= h
            if vec is r:
                fd = (_loss(oracle_mod, n, m, a, th, c, g) - _loss(oracle_mod, n, m, b, th, c, g)) / (2 * h)
            else:
                fd = (_loss(oracle_mod, n, m, r, a, c, g) - _loss(oracle_mod, n, m, r, b, c, g)) / (2 * h)
            assert abs(fd - grad[p]) <= 1e-6 * (1 + abs(grad[p])), (p, fd, grad[p])


def test_series_at_centre(oracle_mod):
    n, m, _, _, c, _ = _setup(oracle_mod)
    th = np.linspace(0, 2 * np.pi, 7)
    r = np.zeros_like(th)
    g = np.ones((th.size, c.shape[1]))
    Z, Zr, Zt = oracle_mod.series_basis(n, m, r, th)
    f = oracle_mod.series_fwd(Z, c)
    assert np.all(f == f[:1])
    _, _, gt = oracle_mod.series_bwd(Z, Zr, Zt, c, g)
    assert np.all(gt == 0.0)


def test_second_derivative_planes_by_central_differences(oracle_mod):
    """d2Z/dr2, d2Z/(dr dtheta), d2Z/dtheta2 against central differences of
    the (pinned) first-derivative planes."""
    n, m, r, th, _, _ = _setup(oracle_mod, nmax=9, npts=6)
    r = 0.05 + 0.9 * r
    Zrr, Zrt, Ztt = oracle_mod.series_basis2(n, m, r, th)
    h = 1e-6
    _, Zr_p, Zt_p = oracle_mod.series_basis(n, m, r + h, th)
    _, Zr_m, Zt_m = oracle_mod.series_basis(n, m, r - h, th)
    assert np.abs((Zr_p - Zr_m) / (2 * h) - Zrr).max() <= 1e-6 * (1 + np.abs(Zrr).max())
    assert np.abs((Zt_p - Zt_m) / (2 * h) - Zrt).max() <= 1e-6 * (1 + np.abs(Zrt).max())
    _, Zr_p, Zt_p = oracle_mod.series_basis(n, m, r, th + h)
    _, Zr_m, Zt_m = oracle_mod.series_basis(n, m, r, th - h)
    assert np.abs((Zr_p - Zr_m) / (2 * h) - Zrt).max() <= 1e-6 * (1 + np.abs(Zrt).max())
    assert np.abs((Zt_p - Zt_m) / (2 * h) - Ztt).max() <= 1e-6 * (1 + np.abs(Ztt).max())


def _l2(o, n, m, r, th, c, g, uc, ur, ut):
    Z, Zr, Zt = o.series_basis(n, m, r, th)
    gc, gr, gt = o.series_bwd(Z, Zr, Zt, c, g)
    return float(np.sum(uc * gc) + np.sum(ur * gr) + np.sum(ut * gt))


def test_second_order_adjoint(oracle_mod):
    """dL2/dg and dL2/dc as exact linear increments (L2 is linear in each of
    g and c); dL2/dr, dL2/dtheta by central differences of the pinned
    first-order adjoint."""
    o = oracle_mod
    n, m, r, th, c, g = _setup(o, nmax=8, npts=9, nb=2, seed=5)
    rng = np.random.default_rng(6)
    uc, ur, ut = rng.standard_normal(c.shape), rng.standard_normal(r.size), rng.standard_normal(r.size)
    Z, Zr, Zt = o.series_basis(n, m, r, th)
    og, oc, orr, ot = o.series_bwd2(Z, Zr, Zt, *o.series_basis2(n, m, r, th), c, g, uc, ur, ut)
    L0 = _l2(o, n, m, r, th, c, g, uc, ur, ut)
    for (p, b) in [(0, 0), (4, 1), (8, 0)]:
        g2 = g.copy()
        g2[p, b] += 1.0
        assert abs(_l2(o, n, m, r, th, c, g2, uc, ur, ut) - L0 - og[p, b]) <= 1e-11 * (1 + abs(og[p, b]))
    for (k, b) in [(0, 0), (10, 1), (n.size - 1, 1)]:
        c2 = c.copy()
        c2[k, b] += 1.0
        assert abs(_l2(o, n, m, r, th, c2, g, uc, ur, ut) - L0 - oc[k, b]) <= 1e-11 * (1 + abs(oc[k, b]))
    h = 1e-6
    for p in range(r.size):
        for vec, grad in ((r, orr), (th, ot)):
            a, b2 = vec.copy(), vec.copy()
            a[p] += h
            b2[p] -= h
            if vec is r:
                fd = (_l2(o, n, m, a, th, c, g, uc, ur, ut) - _l2(o, n, m, b2, th, c, g, uc, ur, ut)) / (2 * h)
            else:
                fd = (_l2(o, n, m, r, a, c, g, uc, ur, ut) - _l2(o, n, m, r, b2, c, g, uc, ur, ut)) / (2 * h)
            assert abs(fd - grad[p]) <= 1e-6 * (1 + abs(grad[p])), (p, fd, grad[p])


# ---- the float64 contraction against exactly summed products -------------------
#
# The series oracle contracts its basis in float64 (BLAS).  The checks below
# recompute sampled outputs as exact sums of products: every product of
# doubles is expanded into an exact sum of doubles by Dekker's TwoProduct with
# Veltkamp's splitting, and the pieces are added by math.fsum (Shewchuk's exact
# summation, correctly rounded).  For the first-order outputs the basis enters
# as the oracle's binary128 value (hi + lo), so rounding it to double is
# covered too; the second-order outputs take the oracle's float64 planes as
# given and check the contraction alone.

import math  # noqa: E402
from fractions import Fraction  # noqa: E402


def _split(a):
    t = 134217729.0 * a  # 2^27 + 1
    hi = t - (t - a)
    return hi, a - hi


def _two_prod(a, b):
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    return p, ((ah * bh - p) + ah * bl + al * bh) + al * bl


def _exact_dot(pieces, *factors):
    """sum_i (sum of pieces)[i] * prod_j factors[j][i] (all broadcast to one
    shape), correctly rounded."""
    shape = np.broadcast_shapes(*(np.shape(x) for x in (*pieces, *factors)))
    pieces = [np.broadcast_to(p, shape) for p in pieces]
    for f in factors:
        nxt = []
        for p in pieces:
            a, b = _two_prod(p, np.broadcast_to(f, shape))
            nxt += [a, b]
        pieces = nxt
    return math.fsum(np.concatenate([np.ravel(p) for p in pieces]).tolist())


def test_exact_dot_helper_against_fractions():
    rng = np.random.default_rng(3)
    a, b, c = (rng.standard_normal(300) * 10.0 ** rng.integers(-8, 8, 300) for _ in range(3))
    lo = a * 2.0 ** -60
    exact = sum(Fraction(x) * Fraction(y) * Fraction(z) + Fraction(w) * Fraction(y) * Fraction(z)
                for x, w, y, z in zip(a, lo, b, c))
    assert _exact_dot([a, lo], b, c) == float(exact)


def _rel_err(got, exact, norm):
    return abs(got - exact) / norm


def test_float64_series_reference_vs_exact_sums(oracle_mod):
    """f, grad_c, grad_r, grad_theta of the oracle (n <= 40, 861 modes) at
    sampled entries: within 1e-13 of the output's largest entry from the
    exactly summed products over the binary128 basis (expected: a few units
    of 1e-16; the GPU bar against this reference is 1e-12)."""
    o = oracle_mod
    rng = np.random.default_rng(23)
    n, m = W.ansi_modes(40)
    P, B = 48, 8
    r, th = W.disc_points(23, P)
    c = rng.standard_normal((n.size, B)) / (n + 1.0)[:, None]
    g = rng.standard_normal((P, B))
    hi, lo = o.basis(n, m, r, th, o.MASK_Z | o.MASK_DR | o.MASK_DTHETA, with_lo=True)
    Z, Zr, Zt = hi
    f = o.series_fwd(Z, c)
    gc, gr, gt = o.series_bwd(Z, Zr, Zt, c, g)
    worst = {}
    nf = np.abs(f).max()
    worst["f"] = max(_rel_err(f[p, b], _exact_dot([hi[0][:, p], lo[0][:, p]], c[:, b]), nf)
                     for p, b in zip(rng.integers(0, P, 40), rng.integers(0, B, 40)))
    nc = np.abs(gc).max()
    worst["grad_c"] = max(_rel_err(gc[k, b], _exact_dot([hi[0][k], lo[0][k]], g[:, b]), nc)
                          for k, b in zip(rng.integers(0, n.size, 40), rng.integers(0, B, 40)))
    for name, q, grad in (("grad_r", 1, gr), ("grad_theta", 2, gt)):
        nrm = np.abs(grad).max()
        worst[name] = max(_rel_err(grad[p], _exact_dot([hi[q][:, p, None], lo[q][:, p, None]], c, g[p][None, :]), nrm)
                          for p in range(0, P, 3))
    assert max(worst.values()) <= 1e-13, worst


def test_float64_second_order_contraction_vs_exact_sums(oracle_mod):
    """The second-order adjoint (out_g, out_c, out_r, out_theta), n <= 24, at
    sampled entries, against exactly summed products of the same float64
    planes: within 1e-13 of each output's largest entry."""
    o = oracle_mod
    rng = np.random.default_rng(24)
    n, m = W.ansi_modes(24)
    P, B = 32, 6
    r, th = W.disc_points(24, P)
    c = rng.standard_normal((n.size, B)) / (n + 1.0)[:, None]
    g = rng.standard_normal((P, B))
    uc, ur, ut = rng.standard_normal(c.shape), rng.standard_normal(P), rng.standard_normal(P)
    Z, Zr, Zt = o.series_basis(n, m, r, th)
    Zrr, Zrt, Ztt = o.series_basis2(n, m, r, th)
    og, oc, orr, ot = o.series_bwd2(Z, Zr, Zt, Zrr, Zrt, Ztt, c, g, uc, ur, ut)
    one = lambda x: [np.asarray(x, dtype=np.float64)]  # noqa: E731
    worst = {}
    # out_g[p,b] = sum_k Z uc + ur sum_k Zr c + ut sum_k Zt c
    nrm = np.abs(og).max()
    worst["out_g"] = max(_rel_err(og[p, b], _exact_dot(one(np.concatenate([Z[:, p], Zr[:, p], Zt[:, p]])),
                                                       np.concatenate([uc[:, b], c[:, b], c[:, b]]),
                                                       np.concatenate([np.ones(n.size), np.full(n.size, ur[p]),
                                                                       np.full(n.size, ut[p])])), nrm)
                         for p, b in zip(rng.integers(0, P, 24), rng.integers(0, B, 24)))
    # out_c[k,b] = sum_p (Zr ur + Zt ut)[k,p] g[p,b]
    nrm = np.abs(oc).max()
    worst["out_c"] = max(_rel_err(oc[k, b], _exact_dot(one(np.concatenate([Zr[k], Zt[k]])), np.concatenate([ur, ut]),
                                                       np.concatenate([g[:, b], g[:, b]])), nrm)
                         for k, b in zip(rng.integers(0, n.size, 24), rng.integers(0, B, 24)))
    # out_r[p] = sum_k sum_b (Zr uc + ur Zrr c + ut Zrt c)[k] g[p,b]; out_t with (Zt, Zrt, Ztt)
    for name, out, (A, Bp, Cp) in (("out_r", orr, (Zr, Zrr, Zrt)), ("out_theta", ot, (Zt, Zrt, Ztt))):
        nrm = np.abs(out).max()
        errs = []
        for p in range(0, P, 4):
            gp = g[p][None, :]
            pieces = [np.concatenate([A[:, p, None], Bp[:, p, None], Cp[:, p, None]])]  # [3M, 1]
            second = np.concatenate([uc, np.full_like(c, ur[p]), np.full_like(c, ut[p])])  # [3M, B]
            third = np.concatenate([np.ones_like(c), c, c])
            errs.append(_rel_err(out[p], _exact_dot(pieces, second, third, gp), nrm))
        worst[name] = max(errs)
    assert max(worst.values()) <= 1e-13, worst
