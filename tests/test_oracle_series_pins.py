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
