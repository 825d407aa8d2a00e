"""Pins for the oracle's three-dimensional spectral series (CPU only).

f[p, q, b] = sum_j c[j, b] R_{n_j}^{|m_j|}(r_p) F_{m_j}(theta_p) F_{l_j}(phi_q)
(the paper's duplicated-mode use, Sec. 3 footnote), with F_l(phi) = cos(l phi)
for l >= 0 and sin(|l| phi) for l < 0.  Pinned by closed forms, by reduction to
the two-dimensional series, by separability, by discrete Fourier
orthogonality, and by exact / central-difference checks of the adjoint.
"""
from __future__ import annotations

import numpy as np

import zp_workloads as W


def _fwd(o, n, m, l, r, th, phi, c):
    Z = o.basis(n, m, r, th, 1)[0]
    return o.series3d_fwd(Z, o.fourier(l, phi), c)


def test_single_mode_closed_forms(oracle_mod):
    o = oracle_mod
    rng = np.random.default_rng(0)
    r, th, phi = rng.random(9), 2 * np.pi * rng.random(9), 2 * np.pi * rng.random(5)
    one = np.ones((1, 1))
    f = _fwd(o, [2], [0], [1], r, th, phi, one)[:, :, 0]
    ref = np.outer(2 * r**2 - 1, np.cos(phi))
    assert np.abs(f - ref).max() <= 1e-14
    f = _fwd(o, [3], [-1], [-2], r, th, phi, one)[:, :, 0]
    ref = np.outer((3 * r**3 - 2 * r) * np.sin(th), np.sin(2 * phi))
    assert np.abs(f - ref).max() <= 1e-14
    f = _fwd(o, [4], [2], [0], r, th, phi, 2.5 * one)[:, :, 0]
    ref = np.outer(2.5 * (4 * r**4 - 3 * r**2) * np.cos(2 * th), np.ones_like(phi))
    assert np.abs(f - ref).max() <= 1e-13


def test_fourier_derivative_and_orthogonality(oracle_mod):
    o = oracle_mod
    Q = 16
    phi = 2 * np.pi * np.arange(Q) / Q
    ls = np.arange(-7, 8)
    F = o.fourier(ls, phi)
    G = F @ F.T
    expect = np.diag(np.where(ls == 0, Q, Q / 2.0))
    assert np.abs(G - expect).max() <= 1e-12
    x = np.array([0.3, 1.7, 4.0])
    h = 1e-6
    fd = (o.fourier(ls, x + h) - o.fourier(ls, x - h)) / (2 * h)
    assert np.abs(fd - o.fourier(ls, x, 1)).max() <= 1e-7


def test_reduces_to_planar_series(oracle_mod):
    o = oracle_mod
    n, m = W.ansi_modes(6)
    rng = np.random.default_rng(1)
    r, th = W.disc_points(2, 40)
    c = rng.standard_normal((n.size, 3))
    f3 = _fwd(o, n, m, np.zeros_like(n), r, th, [0.0, 1.0, 2.0], c)
    f2 = o.series_fwd(o.basis(n, m, r, th, 1)[0], c)
    for q in range(3):
        assert np.abs(f3[:, q, :] - f2).max() <= 1e-13


def test_separable_when_every_mode_shares_l(oracle_mod):
    o = oracle_mod
    n, m = W.ansi_modes(5)
    rng = np.random.default_rng(3)
    r, th = W.disc_points(4, 30)
    phi = 2 * np.pi * rng.random(6)
    c = rng.standard_normal((n.size, 2))
    f3 = _fwd(o, n, m, np.full_like(n, -3), r, th, phi, c)
    f2 = o.series_fwd(o.basis(n, m, r, th, 1)[0], c)
    ref = f2[:, None, :] * np.sin(3 * phi)[None, :, None]
    assert np.abs(f3 - ref).max() <= 1e-13


def test_duplicated_modes_add(oracle_mod):
    """Two copies of one (n, m, l) act as one mode with the summed coefficient."""
    o = oracle_mod
    r, th = W.disc_points(7, 20)
    phi = np.array([0.1, 0.9])
    c = np.array([[0.25], [0.5]])
    f = _fwd(o, [5, 5], [1, 1], [2, 2], r, th, phi, c)
    g = _fwd(o, [5], [1], [2], r, th, phi, np.array([[0.75]]))
    assert np.abs(f - g).max() <= 1e-14


def _case(seed=11):
    rng = np.random.default_rng(seed)
    n, m, l = W.spectral3d_modes(4, 2)
    r, th = W.disc_points(seed, 7)
    phi = 2 * np.pi * rng.random(4)
    c = rng.standard_normal((n.size, 2))
    g = rng.standard_normal((r.size, phi.size, 2))
    return n, m, l, r, th, phi, c, g


def _loss(o, n, m, l, r, th, phi, c, g):
    return float(np.sum(g * _fwd(o, n, m, l, r, th, phi, c)))


def test_adjoint_exact_in_c_and_central_differences(oracle_mod):
    o = oracle_mod
    n, m, l, r, th, phi, c, g = _case()
    Z, Zr, Zt = o.series_basis(n, m, r, th)
    gc, gr, gt, gp = o.series3d_bwd(Z, Zr, Zt, o.fourier(l, phi), o.fourier(l, phi, 1), c, g)
    L0 = _loss(o, n, m, l, r, th, phi, c, g)
    for j, b in [(0, 0), (13, 1), (n.size - 1, 0)]:
        c2 = c.copy()
        c2[j, b] += 1.0
        assert abs(_loss(o, n, m, l, r, th, phi, c2, g) - L0 - gc[j, b]) <= 1e-12 * (1 + abs(gc[j, b]))
    h = 1e-6
    for which, vec, grad in (("r", r, gr), ("t", th, gt), ("p", phi, gp)):
        for i in range(vec.size):
            a, b = vec.copy(), vec.copy()
            a[i] += h
            b[i] -= h
            args_a = dict(r=r, th=th, phi=phi)
            args_b = dict(r=r, th=th, phi=phi)
            key = {"r": "r", "t": "th", "p": "phi"}[which]
            args_a[key], args_b[key] = a, b
            fd = (_loss(o, n, m, l, c=c, g=g, **args_a) - _loss(o, n, m, l, c=c, g=g, **args_b)) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-6 * (1 + abs(grad[i])), (which, i, fd, grad[i])
