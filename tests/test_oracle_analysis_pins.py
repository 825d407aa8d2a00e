"""Pins for the oracle's analysis transform (CPU only).

c_k = (1/N_k) sum_p w_p Z_k(p) f_p inverts the series for band-limited data
when the quadrature integrates Z_k Z_k' exactly: pinned by the round trip
(analysis of a synthesised series returns its coefficients), by integrals
with closed forms, and by the loss of exactness below the stated grid size.
"""
from __future__ import annotations

import numpy as np

import zp_workloads as W


def test_grid_integrates_closed_forms(oracle_mod):
    o = oracle_mod
    r, th, w = o.analysis_grid(6, 13)
    assert abs(w.sum() - np.pi) <= 1e-14                      # area of the unit disc
    assert abs(np.sum(w * r**2) - np.pi / 2) <= 1e-14         # integral of r^2
    assert abs(np.sum(w * r**10) - np.pi / 6) <= 1e-14        # integral of r^10 = 2 pi / 12
    assert abs(np.sum(w * (r * np.cos(th)) ** 2) - np.pi / 4) <= 1e-14  # integral of x^2
    assert abs(np.sum(w * r**3 * np.sin(3 * th))) <= 1e-14


def test_mode_norms_match_quadrature(oracle_mod):
    o = oracle_mod
    L = 12
    n, m = W.ansi_modes(L)
    r, th, w = o.analysis_grid((L + 2) // 2 + 1, 2 * L + 3)
    Z = o.basis(n, m, r, th, 1)[0]
    G = (Z * w) @ Z.T
    assert np.abs(G - np.diag(o.mode_norms(n, m))).max() <= 1e-14


def test_round_trip_exact_grid(oracle_mod):
    o = oracle_mod
    rng = np.random.default_rng(4)
    for L in (0, 1, 7, 20):
        n, m = W.ansi_modes(L)
        nr, nt = (L + 2) // 2, 2 * L + 1  # ceil((L+1)/2), 2L+1
        r, th, w = o.analysis_grid(nr, nt)
        Z = o.basis(n, m, r, th, 1)[0]
        c = rng.standard_normal((n.size, 3))
        back = o.analysis(Z, n, m, w, o.series_fwd(Z, c))
        assert np.abs(back - c).max() <= 1e-12, L


def test_round_trip_fails_below_stated_grid(oracle_mod):
    """One radial node or angle fewer than stated breaks exactness."""
    o = oracle_mod
    rng = np.random.default_rng(5)
    L = 10
    n, m = W.ansi_modes(L)
    c = rng.standard_normal((n.size, 1))
    for nr, nt in (((L + 2) // 2 - 1, 2 * L + 1), ((L + 2) // 2, 2 * L)):
        r, th, w = o.analysis_grid(nr, nt)
        Z = o.basis(n, m, r, th, 1)[0]
        assert np.abs(o.analysis(Z, n, m, w, o.series_fwd(Z, c)) - c).max() > 1e-3
