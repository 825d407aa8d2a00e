"""Helpers for the GPU parity tests: tolerances and error reduction.

Tolerances: max over points of |GPU - oracle| <= 1e-13 (n+1)^(2j) for the
j-th r-derivative of each mode (R or Z), and 1e-13 (n+1) for dZ/dtheta (one
theta-derivative brings a factor |m| <= n).
"""
from __future__ import annotations

import numpy as np


def radial_tol(n, j: int) -> np.ndarray:
    return 1e-13 * (np.asarray(n, dtype=np.float64) + 1.0) ** (2 * j)


def dtheta_tol(n) -> np.ndarray:
    return 1e-13 * (np.asarray(n, dtype=np.float64) + 1.0)


def worst_ratio(got: np.ndarray, ref: np.ndarray, tol: np.ndarray):
    """got, ref: [M, P]; tol: [M].  Returns (max err/tol, argmax mode, max err)."""
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got)), "non-finite GPU output"
    err = np.abs(got - ref).max(axis=1) if got.size else np.zeros(got.shape[0])
    ratio = err / tol
    i = int(np.argmax(ratio)) if ratio.size else 0
    return (float(ratio[i]) if ratio.size else 0.0), i, (float(err[i]) if err.size else 0.0)
