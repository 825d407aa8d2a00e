"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds input structure only -- mode index sets, point grids and
random draws -- and none of the arithmetic of the Zernike method, so that the
GPU library and the reference oracle can both be fed from it without sharing
any computation.

Mode validity (paper Sec. 2): n >= 0, |m| <= n, n - |m| even.

Workloads (each named for what it is):
  radial_n16       radial pairs 0 <= m <= n <= 16 (81 pairs), derivative orders
                   0..3, 1000 uniform r from seed 0 plus r = 0 and r = 1 exactly.
  basis_L50        ANSI index set n <= 50 (1326 modes); polar grid of 64 radial
                   Chebyshev-Gauss-Lobatto points mapped to [0, 1] times 128
                   equispaced theta (8192 points); outputs Z, dZ/dr, d2Z/dr2,
                   d3Z/dr3, dZ/dtheta.
  radial_n200      radial pairs with n <= 200 (10201 pairs), derivative orders
                   0..2, 100000 r: half uniform, a quarter at 1 - 10^U(-8,0) and
                   a quarter at 10^U(-8,0) (seed 2).
  series_n40       ANSI n <= 40 (861 modes), 256 coefficient sets with
                   c_nm ~ N(0, 1/(n+1)^2), 16384 disc points r = sqrt(U),
                   theta = 2 pi U, upstream gradient N(0, 1) (seed 3), FP64.
  series_n64       ANSI n <= 64 (2145 modes), 65536 disc points, 1024
                   coefficient sets, same distributions (seed 4).
Draw order from ``numpy.random.default_rng(seed)``: r, theta, c, g.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def radial_pairs(nmax: int):
    """(n, m) with 0 <= m <= n <= nmax and n - m even, ordered by n then m."""
    n, m = [], []
    for nn in range(nmax + 1):
        for mm in range(nn % 2, nn + 1, 2):
            n.append(nn)
            m.append(mm)
    return np.array(n, dtype=np.int32), np.array(m, dtype=np.int32)


def ansi_modes(nmax: int):
    """ANSI (OSA) single-index order: n ascending, then m = -n, -n+2, ..., n.

    Mode j sits at index (n(n+2) + m) / 2."""
    n, m = [], []
    for nn in range(nmax + 1):
        for mm in range(-nn, nn + 1, 2):
            n.append(nn)
            m.append(mm)
    return np.array(n, dtype=np.int32), np.array(m, dtype=np.int32)


def cgl_polar_axes(nr: int = 64, nt: int = 128):
    """The two axes of the polar grid: nr Chebyshev-Gauss-Lobatto radii
    mapped to [0, 1], ascending, with the end points exactly 0 and 1, and nt
    equispaced theta in [0, 2 pi)."""
    i = np.arange(nr, dtype=np.float64)
    rr = np.sin(np.pi * i / (2.0 * (nr - 1))) ** 2  # (1 - cos(pi i/(nr-1))) / 2
    rr[0], rr[-1] = 0.0, 1.0
    th = 2.0 * np.pi * np.arange(nt, dtype=np.float64) / nt
    return rr, th


def cgl_polar_grid(nr: int = 64, nt: int = 128):
    """The polar grid's points, flattened: point p = nt * i + j (theta
    fastest) at (rr[i], th[j]) of ``cgl_polar_axes``."""
    rr, th = cgl_polar_axes(nr, nt)
    r = np.repeat(rr, nt)
    theta = np.tile(th, nr)
    return r, theta


@dataclass
class Workload:
    name: str
    n: np.ndarray
    m: np.ndarray
    r: np.ndarray
    theta: np.ndarray | None = None
    max_dr: int = 0
    mask: int = 0
    c: np.ndarray | None = None
    g: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.n.size)

    @property
    def P(self) -> int:
        return int(self.r.size)

    @property
    def B(self) -> int:
        return 0 if self.c is None else int(self.c.shape[1])


def radial_n16(seed: int = 0, npts: int = 1000) -> Workload:
    rng = np.random.default_rng(seed)
    n, m = radial_pairs(16)
    r = np.concatenate([rng.random(npts), [0.0, 1.0]])
    return Workload("radial_n16", n, m, r, max_dr=3)


def basis_L50(nr: int = 64, nt: int = 128) -> Workload:
    n, m = ansi_modes(50)
    r, theta = cgl_polar_grid(nr, nt)
    return Workload("basis_L50", n, m, r, theta, max_dr=3, mask=31)


def clustered_r(rng: np.random.Generator, npts: int) -> np.ndarray:
    """Half uniform on [0, 1); a quarter at 1 - 10^U(-8,0); a quarter at 10^U(-8,0)."""
    h = npts // 2
    q = (npts - h) // 2
    u = rng.random(h)
    near_edge = 1.0 - 10.0 ** rng.uniform(-8.0, 0.0, q)
    near_axis = 10.0 ** rng.uniform(-8.0, 0.0, npts - h - q)
    return np.concatenate([u, near_edge, near_axis])


def radial_n200(seed: int = 2, npts: int = 100_000, nmax: int = 200) -> Workload:
    rng = np.random.default_rng(seed)
    n, m = radial_pairs(nmax)
    return Workload("radial_n200", n, m, clustered_r(rng, npts), max_dr=2)


def _series(name: str, nmax: int, npts: int, nb: int, seed: int) -> Workload:
    rng = np.random.default_rng(seed)
    n, m = ansi_modes(nmax)
    r = np.sqrt(rng.random(npts))
    theta = 2.0 * np.pi * rng.random(npts)
    c = rng.standard_normal((n.size, nb)) / (n.astype(np.float64) + 1.0)[:, None]
    g = rng.standard_normal((npts, nb))
    return Workload(name, n, m, r, theta, c=c, g=g)


def series_n40(seed: int = 3, npts: int = 16384, nb: int = 256) -> Workload:
    return _series("series_n40", 40, npts, nb, seed)


def series_n64(seed: int = 4, npts: int = 65536, nb: int = 1024) -> Workload:
    return _series("series_n64", 64, npts, nb, seed)


def disc_points(seed: int, npts: int):
    """Random disc points: r = sqrt(U), theta = 2 pi U."""
    rng = np.random.default_rng(seed)
    return np.sqrt(rng.random(npts)), 2.0 * np.pi * rng.random(npts)


def n_entries(M: int, P: int, nout: int) -> int:
    return int(M) * int(P) * int(nout)


__all__ = [
    "radial_pairs", "ansi_modes", "cgl_polar_axes", "cgl_polar_grid", "clustered_r", "disc_points", "Workload",
    "radial_n16", "basis_L50", "radial_n200", "series_n40", "series_n64", "n_entries",
]


@dataclass
class Spectral3D:
    """Three-dimensional spectral series: modes (n, m, l), polar points
    (r_p, theta_p) times toroidal angles phi_q, B coefficient sets."""
    name: str
    n: np.ndarray
    m: np.ndarray
    l: np.ndarray
    r: np.ndarray
    theta: np.ndarray
    phi: np.ndarray
    c: np.ndarray
    g: np.ndarray

    @property
    def J(self) -> int:
        return int(self.n.size)


def spectral3d_modes(nmax: int, lmax: int):
    """Every ANSI Zernike mode n <= nmax paired with every l in [-lmax, lmax]
    (l outer), so each (n, m) appears 2 lmax + 1 times."""
    n2, m2 = ansi_modes(nmax)
    L = np.arange(-lmax, lmax + 1)
    return np.tile(n2, L.size), np.tile(m2, L.size), np.repeat(L, n2.size).astype(np.int32)


def spectral3d(name: str, nmax: int, lmax: int, r, theta, nphi: int, nb: int, seed: int) -> Spectral3D:
    rng = np.random.default_rng(seed)
    n, m, l = spectral3d_modes(nmax, lmax)
    phi = 2.0 * np.pi * np.arange(nphi, dtype=np.float64) / nphi
    scale = 1.0 / ((n + 1.0) * (np.abs(l) + 1.0))
    c = rng.standard_normal((n.size, nb)) * scale[:, None]
    g = rng.standard_normal((np.asarray(r).size, nphi, nb))
    return Spectral3D(name, n, m, l, np.asarray(r), np.asarray(theta), phi, c, g)


def spectral3d_small(seed: int = 5) -> Spectral3D:
    """n <= 8 (45 modes) x |l| <= 3: 315 modes, 300 disc points, 8 toroidal planes, 2 sets."""
    r, theta = disc_points(seed, 300)
    return spectral3d("spectral3d_small", 8, 3, r, theta, 8, 2, seed)


def spectral3d_L32(seed: int = 6) -> Spectral3D:
    """n <= 32 (561 modes) x |l| <= 16: 18 513 modes; 128 CGL radii x 256 theta
    = 32 768 polar points; 64 toroidal planes; one coefficient set."""
    r, theta = cgl_polar_grid(128, 256)
    return spectral3d("spectral3d_L32", 32, 16, r, theta, 64, 1, seed)
