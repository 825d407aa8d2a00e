"""zp_basis_polar (the basis on a tensor grid of radii x angles) against
zp_basis on the same points flattened -- bit for bit, since every value is
formed the same way -- and against the oracle, on ragged and degenerate grid
shapes (odd angle counts take the one-point-per-lane path)."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import zp_workloads as W
from tests.gpu_util import dtheta_tol, radial_tol, worst_ratio

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def zp():
    import paper_2409_19156_amd as zp

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return zp


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _both(zp, n, m, rr, th, mask):
    r = np.repeat(rr, th.size)
    theta = np.tile(th, rr.size)
    pol = zp.basis_polar(n, m, _dev(rr), _dev(th), mask).cpu().numpy()
    flat = zp.basis(n, m, _dev(r), _dev(theta), mask).cpu().numpy()
    return pol, flat, r, theta


def test_metric_grid_bitwise_equal_to_basis(zp):
    """The 1326-mode basis on 64 CGL radii x 128 angles, all five outputs."""
    n, m = W.ansi_modes(50)
    rr, th = W.cgl_polar_axes(64, 128)
    _say(f"[polar] L50: M={n.size} grid 64 x 128")
    pol, flat, _, _ = _both(zp, n, m, rr, th, 31)
    assert np.array_equal(pol, flat)


@pytest.mark.parametrize("nr,nt", [(1, 1), (1, 2), (3, 5), (7, 64), (5, 129), (33, 257), (2, 1000), (65, 8)])
def test_ragged_grids_against_basis_and_oracle(zp, oracle_mod, nr, nt):
    n, m = W.ansi_modes(12)
    n = np.concatenate([n, [12, 4, 7]]).astype(np.int32)  # a duplicate and an odd-n sin mode
    m = np.concatenate([m, [-2, 0, -3]]).astype(np.int32)
    rng = np.random.default_rng(nr * 1000 + nt)
    rr = np.sort(np.concatenate([[0.0, 1.0], rng.random(max(nr - 2, 0))]))[:nr]
    th = 2 * np.pi * rng.random(nt)
    _say(f"[polar] grid {nr} x {nt}, M={n.size}")
    pol, flat, r, theta = _both(zp, n, m, rr, th, 31)
    assert np.array_equal(pol, flat)
    ref = oracle_mod.basis(n, m, r, theta, 31)
    for q in range(5):
        tol = dtheta_tol(n) if q == 4 else radial_tol(n, q)
        ratio, i, err = worst_ratio(pol[q], ref[q], tol)
        assert ratio <= 1.0, f"plane {q}: err {err:.3g} at (n,m)=({n[i]},{m[i]}), {ratio:.3g} x tol"


@pytest.mark.parametrize("mask", [1, 2, 16, 1 | 8, 2 | 4 | 16])
def test_mask_subsets_equal_full_mask(zp, mask):
    n, m = W.ansi_modes(20)
    rr, th = W.cgl_polar_axes(16, 48)
    full = zp.basis_polar(n, m, _dev(rr), _dev(th), 31).cpu().numpy()
    sub = zp.basis_polar(n, m, _dev(rr), _dev(th), mask).cpu().numpy()
    planes = [q for q in range(5) if (mask >> q) & 1]
    assert np.array_equal(sub, full[planes])


def test_empty_grids_are_noops(zp):
    n, m = W.ansi_modes(4)
    for nr, nt in ((0, 5), (5, 0), (0, 0)):
        out = zp.basis_polar(n, m, _dev(np.zeros(nr)), _dev(np.zeros(nt)), 31)
        assert out.shape == (5, n.size, 0)
