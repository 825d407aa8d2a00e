"""GPU parity of the analysis transform (zp_series_analysis): coefficients
c_k = (1/N_k) sum_p w_p Z_k(p) f_p from samples, against the oracle on the
same inputs, plus the round trip analysis(series(c)) = c on an exact grid.

The quadrature points and weights given to both sides come from the oracle's
rule (numpy's Gauss-Legendre) or from seeded random disc points.
Error measure: ||GPU - oracle||_inf / ||oracle||_inf per coefficient tensor;
1e-12 for FP64, 5e-7 (half the 1e-6 bar of the mixed-precision series) for
the FP32 and split-BF16x3 contractions.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import zp_workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 5e-7, "bf16x3": 5e-7}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def zp():
    import paper_2409_19156_amd as zp

    assert torch.cuda.is_available()
    return zp


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _rel(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got))
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def _case(o, L, nr, nt, B, seed):
    rng = np.random.default_rng(seed)
    n, m = W.ansi_modes(L)
    r, th, w = o.analysis_grid(nr, nt)
    f = rng.standard_normal((r.size, B))
    return n, m, r, th, w, f


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("L,nr,nt,B", [(20, 11, 41, 3), (64, 33, 129, 64)])
def test_analysis_matches_oracle(zp, oracle_mod, prec, L, nr, nt, B):
    n, m, r, th, w, f = _case(oracle_mod, L, nr, nt, B, seed=L)
    _say(f"analysis L={L} modes={n.size} P={r.size} B={B} prec={prec}")
    Z = oracle_mod.basis(n, m, r, th, 1)[0]
    ref = oracle_mod.analysis(Z, n, m, w, f)
    got = zp.series_analysis(n, m, _dev(r), _dev(th), _dev(w), _dev(f), prec).cpu().numpy()
    e = _rel(got, ref)
    _say(f"  rel err {e:.2e}")
    assert e <= TOL[prec]


@pytest.fixture(scope="module")
def full_ref(oracle_mod):
    """The timed configuration: 2145 modes (n <= 64) from samples on a 256 x 512
    grid (131072 points) for 1024 sets; the oracle forms every mode's
    coefficient for 32 sampled sets, summing chunks of points (the transform
    is linear in the samples)."""
    n, m, r, th, w, f = _case(oracle_mod, 64, 256, 512, 1024, seed=65)
    bs = np.sort(np.random.default_rng(66).choice(f.shape[1], 32, replace=False))
    _say(f"[oracle] analysis modes={n.size} P={r.size} on {bs.size} sets")
    acc = np.zeros((n.size, bs.size))
    step = 16384
    for p0 in range(0, r.size, step):
        sl = slice(p0, p0 + step)
        Z = oracle_mod.basis(n, m, r[sl], th[sl], oracle_mod.MASK_Z)[0]
        acc += oracle_mod.analysis(Z, n, m, w[sl], f[sl][:, bs])
    return (n, m, r, th, w, f), bs, acc


@pytest.mark.parametrize("prec", ["bf16x3", "fp64"])
def test_analysis_full_size_sampled(zp, full_ref, prec):
    (n, m, r, th, w, f), bs, ref = full_ref
    _say(f"analysis full size {prec}")
    got = zp.series_analysis(n, m, _dev(r), _dev(th), _dev(w), _dev(f), prec).cpu().numpy()
    e = _rel(got[:, bs], ref)
    _say(f"  rel err {e:.2e}")
    assert e <= TOL[prec]


def test_analysis_any_rule(zp, oracle_mod):
    """Random disc points with equal weights (a Monte Carlo rule): not exact,
    but both sides compute the same sum."""
    n, m = W.ansi_modes(15)
    r, th = W.disc_points(12, 777)
    w = np.full(r.size, np.pi / r.size)
    f = np.random.default_rng(13).standard_normal((r.size, 5))
    ref = oracle_mod.analysis(oracle_mod.basis(n, m, r, th, 1)[0], n, m, w, f)
    for prec in ("fp64", "bf16x3"):
        got = zp.series_analysis(n, m, _dev(r), _dev(th), _dev(w), _dev(f), prec).cpu().numpy()
        assert _rel(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_round_trip_on_exact_grid(zp, oracle_mod, prec):
    """analysis(series(c)) = c for band-limited data (both on the GPU)."""
    L = 40
    n, m = W.ansi_modes(L)
    r, th, w = oracle_mod.analysis_grid((L + 2) // 2, 2 * L + 1)
    c = np.random.default_rng(3).standard_normal((n.size, 7)) / (n + 1.0)[:, None]
    f = zp.series_forward(n, m, _dev(r), _dev(th), _dev(c), "fp64")
    back = zp.series_analysis(n, m, _dev(r), _dev(th), _dev(w), f, prec).cpu().numpy()
    e = _rel(back, c)
    _say(f"round trip L={L} prec={prec}: {e:.2e}")
    assert e <= (1e-12 if prec == "fp64" else 5e-7)


def test_analysis_with_library_grid(zp, oracle_mod):
    """The library's own host rule gives the same exact round trip."""
    L = 30
    n, m = W.ansi_modes(L)
    r, th, w = zp.analysis_grid((L + 2) // 2, 2 * L + 1)
    c = np.random.default_rng(8).standard_normal((n.size, 2))
    Z = oracle_mod.basis(n, m, r, th, 1)[0]
    f = oracle_mod.series_fwd(Z, c)
    back = zp.series_analysis(n, m, _dev(r), _dev(th), _dev(w), _dev(f)).cpu().numpy()
    assert np.abs(back - c).max() <= 1e-12


def test_analysis_chunked_and_edge_cases(zp, oracle_mod):
    import ctypes

    from paper_2409_19156_amd import _lib

    n, m, r, th, w, f = _case(oracle_mod, 12, 7, 25, 2, seed=1)
    full, mn = ctypes.c_size_t(), ctypes.c_size_t()
    lib = _lib.load()
    assert lib.zp_series_analysis_workspace(n.size, r.size, 2, 0, ctypes.byref(full), ctypes.byref(mn)) == 0
    a = zp.series_analysis(n, m, _dev(r), _dev(th), _dev(w), _dev(f)).cpu().numpy()
    ws = torch.empty(mn.value, dtype=torch.uint8, device="cuda")
    b = zp.series_analysis(n, m, _dev(r), _dev(th), _dev(w), _dev(f), ws=ws).cpu().numpy()
    assert _rel(b, a) <= 1e-13
    # no points: all coefficients zero; duplicated / unsorted modes
    z = zp.series_analysis(n, m, _dev([]), _dev([]), _dev([]), _dev(np.zeros((0, 3)))).cpu().numpy()
    assert z.shape == (n.size, 3) and not z.any()
    perm = np.random.default_rng(2).permutation(n.size)
    n2, m2 = np.concatenate([n[perm], n[:3]]), np.concatenate([m[perm], m[:3]])
    c2 = zp.series_analysis(n2, m2, _dev(r), _dev(th), _dev(w), _dev(f)).cpu().numpy()
    assert _rel(c2[: n.size], a[perm]) <= 1e-14 and _rel(c2[n.size:], a[:3]) <= 1e-14
