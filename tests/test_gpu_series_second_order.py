"""GPU parity of the second-order adjoint of the series (zp_series_bwd2:
double backward / Hessian-vector products) against the oracle's term-by-term
formula, and torch's double-backward checks through ZernikeSeries.

Error measure: ||GPU - oracle||_inf / ||oracle||_inf per output tensor; 1e-12
for FP64, 5e-7 (half the 1e-6 bar of the mixed-precision series) for the
FP32 and split-BF16x3 contractions.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import zp_workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 5e-7, "bf16x3": 5e-7}
NAMES = ("out_g", "out_c", "out_r", "out_t")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def zp():
    import paper_2409_19156_amd as zp

    assert torch.cuda.is_available()
    return zp


def _dev(x):
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _rel(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got))
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def _case(nmax, npts, nb, seed):
    rng = np.random.default_rng(seed)
    n, m = W.ansi_modes(nmax)
    r, th = W.disc_points(seed, npts)
    c = rng.standard_normal((n.size, nb)) / (n + 1.0)[:, None]
    g = rng.standard_normal((npts, nb))
    uc = rng.standard_normal((n.size, nb))
    ur, ut = rng.standard_normal(npts), rng.standard_normal(npts)
    return n, m, r, th, c, g, uc, ur, ut


def _oracle(o, n, m, r, th, c, g, uc, ur, ut):
    Z, Zr, Zt = o.series_basis(n, m, r, th)
    zero = np.zeros
    uc = zero(c.shape) if uc is None else uc
    ur = zero(r.size) if ur is None else ur
    ut = zero(r.size) if ut is None else ut
    return o.series_bwd2(Z, Zr, Zt, *o.series_basis2(n, m, r, th), c, g, uc, ur, ut)


def _gpu(zp, n, m, r, th, c, g, uc, ur, ut, prec, ws=None):
    outs = zp.series_backward2(n, m, _dev(r), _dev(th), _dev(c), _dev(g), _dev(uc), _dev(ur), _dev(ut), prec, ws=ws)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in outs]


@pytest.fixture(scope="module")
def case12(oracle_mod):
    args = _case(12, 700, 3, seed=31)
    return args, _oracle(oracle_mod, *args)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_bwd2_matches_oracle(zp, case12, prec):
    args, ref = case12
    got = _gpu(zp, *args, prec)
    errs = {k: _rel(a, b) for k, a, b in zip(NAMES, got, ref)}
    _say(f"bwd2 n<=12 P=700 B=3 {prec}:", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, e in errs.items():
        assert e <= TOL[prec], (k, e)


@pytest.mark.parametrize("which", ["uc", "ur", "ut", "none"])
def test_bwd2_partial_cotangents(zp, oracle_mod, which):
    n, m, r, th, c, g, uc, ur, ut = _case(9, 300, 2, seed=32)
    keep = {"uc": (uc, None, None), "ur": (None, ur, None), "ut": (None, None, ut), "none": (None, None, None)}[which]
    ref = _oracle(oracle_mod, n, m, r, th, c, g, *keep)
    got = _gpu(zp, n, m, r, th, c, g, *keep, "fp64")
    for k, a, b in zip(NAMES, got, ref):
        if not np.any(b):
            assert not np.any(a), (which, k)
        else:
            assert _rel(a, b) <= 1e-12, (which, k)


def test_bwd2_chunked_workspace(zp, case12):
    import ctypes

    from paper_2409_19156_amd import _lib

    args, ref = case12
    n = args[0]
    full, mn = ctypes.c_size_t(), ctypes.c_size_t()
    assert _lib.load().zp_series_bwd2_workspace(n.size, 700, 3, 0, ctypes.byref(full), ctypes.byref(mn)) == 0
    assert mn.value < full.value
    ws = torch.empty(mn.value, dtype=torch.uint8, device="cuda")
    got = _gpu(zp, *args, "fp64", ws=ws)
    for k, a, b in zip(NAMES, got, ref):
        assert _rel(a, b) <= 1e-12, k


def test_bwd2_fp64_chunks_read_g_in_place(zp, oracle_mod):
    """FP64 with 128 sets and the smallest workspace: chunks of 128 points read
    their rows of g in place at offset p0 > 0; the ragged last chunk (100
    points) goes through the padded copy.  Against the oracle."""
    import ctypes

    from paper_2409_19156_amd import _lib

    P, B = 12 * 128 + 100, 128
    args = _case(16, P, B, seed=42)
    n = args[0]
    full, mn = ctypes.c_size_t(), ctypes.c_size_t()
    assert _lib.load().zp_series_bwd2_workspace(n.size, P, B, 0, ctypes.byref(full), ctypes.byref(mn)) == 0
    assert mn.value < full.value
    ws = torch.empty(mn.value, dtype=torch.uint8, device="cuda")
    _say(f"bwd2 fp64 in-place g chunks: M={n.size} P={P} B={B} ws={mn.value}")
    got = _gpu(zp, *args, "fp64", ws=ws)
    ref = _oracle(oracle_mod, *args)
    for k, a, b in zip(NAMES, got, ref):
        assert _rel(a, b) <= 1e-12, k


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_bwd2_n40(zp, oracle_mod, prec):
    """861 modes, 4096 points, 64 sets."""
    args = _case(40, 4096, 64, seed=33)
    ref = _oracle(oracle_mod, *args)
    got = _gpu(zp, *args, prec)
    errs = {k: _rel(a, b) for k, a, b in zip(NAMES, got, ref)}
    _say(f"bwd2 n<=40 P=4096 B=64 {prec}:", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, e in errs.items():
        assert e <= TOL[prec], (k, e)


@pytest.fixture(scope="module")
def n64_bwd2_ref(oracle_mod):
    """The timed configuration: 2145 modes, 65536 points, 1024 sets, with the
    cotangents drawn as in the benchmark.  The oracle evaluates dL2/dg,
    dL2/dr and dL2/dtheta on 256 sampled points (all sets; they are pointwise
    in p), and dL2/dc on 32 sampled sets (all modes), summed over chunks of
    points.  dL2/dc does not involve Z or the second-order planes, so those
    chunks pass zeros for them."""
    o = oracle_mod
    wl = W.series_n64()
    rng = np.random.default_rng(7)
    uc = rng.standard_normal(wl.c.shape) / (wl.n + 1.0)[:, None]
    ur, ut = rng.standard_normal(wl.P), rng.standard_normal(wl.P)
    pick = np.random.default_rng(98)
    ps = np.sort(pick.choice(wl.P, 256, replace=False))
    bs = np.sort(pick.choice(wl.B, 32, replace=False))
    _say(f"[oracle] bwd2 n64 on {ps.size} points and {bs.size} sets")
    g_ref, _, r_ref, t_ref = _oracle(o, wl.n, wl.m, wl.r[ps], wl.theta[ps], wl.c, wl.g[ps], uc, ur[ps], ut[ps])
    c_ref = np.zeros((wl.M, bs.size))
    step = 8192
    for p0 in range(0, wl.P, step):
        sl = slice(p0, p0 + step)
        Zr, Zt = o.basis(wl.n, wl.m, wl.r[sl], wl.theta[sl], o.MASK_DR | o.MASK_DTHETA)
        zero = np.zeros_like(Zr)
        c_ref += o.series_bwd2(zero, Zr, Zt, zero, zero, zero, wl.c[:, bs], wl.g[sl][:, bs], uc[:, bs], ur[sl],
                               ut[sl])[1]
    return wl, (uc, ur, ut), ps, bs, (g_ref, c_ref, r_ref, t_ref)


@pytest.mark.parametrize("prec", ["bf16x3", "fp64"])
def test_bwd2_n64_full_size_sampled(zp, n64_bwd2_ref, prec):
    wl, (uc, ur, ut), ps, bs, (g_ref, c_ref, r_ref, t_ref) = n64_bwd2_ref
    _say(f"[bwd2] n64 full size {prec}")
    out_g, out_c, out_r, out_t = _gpu(zp, wl.n, wl.m, wl.r, wl.theta, wl.c, wl.g, uc, ur, ut, prec)
    errs = {"out_g": _rel(out_g[ps], g_ref), "out_c": _rel(out_c[:, bs], c_ref), "out_r": _rel(out_r[ps], r_ref),
            "out_t": _rel(out_t[ps], t_ref)}
    _say(f"  {prec}:", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, e in errs.items():
        assert e <= TOL[prec], (k, e)


def test_double_backward_gradgradcheck(zp):
    n, m = W.ansi_modes(5)
    rng = np.random.default_rng(34)
    r, th = W.disc_points(35, 6)
    r = _dev(0.1 + 0.8 * r).requires_grad_()
    th = _dev(th).requires_grad_()
    c = _dev(rng.standard_normal((n.size, 2))).requires_grad_()
    fn = lambda c_, r_, t_: zp.series(c_, r_, t_, n, m, "fp64")  # noqa: E731
    assert torch.autograd.gradgradcheck(fn, (c, r, th), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_hessian_vector_product_matches_oracle(zp, oracle_mod):
    """Hv of L = sum(w * f) through autograd's double backward (which calls
    zp_series_bwd2) against the oracle formula: with g = w fixed, the gradient
    (grad_c, grad_r, grad_t) has the directional derivative along
    (vc, vr, vt) given by series_bwd2 with cotangents (vc, vr, vt)."""
    n, m, r, th, c, w, vc, vr, vt = _case(10, 257, 2, seed=36)
    rt, tt, ct = (_dev(x).requires_grad_() for x in (r, th, c))
    f = zp.series(ct, rt, tt, n, m, "fp64")
    L = (f * _dev(w)).sum()
    gc, gr, gt = torch.autograd.grad(L, (ct, rt, tt), create_graph=True)
    s = (gc * _dev(vc)).sum() + (gr * _dev(vr)).sum() + (gt * _dev(vt)).sum()
    hc, hr, ht = torch.autograd.grad(s, (ct, rt, tt))
    _, oc, orr, ot = _oracle(oracle_mod, n, m, r, th, c, w, vc, vr, vt)
    for got, ref in ((hc, oc), (hr, orr), (ht, ot)):
        assert _rel(got.cpu().numpy(), ref) <= 1e-12
