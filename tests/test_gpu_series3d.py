"""GPU parity of the three-dimensional spectral series (zp_series3d_fwd /
zp_series3d_bwd; the paper's duplicated-mode use, Sec. 3 footnote) against
the oracle, which evaluates the full, duplicated mode list with no
deduplication.

Error measure per output tensor: ||GPU - oracle||_inf / ||oracle||_inf, with
the planar series' bounds: 1e-12 for FP64, 5e-7 (half the 1e-6 bar of the
mixed-precision series) for the FP32 and split-BF16x3 contractions.
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


def _oracle(o, w, pts=None):
    """Oracle f and adjoint (grad_c only when all points are used)."""
    r, th, g = w.r, w.theta, w.g
    if pts is not None:
        r, th, g = r[pts], th[pts], g[pts]
    Z, Zr, Zt = o.series_basis(w.n, w.m, r, th)
    F, dF = o.fourier(w.l, w.phi), o.fourier(w.l, w.phi, 1)
    f = o.series3d_fwd(Z, F, w.c)
    return (f, *o.series3d_bwd(Z, Zr, Zt, F, dF, w.c, g))


def _gpu(zp, w, prec, cache=True, ws=None, mem_budget=None):
    r, th, ph, c, g = _dev(w.r), _dev(w.theta), _dev(w.phi), _dev(w.c), _dev(w.g)
    cache_t = None
    if cache:
        _, _, cb = zp.series3d_sizes(w.n, w.m, w.l, w.r.size, w.phi.size, w.c.shape[1], prec)
        cache_t = torch.empty(cb, dtype=torch.uint8, device="cuda")
    f = zp.series3d_forward(w.n, w.m, w.l, r, th, ph, c, prec, cache=cache_t, ws=ws, mem_budget=mem_budget)
    grads = zp.series3d_backward(w.n, w.m, w.l, r, th, ph, c, g, prec, cache=cache_t, ws=ws, mem_budget=mem_budget)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (f, *grads)]


@pytest.fixture(scope="module")
def small(oracle_mod):
    w = W.spectral3d_small()
    return w, _oracle(oracle_mod, w)


NAMES = ("f", "grad_c", "grad_r", "grad_theta", "grad_phi")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("cache", [True, False])
def test_series3d_matches_oracle(zp, small, prec, cache):
    w, ref = small
    _say(f"series3d small: J={w.J} P={w.r.size} Q={w.phi.size} B={w.c.shape[1]} prec={prec} cache={cache}")
    got = _gpu(zp, w, prec, cache=cache)
    errs = {k: _rel(a, b) for k, a, b in zip(NAMES, got, ref)}
    _say("  rel err", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, e in errs.items():
        assert e <= TOL[prec], (k, e)


def test_series3d_equals_planar_series_over_duplicated_modes(zp, small):
    """The deduplicated path against the planar series over all J modes with
    coefficients c[j][b] F_{l_j}(phi_q) (both on the GPU)."""
    w, _ = small
    Q, B = w.phi.size, w.c.shape[1]
    a = np.abs(w.l)[:, None] * w.phi[None, :]
    F = np.where(w.l[:, None] >= 0, np.cos(a), np.sin(a))
    cq = (w.c[:, None, :] * F[:, :, None]).reshape(w.J, Q * B)
    f2 = zp.series_forward(w.n, w.m, _dev(w.r), _dev(w.theta), _dev(cq), "fp64").cpu().numpy().reshape(-1, Q, B)
    f3 = _gpu(zp, w, "fp64")[0]
    assert _rel(f3, f2) <= 1e-12


def test_series3d_chunked_workspace(zp, small):
    w, ref = small
    full, mn, _ = zp.series3d_sizes(w.n, w.m, w.l, w.r.size, w.phi.size, w.c.shape[1], "fp64")
    assert mn < full
    a = _gpu(zp, w, "fp64", cache=False)
    ws = torch.empty(mn, dtype=torch.uint8, device="cuda")
    b = _gpu(zp, w, "fp64", cache=False, ws=ws)
    assert np.array_equal(a[0], b[0])  # each point's row is computed the same way
    for x, y, k in zip(a[1:], b[1:], NAMES[1:]):
        assert _rel(y, x) <= 1e-13, k
    for x, y in zip(b, ref):
        assert _rel(x, y) <= 1e-12


def test_series3d_deterministic(zp, small):
    w, _ = small
    a = _gpu(zp, w, "bf16x3")
    b = _gpu(zp, w, "bf16x3")
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_series3d_ragged_and_large_l(zp, oracle_mod):
    """Unsorted modes, repeated triples, large |l|, one point / plane / set."""
    rng = np.random.default_rng(8)
    n = np.array([6, 0, 6, 3, 6, 3, 12, 12, 0], dtype=np.int32)
    m = np.array([-2, 0, -2, 1, 4, -3, 0, 0, 0], dtype=np.int32)
    l = np.array([5, 0, 5, -1000, 2, 7, -3, 3, 999], dtype=np.int32)
    for P, Q, B in [(1, 1, 1), (129, 3, 1), (40, 1, 5), (257, 17, 2)]:
        r, th = W.disc_points(int(rng.integers(1 << 30)), P)
        w = W.Spectral3D("ragged", n, m, l, r, th, 2 * np.pi * rng.random(Q), rng.standard_normal((n.size, B)),
                         rng.standard_normal((P, Q, B)))
        ref = _oracle(oracle_mod, w)
        for prec in ("fp64", "bf16x3"):
            got = _gpu(zp, w, prec, cache=(P % 2 == 1))
            for k, a, b in zip(NAMES, got, ref):
                assert _rel(a, b) <= TOL[prec], (P, Q, B, prec, k)


def test_series3d_empty(zp):
    r, th, ph = _dev([0.5, 0.1]), _dev([1.0, 2.0]), _dev([0.3])
    f = zp.series3d_forward([], [], [], r, th, ph, _dev(np.zeros((0, 2))))
    assert f.shape == (2, 1, 2) and not f.any()
    gc, gr, gt, gp = zp.series3d_backward([], [], [], r, th, ph, _dev(np.zeros((0, 2))), _dev(np.ones((2, 1, 2))))
    assert gc.shape == (0, 2) and not gr.any() and not gt.any() and not gp.any()
    f = zp.series3d_forward([2], [0], [1], r, th, _dev([]), _dev([[1.0]]))
    assert f.shape == (2, 0, 1)
    # the planar series' empty sum is zero as well
    f = zp.series_forward([], [], r, th, _dev(np.zeros((0, 3))))
    assert f.shape == (2, 3) and not f.any()


def test_series3d_gradcheck(zp):
    n, m, l = W.spectral3d_modes(3, 1)
    rng = np.random.default_rng(2)
    r, th = W.disc_points(3, 5)
    r = _dev(0.1 + 0.8 * r).requires_grad_()
    th = _dev(th).requires_grad_()
    ph = _dev(2 * np.pi * rng.random(3)).requires_grad_()
    c = _dev(rng.standard_normal((n.size, 2))).requires_grad_()
    fn = lambda c_, r_, t_, p_: zp.series3d(c_, r_, t_, p_, n, m, l, "fp64")  # noqa: E731
    assert torch.autograd.gradcheck(fn, (c, r, th, ph), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_series3d_autograd_matches_adjoint(zp, small):
    w, ref = small
    r, th, ph, c = (_dev(x).requires_grad_() for x in (w.r, w.theta, w.phi, w.c))
    f = zp.series3d(c, r, th, ph, w.n, w.m, w.l, "fp64")
    f.backward(_dev(w.g))
    for got, k, exp in zip((c.grad, r.grad, th.grad, ph.grad), NAMES[1:], ref[1:]):
        assert _rel(got.cpu().numpy(), exp) <= 1e-12, k


def _oracle_all_points(o, w, chunk=1024):
    """The oracle at every point, plane and mode of a large workload.  The basis
    of mode j is the oracle basis of its pair (n_j, m_j), evaluated at every
    point once per distinct pair; ``series3d_fwd`` / ``series3d_bwd`` then run
    over consecutive chunks of the full (duplicated) mode list: grad_c of a
    mode depends on that mode alone, and f, grad_r, grad_theta and grad_phi
    are sums over modes, so the chunks' results add up."""
    pairs, inv = np.unique(np.stack([w.n, w.m]), axis=1, return_inverse=True)
    inv = inv.reshape(-1)
    Zu, Zru, Ztu = o.series_basis(pairs[0], pairs[1], w.r, w.theta)
    F, dF = o.fourier(w.l, w.phi), o.fourier(w.l, w.phi, 1)
    P, Q, B = w.r.size, w.phi.size, w.c.shape[1]
    f, gc = np.zeros((P, Q, B)), np.zeros(w.c.shape)
    gr, gt, gp = np.zeros(P), np.zeros(P), np.zeros(Q)
    for j0 in range(0, w.J, chunk):
        sl = slice(j0, min(w.J, j0 + chunk))
        u = inv[sl]
        f += o.series3d_fwd(Zu[u], F[sl], w.c[sl])
        a, b, c, d = o.series3d_bwd(Zu[u], Zru[u], Ztu[u], F[sl], dF[sl], w.c[sl], w.g)
        gc[sl] = a
        gr += b
        gt += c
        gp += d
    return f, gc, gr, gt, gp


@pytest.fixture(scope="module")
def l32(oracle_mod):
    w = W.spectral3d_L32()
    _say(f"series3d L32 oracle: J={w.J} P={w.r.size} Q={w.phi.size} (every point, plane and mode)")
    return w, _oracle_all_points(oracle_mod, w)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_series3d_L32_full_size(zp, l32, prec):
    """The benchmark workload (18 513 modes = 561 (n, m) pairs x 33 values of l,
    32 768 polar points, 64 planes): every element of f, grad_c (all modes),
    grad_r, grad_theta (all points) and grad_phi (all planes) against the
    oracle; in addition, the adjoint identity <grad_c, dc> = <g, f(dc)> (f is
    linear in c) and a central difference in phi."""
    w, ref = l32
    P, Q, B = w.r.size, w.phi.size, w.c.shape[1]
    _say(f"series3d L32: J={w.J} P={P} Q={Q} B={B} prec={prec}")
    got = _gpu(zp, w, prec)
    errs = {k: _rel(a, b) for k, a, b in zip(NAMES, got, ref)}
    _say("  rel err", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, e in errs.items():
        assert e <= TOL[prec], (k, e)
    rng = np.random.default_rng(9)
    # adjoint identity in c (FP64 forward of a random direction)
    dc = rng.standard_normal(w.c.shape)
    r, th, ph = _dev(w.r), _dev(w.theta), _dev(w.phi)
    fd = zp.series3d_forward(w.n, w.m, w.l, r, th, ph, _dev(dc), "fp64").cpu().numpy()
    lhs, rhs = float(np.sum(got[1] * dc)), float(np.sum(w.g * fd))
    assert abs(lhs - rhs) <= TOL[prec] * np.abs(got[1]).sum() * np.abs(dc).max(), (lhs, rhs)
    # central difference in phi along a random direction (FP64)
    dp = rng.standard_normal(Q)
    h = 1e-5
    fp = zp.series3d_forward(w.n, w.m, w.l, r, th, _dev(w.phi + h * dp), _dev(w.c), "fp64").cpu().numpy()
    fm = zp.series3d_forward(w.n, w.m, w.l, r, th, _dev(w.phi - h * dp), _dev(w.c), "fp64").cpu().numpy()
    num = float(np.sum(w.g * (fp - fm)) / (2 * h))
    ana = float(np.dot(got[4], dp))
    assert abs(num - ana) <= 2e-6 * float(np.abs(got[4]) @ np.abs(dp)), (num, ana)
