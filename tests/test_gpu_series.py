"""GPU parity of the Zernike series and its adjoint (zp_series_fwd / zp_series_bwd)
against the oracle: the oracle basis (binary128, rounded to double) contracted
in float64.

Error measure per output tensor: ||GPU - oracle||_inf / ||oracle||_inf.
Bounds: 1e-12 for the FP64 contraction; 5e-7 for the FP32 and split-BF16x3
contractions (FP32 accumulation, flushed into FP64 every 16 to 64 terms): half
the 1e-6 relative error the mixed-precision series is held to.
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
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert np.all(np.isfinite(got))
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def _gpu_all(zp, wl, prec, cache=True, mem_budget=None):
    r, th, c, g = _dev(wl.r), _dev(wl.theta), _dev(wl.c), _dev(wl.g)
    full, mn, cb = zp.series_sizes(wl.M, wl.P, wl.B, prec)
    cache_t = torch.empty(cb, dtype=torch.uint8, device="cuda") if cache else None
    f = zp.series_forward(wl.n, wl.m, r, th, c, prec, cache=cache_t, mem_budget=mem_budget)
    gc, gr, gt = zp.series_backward(wl.n, wl.m, r, th, c, g, prec, cache=cache_t, mem_budget=mem_budget)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (f, gc, gr, gt)]


@pytest.fixture(scope="module")
def n40_ref(oracle_mod):
    wl = W.series_n40()
    _say(f"[oracle] series_n40 basis M={wl.M} P={wl.P}")
    Z, Zr, Zt = oracle_mod.series_basis(wl.n, wl.m, wl.r, wl.theta)
    f = oracle_mod.series_fwd(Z, wl.c)
    gc, gr, gt = oracle_mod.series_bwd(Z, Zr, Zt, wl.c, wl.g)
    return wl, (f, gc, gr, gt)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_series_n40_full(zp, n40_ref, prec):
    """861 modes, 16384 points, 256 coefficient sets: forward and all three
    gradients over the full size."""
    wl, ref = n40_ref
    _say(f"[series] n40 {prec}")
    got = _gpu_all(zp, wl, prec)
    for name, a, b in zip(("f", "grad_c", "grad_r", "grad_theta"), got, ref):
        e = _rel(a, b)
        _say(f"  {prec} {name}: rel err {e:.3g}")
        assert e <= TOL[prec], (prec, name, e)


def test_cache_and_recompute_are_bitwise_equal(zp):
    """Keeping the basis from the forward or recomputing it in the backward
    gives bitwise identical gradients (same workspace, same chunking)."""
    wl = W.series_n40(npts=3000, nb=40)
    for prec in ("fp64", "bf16x3"):
        a = _gpu_all(zp, wl, prec, cache=True)
        b = _gpu_all(zp, wl, prec, cache=False)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), prec


def test_chunked_workspace_matches_oracle(zp, oracle_mod):
    """A workspace budget far below the one-pass size forces chunking over points."""
    wl = W.series_n40(npts=5000, nb=24)
    full, mn, _ = zp.series_sizes(wl.M, wl.P, wl.B, "fp64")
    budget = max(mn, full // 7)
    got = _gpu_all(zp, wl, "fp64", cache=False, mem_budget=budget)
    Z, Zr, Zt = oracle_mod.series_basis(wl.n, wl.m, wl.r, wl.theta)
    ref = (oracle_mod.series_fwd(Z, wl.c),) + oracle_mod.series_bwd(Z, Zr, Zt, wl.c, wl.g)
    for a, b in zip(got, ref):
        assert _rel(a, b) <= 1e-12


def test_fp64_chunks_read_g_in_place(zp, oracle_mod):
    """FP64 with 128 sets and the smallest workspace: chunks of 128 points whose
    rows of g already have the padded layout, so every chunk but the last reads
    g in place at its offset (p0 > 0 for all but the first); the ragged last
    chunk (100 points) goes through the padded copy.  Against the oracle."""
    rng = np.random.default_rng(41)
    n, m = W.ansi_modes(20)
    P, B = 12 * 128 + 100, 128
    r, th = W.disc_points(41, P)
    c = rng.standard_normal((n.size, B)) / (n + 1.0)[:, None]
    g = rng.standard_normal((P, B))
    full, mn, _ = zp.series_sizes(n.size, P, B, "fp64")
    assert mn < full
    ws = torch.empty(mn, dtype=torch.uint8, device="cuda")
    _say(f"[series] fp64 in-place g chunks: M={n.size} P={P} B={B} ws={mn}")
    got = zp.series_backward(n, m, _dev(r), _dev(th), _dev(c), _dev(g), "fp64", ws=ws)
    torch.cuda.synchronize()
    Z, Zr, Zt = oracle_mod.series_basis(n, m, r, th)
    ref = oracle_mod.series_bwd(Z, Zr, Zt, c, g)
    for name, a, b in zip(("grad_c", "grad_r", "grad_theta"), got, ref):
        assert _rel(a.cpu().numpy(), b) <= 1e-12, name


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_pipelined_forward(zp, oracle_mod, prec):
    """With many points the forward runs chunks of points on two streams (on
    256 compute units and 1024 sets: chunks of 4096 points for FP64 and FP32,
    8192 for bf16).  A ragged point count, with and without the cache: equal
    to the oracle, and bitwise equal to a forward that runs sequential chunks
    (a small workspace budget turns the pipeline off); the same for the
    forward-mode derivative."""
    rng = np.random.default_rng(12)
    n, m = W.ansi_modes(20)
    P, B = 20001, 1024
    r, th = np.sqrt(rng.random(P)), 2 * np.pi * rng.random(P)
    c = rng.standard_normal((n.size, B))
    Z = oracle_mod.basis(n, m, r, th, 1)[0]
    ref = Z.T @ c
    rd, td, cd = _dev(r), _dev(th), _dev(c)
    full, mn, cb = zp.series_sizes(n.size, P, B, prec)
    seq = zp.series_forward(n, m, rd, td, cd, prec, mem_budget=max(mn, full // 3))
    for cache in (None, torch.empty(cb, dtype=torch.uint8, device="cuda")):
        _say(f"[series] pipelined forward {prec} P={P} cache={cache is not None}")
        f = zp.series_forward(n, m, rd, td, cd, prec, cache=cache)
        torch.cuda.synchronize()
        assert torch.equal(f, seq), (prec, cache is not None)
        assert _rel(f.cpu().numpy(), ref) <= TOL[prec]
    # the forward-mode derivative pipelines its chunks the same way
    tc, tr, tt = _dev(rng.standard_normal((n.size, B))), _dev(rng.standard_normal(P)), _dev(rng.standard_normal(P))
    tf = zp.series_jvp(n, m, rd, td, cd, tc, tr, tt, prec=prec)
    tf_seq = zp.series_jvp(n, m, rd, td, cd, tc, tr, tt, prec=prec, mem_budget=mn)
    torch.cuda.synchronize()
    assert torch.equal(tf, tf_seq), prec


@pytest.mark.parametrize("M_n,P,B", [(0, 1, 1), (1, 1, 1), (3, 65, 3), (7, 129, 65), (10, 300, 130)])
def test_ragged_shapes(zp, oracle_mod, M_n, P, B):
    rng = np.random.default_rng(P + B)
    n, m = W.ansi_modes(M_n)
    r, th = np.sqrt(rng.random(P)), 2 * np.pi * rng.random(P)
    c = rng.standard_normal((n.size, B))
    g = rng.standard_normal((P, B))
    wl = W.Workload("ragged", n, m, r, th, c=c, g=g)
    Z, Zr, Zt = oracle_mod.series_basis(n, m, r, th)
    ref = (oracle_mod.series_fwd(Z, c),) + oracle_mod.series_bwd(Z, Zr, Zt, c, g)
    for prec in ("fp64", "fp32", "bf16x3"):
        got = _gpu_all(zp, wl, prec)
        for a, b in zip(got, ref):
            assert _rel(a, b) <= TOL[prec], (prec, M_n, P, B)


def test_gradcheck_small(zp):
    """torch.autograd.gradcheck (central differences) through ZernikeSeries."""
    rng = np.random.default_rng(8)
    n, m = W.ansi_modes(6)
    P, B = 7, 2
    r = _dev(0.1 + 0.8 * rng.random(P)).requires_grad_()
    th = _dev(2 * np.pi * rng.random(P)).requires_grad_()
    c = _dev(rng.standard_normal((n.size, B))).requires_grad_()
    assert torch.autograd.gradcheck(lambda c_, r_, t_: zp.series(c_, r_, t_, n, m, "fp64"), (c, r, th),
                                    eps=1e-6, atol=1e-8, rtol=1e-6)


def test_autograd_matches_adjoint_and_budget_paths(zp):
    """loss.backward() through ZernikeSeries equals a direct zp_series_bwd call,
    with the basis kept (large budget) or recomputed (tiny budget)."""
    wl = W.series_n40(npts=2000, nb=16)
    g = _dev(wl.g)
    outs = []
    for budget in (1 << 34, 1 << 20):
        r = _dev(wl.r).requires_grad_()
        th = _dev(wl.theta).requires_grad_()
        c = _dev(wl.c).requires_grad_()
        f = zp.series(c, r, th, wl.n, wl.m, "fp64", mem_budget=budget)
        (f * g).sum().backward()
        outs.append((f.detach(), c.grad, r.grad, th.grad))
    gc, gr, gt = zp.series_backward(wl.n, wl.m, _dev(wl.r), _dev(wl.theta), _dev(wl.c), g, "fp64")
    for k, ref in enumerate((gc, gr, gt)):
        assert torch.equal(outs[0][k + 1], ref)
        rel = ((outs[1][k + 1] - ref).abs().max() / ref.abs().max()).item()
        assert rel <= 1e-13


def test_series_at_centre_has_no_theta_gradient(zp):
    n, m = W.ansi_modes(12)
    P, B = 9, 3
    r = torch.zeros(P, dtype=torch.float64, device="cuda")
    th = _dev(np.linspace(0, 6, P))
    c = _dev(np.random.default_rng(1).standard_normal((n.size, B)))
    g = torch.ones((P, B), dtype=torch.float64, device="cuda")
    f = zp.series_forward(n, m, r, th, c)
    assert torch.equal(f, f[:1].expand_as(f))
    _, _, gt = zp.series_backward(n, m, r, th, c, g)
    assert torch.all(gt == 0)


def test_deterministic(zp):
    wl = W.series_n40(npts=4096, nb=64)
    for prec in ("fp64", "bf16x3"):
        a = _gpu_all(zp, wl, prec)
        b = _gpu_all(zp, wl, prec)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


@pytest.fixture(scope="module")
def n64_ref(oracle_mod):
    """The full n <= 64 mixed-precision workload (2145 modes, 65536 points,
    1024 sets), with the oracle evaluated on samples: f on 384 points (all
    sets), grad_c on 48 sets (all modes; needs the oracle basis at every
    point), grad_r and grad_theta on the same 384 points."""
    wl = W.series_n64()
    rng = np.random.default_rng(99)
    ps = np.sort(rng.choice(wl.P, 384, replace=False))
    bs = np.sort(rng.choice(wl.B, 48, replace=False))
    _say(f"[oracle] series_n64 basis at all {wl.P} points (Z only)")
    Z = oracle_mod.basis(wl.n, wl.m, wl.r, wl.theta, 1)[0]
    gc_ref = Z @ wl.g[:, bs]
    del Z
    Zs, Zrs, Zts = oracle_mod.series_basis(wl.n, wl.m, wl.r[ps], wl.theta[ps])
    f_ref = Zs.T @ wl.c
    gr_ref = np.einsum("pb,pb->p", wl.g[ps], Zrs.T @ wl.c)
    gt_ref = np.einsum("pb,pb->p", wl.g[ps], Zts.T @ wl.c)
    return wl, ps, bs, (f_ref, gc_ref, gr_ref, gt_ref)


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "fp64"])
def test_series_n64_mixed_full_size_sampled(zp, n64_ref, prec):
    wl, ps, bs, ref = n64_ref
    _say(f"[series] n64 full size {prec}")
    f, gc, gr, gt = _gpu_all(zp, wl, prec)
    got = (f[ps], gc[:, bs], gr[ps], gt[ps])
    tol = TOL[prec]
    for name, a, b in zip(("f", "grad_c", "grad_r", "grad_theta"), got, ref):
        e = _rel(a, b)
        _say(f"  {prec} {name}: rel err {e:.3g} (sampled)")
        assert e <= tol, (prec, name, e)


def test_bad_arguments_raise(zp):
    n, m = W.ansi_modes(3)
    r = _dev(np.linspace(0, 1, 5))
    c = _dev(np.ones((n.size, 2)))
    with pytest.raises(ValueError):
        zp.series_forward(n, m, r, r, c, "fp16")
    with pytest.raises(zp.ZpError):
        zp.series_forward(n, m, r, r, c, 7)
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(zp.ZpError):
        zp.series_forward(n, m, r, r, c, "fp64", ws=ws)


# ------------------------------------------------------- forward mode (JVP) --

def _jvp_case(seed=5, nmax=40, P=3000, B=24):
    rng = np.random.default_rng(seed)
    n, m = W.ansi_modes(nmax)
    r, th = np.sqrt(rng.random(P)), 2 * np.pi * rng.random(P)
    c = rng.standard_normal((n.size, B)) / (n + 1.0)[:, None]
    tc = rng.standard_normal((n.size, B))
    tr, tt = rng.standard_normal(P), rng.standard_normal(P)
    return n, m, r, th, c, tc, tr, tt


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_jvp_matches_oracle(zp, oracle_mod, prec):
    """tf = Z^T tc + (tr dZ/dr + ttheta dZ/dtheta)^T c against the oracle basis."""
    n, m, r, th, c, tc, tr, tt = _jvp_case()
    Z, Zr, Zt = oracle_mod.series_basis(n, m, r, th)
    ref = Z.T @ tc + tr[:, None] * (Zr.T @ c) + tt[:, None] * (Zt.T @ c)
    got = zp.series_jvp(n, m, _dev(r), _dev(th), _dev(c), _dev(tc), _dev(tr), _dev(tt), prec).cpu().numpy()
    e = _rel(got, ref)
    _say(f"  jvp {prec}: rel err {e:.3g}")
    assert e <= TOL[prec]


def test_jvp_partial_tangents(zp, oracle_mod):
    n, m, r, th, c, tc, tr, tt = _jvp_case(seed=6, nmax=20, P=700, B=5)
    Z, Zr, Zt = oracle_mod.series_basis(n, m, r, th)
    d = {k: _dev(v) for k, v in dict(r=r, th=th, c=c, tc=tc, tr=tr, tt=tt).items()}
    cases = [
        (dict(tc=d["tc"]), Z.T @ tc),
        (dict(tr=d["tr"]), tr[:, None] * (Zr.T @ c)),
        (dict(ttheta=d["tt"]), tt[:, None] * (Zt.T @ c)),
        (dict(tc=d["tc"], ttheta=d["tt"]), Z.T @ tc + tt[:, None] * (Zt.T @ c)),
    ]
    for prec in ("fp64", "bf16x3"):
        for kw, ref in cases:
            got = zp.series_jvp(n, m, d["r"], d["th"], d["c"], prec=prec, **kw).cpu().numpy()
            assert _rel(got, ref) <= TOL[prec], (prec, list(kw))
    zero = zp.series_jvp(n, m, d["r"], d["th"], d["c"]).cpu().numpy()
    assert np.all(zero == 0)


def test_jvp_vjp_duality(zp):
    """<g, J v> = <J^T g, v> between the forward-mode and reverse-mode kernels."""
    n, m, r, th, c, tc, tr, tt = _jvp_case(seed=7, nmax=30, P=2000, B=16)
    g = np.random.default_rng(8).standard_normal((r.size, c.shape[1]))
    tf = zp.series_jvp(n, m, _dev(r), _dev(th), _dev(c), _dev(tc), _dev(tr), _dev(tt)).cpu().numpy()
    gc, gr, gt = (x.cpu().numpy() for x in zp.series_backward(n, m, _dev(r), _dev(th), _dev(c), _dev(g)))
    lhs = np.sum(g * tf)
    rhs = np.sum(gc * tc) + np.sum(gr * tr) + np.sum(gt * tt)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs))


def test_forward_mode_autograd(zp):
    """torch forward-mode AD through ZernikeSeries, and gradcheck of both modes."""
    import torch.autograd.forward_ad as fwAD

    n, m, r, th, c, tc, tr, tt = _jvp_case(seed=9, nmax=12, P=50, B=3)
    with fwAD.dual_level():
        f = zp.series(fwAD.make_dual(_dev(c), _dev(tc)), fwAD.make_dual(_dev(r), _dev(tr)),
                      fwAD.make_dual(_dev(th), _dev(tt)), n, m)
        tangent = fwAD.unpack_dual(f).tangent
    ref = zp.series_jvp(n, m, _dev(r), _dev(th), _dev(c), _dev(tc), _dev(tr), _dev(tt))
    assert torch.equal(tangent, ref)
    n2, m2 = W.ansi_modes(5)
    rng = np.random.default_rng(10)
    rr = _dev(0.1 + 0.8 * rng.random(6)).requires_grad_()
    tt2 = _dev(2 * np.pi * rng.random(6)).requires_grad_()
    cc = _dev(rng.standard_normal((n2.size, 2))).requires_grad_()
    assert torch.autograd.gradcheck(lambda c_, r_, t_: zp.series(c_, r_, t_, n2, m2), (cc, rr, tt2), eps=1e-6,
                                    atol=1e-8, rtol=1e-6, check_forward_ad=True)


def test_jvp_n64_full_size_sampled(zp, n64_ref, oracle_mod):
    """The n <= 64 workload's forward-mode derivative, sampled rows, per precision."""
    wl, ps, _, _ = n64_ref
    rng = np.random.default_rng(77)
    tc = rng.standard_normal(wl.c.shape) / (wl.n + 1.0)[:, None]
    tr, tt = rng.standard_normal(wl.P), rng.standard_normal(wl.P)
    Zs, Zrs, Zts = oracle_mod.series_basis(wl.n, wl.m, wl.r[ps], wl.theta[ps])
    ref = Zs.T @ tc + tr[ps, None] * (Zrs.T @ wl.c) + tt[ps, None] * (Zts.T @ wl.c)
    for prec in ("bf16x3", "fp32", "fp64"):
        got = zp.series_jvp(wl.n, wl.m, _dev(wl.r), _dev(wl.theta), _dev(wl.c), _dev(tc), _dev(tr), _dev(tt),
                            prec).cpu().numpy()[ps]
        e = _rel(got, ref)
        _say(f"  jvp n64 {prec}: rel err {e:.3g} (sampled)")
        assert e <= TOL[prec]
