"""The library runs on the caller's stream and does not block the host.

Each entry point is asynchronous on the stream it is given (torch's current
stream in the binding).  Queued behind a ~0.1 s spin on a side stream, a call
must return at once, leave that stream busy, and after the stream finishes its
output must equal the result computed on the default stream.  (Whether the
output is still untouched while the spin runs cannot be observed from a second
stream here: HIP multiplexes streams onto a few hardware queues, and a second
stream may share the side stream's queue and wait behind it.)
"""
from __future__ import annotations

import time

import numpy as np
import pytest
import torch

import zp_workloads as W

pytestmark = pytest.mark.gpu

SPIN_CYCLES = 200_000_000  # about 0.1 s of GPU clock


@pytest.fixture(scope="module")
def zp():
    import paper_2409_19156_amd as zp

    assert torch.cuda.is_available()
    return zp


def _queued_behind_spin(fn, out):
    """Run fn() on a side stream behind a spin kernel; return (host seconds of
    the call, whether the stream was still busy right after it)."""
    if not hasattr(torch.cuda, "_sleep"):
        pytest.skip("torch.cuda._sleep is not available in this torch build")
    side = torch.cuda.Stream()
    out.fill_(float("nan"))
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        torch.cuda._sleep(SPIN_CYCLES)
        t0 = time.perf_counter()
        fn()
        dt = time.perf_counter() - t0
    busy = not side.query()
    side.synchronize()
    return dt, busy


def test_basis_on_caller_stream(zp):
    n, m = W.ansi_modes(30)
    r, th = W.disc_points(1, 4000)
    rd, td = torch.from_numpy(r).cuda(), torch.from_numpy(th).cuda()
    ref = zp.basis(n, m, rd, td, 31)  # default stream; also builds the plan
    out = torch.empty_like(ref)
    dt, busy = _queued_behind_spin(lambda: zp.basis(n, m, rd, td, 31, out=out), out)
    assert busy, "the spin finished before the check; lengthen it"
    assert dt < 0.05, f"the call blocked the host for {dt:.3f} s"
    assert torch.equal(out, ref)


def test_series_on_caller_stream(zp):
    wl = W.series_n40(npts=2048, nb=16)
    r, th, c = (torch.from_numpy(x).cuda() for x in (wl.r, wl.theta, wl.c))
    full, _, _ = zp.series_sizes(wl.M, wl.P, wl.B, "bf16x3")
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    ref = zp.series_forward(wl.n, wl.m, r, th, c, "bf16x3", ws=ws)
    torch.cuda.synchronize()
    out = torch.empty_like(ref)

    def call():
        out.copy_(zp.series_forward(wl.n, wl.m, r, th, c, "bf16x3", ws=ws))

    dt, busy = _queued_behind_spin(call, out)
    assert busy
    assert dt < 0.05, f"the call blocked the host for {dt:.3f} s"
    assert torch.equal(out, ref)


def test_pipelined_series_on_caller_stream(zp):
    """A forward and a forward-mode derivative large enough to run their chunks
    on the library's helper stream (20001 points x 1024 sets) stay ordered on
    the caller's stream: queued behind the spin they return at once, and once
    the caller's stream has finished their outputs are complete."""
    n, m = W.ansi_modes(20)
    r, th = W.disc_points(3, 20001)
    rng = np.random.default_rng(4)
    rd, td = torch.from_numpy(r).cuda(), torch.from_numpy(th).cuda()
    c = torch.from_numpy(rng.standard_normal((n.size, 1024))).cuda()
    tr = torch.from_numpy(rng.standard_normal(r.size)).cuda()
    for prec in ("fp64", "bf16x3"):
        ref = zp.series_forward(n, m, rd, td, c, prec)
        ref_t = zp.series_jvp(n, m, rd, td, c, c, tr, None, prec=prec)
        torch.cuda.synchronize()
        out = torch.empty_like(ref)
        out_t = torch.empty_like(ref_t)

        def call():
            out.copy_(zp.series_forward(n, m, rd, td, c, prec))
            out_t.copy_(zp.series_jvp(n, m, rd, td, c, c, tr, None, prec=prec))

        out_t.fill_(float("nan"))
        dt, busy = _queued_behind_spin(call, out)
        assert busy
        assert dt < 0.05, f"the call blocked the host for {dt:.3f} s"
        assert torch.equal(out, ref), prec
        assert torch.equal(out_t, ref_t), prec


def test_two_streams_concurrently(zp):
    """Two independent problems on two streams at once (shared plan cache):
    each equals its default-stream result."""
    n1, m1 = W.ansi_modes(25)
    n2, m2 = W.radial_pairs(40)
    r, th = W.disc_points(2, 3000)
    rd, td = torch.from_numpy(r).cuda(), torch.from_numpy(th).cuda()
    ref1 = zp.basis(n1, m1, rd, td, 3)
    ref2 = zp.radial(n2, m2, rd, 2)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for _ in range(5):
        with torch.cuda.stream(s1):
            a = zp.basis(n1, m1, rd, td, 3)
        with torch.cuda.stream(s2):
            b = zp.radial(n2, m2, rd, 2)
        outs.append((a, b))
    torch.cuda.synchronize()
    for a, b in outs:
        assert torch.equal(a, ref1) and torch.equal(b, ref2)
