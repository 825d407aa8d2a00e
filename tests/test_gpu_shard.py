"""Per-point outputs do not depend on the other points.

A series forward and backward over a leading subset of the points (the share
one GPU would hold when the points are split across GPUs) must give exactly
the rows of the full run for f, dL/dr and dL/dtheta: each of those rows sums
over modes and sets only, in an order that the number of points, the chunking
of the points and the tile shape chosen for the problem size do not change.
dL/dc sums over the points and is that GPU's partial sum, checked against the
full run's dL/dc minus the rest of the points' contribution within rounding.
The n <= 40 workload with 256 sets is used in full (16 384 points, the narrow
FP64 backward tiles and the two-stream backward) and on 2048 and 8192 points.
"""
from __future__ import annotations

import pytest
import torch

import zp_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zp():
    import paper_2409_19156_amd as zp

    assert torch.cuda.is_available()
    return zp


@pytest.fixture(scope="module")
def wl():
    return W.series_n40()


def _fwd_bwd(zp, wl, ps, q0, prec):
    dev = torch.device("cuda:0")
    r = torch.from_numpy(wl.r[q0:q0 + ps]).to(dev)
    th = torch.from_numpy(wl.theta[q0:q0 + ps]).to(dev)
    c = torch.from_numpy(wl.c).to(dev)
    g = torch.from_numpy(wl.g[q0:q0 + ps]).to(dev)
    f = zp.series_forward(wl.n, wl.m, r, th, c, prec)
    gc, gr, gt = zp.series_backward(wl.n, wl.m, r, th, c, g, prec)
    torch.cuda.synchronize()
    return f, gc, gr, gt


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_subset_rows_equal_full_run(zp, wl, prec):
    print(f"shard parity: n<=40, {wl.P} points, {wl.B} sets, {prec}", flush=True)
    f, gc, gr, gt = _fwd_bwd(zp, wl, wl.P, 0, prec)
    for ps in (2048, 8192):
        fs, gcs, grs, gts = _fwd_bwd(zp, wl, ps, 0, prec)
        assert torch.equal(fs, f[:ps]), f"{prec}, {ps} points: f rows differ"
        assert torch.equal(grs, gr[:ps]), f"{prec}, {ps} points: dL/dr rows differ"
        assert torch.equal(gts, gt[:ps]), f"{prec}, {ps} points: dL/dtheta rows differ"
        # dL/dc over the subset plus over the remaining points is the full dL/dc
        _, gcr, _, _ = _fwd_bwd(zp, wl, wl.P - ps, ps, prec)
        scale = gc.abs().max().item()
        err = (gcs + gcr - gc).abs().max().item() / scale
        tol = 1e-13 if prec == "fp64" else 5e-7
        assert err <= tol, f"{prec}, {ps} points: partial dL/dc sums off by {err:.2e}"
