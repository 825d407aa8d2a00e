"""The series backward computes only the outputs asked for, bit for bit.

Leaving out dL/dc (no split-K contraction; bf16 converts the upstream
gradient for the column-dot alone) or dL/dr and dL/dtheta (no column-dot, no
second stream) must not change the outputs that are computed: each subset of
(dL/dc, dL/dr, dL/dtheta) equals the corresponding outputs of the full call,
in all three precisions, with and without the basis cache.
"""
from __future__ import annotations

import itertools

import pytest
import torch

import zp_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zp():
    import paper_2409_19156_amd as zp

    assert torch.cuda.is_available()
    return zp


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("cached", [False, True])
def test_output_subsets_match_full_backward(zp, prec, cached):
    print(f"partial outputs: n<=24, 3000 points, 40 sets, {prec}, cache={cached}", flush=True)
    n, m = W.ansi_modes(24)
    r, th = W.disc_points(7, 3000)
    dev = torch.device("cuda:0")
    rd, td = torch.from_numpy(r).to(dev), torch.from_numpy(th).to(dev)
    gen = torch.Generator().manual_seed(7)
    c = torch.randn(len(n), 40, generator=gen, dtype=torch.float64).to(dev)
    g = torch.randn(r.size, 40, generator=gen, dtype=torch.float64).to(dev)
    cache = None
    if cached:
        _, _, cb = zp.series_sizes(len(n), r.size, 40, prec)
        cache = torch.empty(cb, dtype=torch.uint8, device=dev)
        zp.series_forward(n, m, rd, td, c, prec, cache=cache)
    full = zp.series_backward(n, m, rd, td, c, g, prec, cache=cache)
    for need in itertools.product((False, True), repeat=3):
        if not any(need) or all(need):
            continue
        part = zp.series_backward(n, m, rd, td, c, g, prec, cache=cache, need=need)
        for name, want, f, p in zip(("dL/dc", "dL/dr", "dL/dtheta"), need, full, part):
            if want:
                assert torch.equal(p, f), f"{prec}, need={need}: {name} differs from the full call"
            else:
                assert p is None
