"""Every entry of the n <= 200 stress workload against the oracle.

10 201 radial pairs x 100 000 clustered points x orders 0..2 = 3.06e9 values
from one launch over all points (the launch the benchmark times), compared in
chunks of 5000 points, each against 1e-13 (n+1)^(2j) per (mode, order).  The
quad-precision oracle needs about two minutes of host time (all threads) for
the whole set.
"""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest
import torch

import zp_workloads as W
from tests.gpu_util import radial_tol

pytestmark = pytest.mark.gpu

CHUNK = 5000


def test_radial_n200_every_point(oracle_mod):
    import paper_2409_19156_amd as zp

    wl = W.radial_n200()
    J = wl.max_dr
    print(f"[full sweep] {wl.name}: M={wl.M} P={wl.P} J={J}, one launch", flush=True)
    out = zp.radial(wl.n, wl.m, torch.from_numpy(wl.r).cuda(), J)  # [J+1, M, P]
    torch.cuda.synchronize()
    tol = np.stack([radial_tol(wl.n, j) for j in range(J + 1)])  # [J+1, M]
    worst = np.zeros((J + 1, wl.M))
    t0 = time.perf_counter()
    for c0 in range(0, wl.P, CHUNK):
        r = wl.r[c0:c0 + CHUNK]
        got = out[:, :, c0:c0 + r.size].cpu().numpy()
        ref = oracle_mod.radial(wl.n, wl.m, r, J)
        assert np.all(np.isfinite(got))
        worst = np.maximum(worst, np.abs(got - ref).max(axis=2) / tol)
        print(f"points {c0}..{c0 + r.size - 1}: worst so far {worst.max():.4f} x tol "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
        sys.stdout.flush()
    del out
    torch.cuda.empty_cache()
    for j in range(J + 1):
        k = int(np.argmax(worst[j]))
        print(f"order {j}: worst {worst[j, k]:.4f} x tol at (n, m) = ({wl.n[k]}, {wl.m[k]})", flush=True)
    assert worst.max() <= 1.0
