"""The stored oracle samples of the timed series workloads (written by
tests/golden/make_series_refs.py, read by the benchmark's error report) match
the current input generators and the oracle."""
from __future__ import annotations

import os

import numpy as np
import pytest

import zp_workloads as W
from tests.golden import make_series_refs as G

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name,make", [("series_n64_oracle_sample.npz", W.series_n64),
                                       ("series_n40_oracle_sample.npz", W.series_n40)])
def test_stored_sample_matches_workload(name, make):
    d = np.load(os.path.join(HERE, name), allow_pickle=False)
    assert str(d["digest"]) == G.workload_digest(make())


def test_stored_n40_sample_matches_oracle(oracle_mod):
    wl = W.series_n40()
    d = np.load(os.path.join(HERE, "series_n40_oracle_sample.npz"), allow_pickle=False)
    ps, bs_f = d["ps"], d["bs_f"]
    Z, Zr, Zt = oracle_mod.series_basis(wl.n, wl.m, wl.r[ps], wl.theta[ps])
    f = oracle_mod.series_fwd(Z, wl.c[:, bs_f])
    _, gr, gt = oracle_mod.series_bwd(Z, Zr, Zt, wl.c, wl.g[ps])
    for a, b in ((f, d["f"]), (gr, d["grad_r"]), (gt, d["grad_theta"])):
        assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()
