"""zp_series_fwd_noalloc (the series forward whose workspace and plan tables
live in the library's fixed per-GPU array) against zp_series_fwd with a
caller workspace, through the C ABI.

Both compute every output element with the same sums in the same order (the
chunking of the points differs, which does not change any element's
arithmetic), so the outputs must be identical.  Two calls in a row on
different mode lists, the second smaller; then the second list again (its
tables already in place) on other points; and a size beyond the array.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PRECS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
ERR_WS = 4


def _case(nmax, P, B, seed):
    import zp_workloads as W

    n, m = W.ansi_modes(nmax)
    rng = np.random.default_rng(seed)
    r = np.concatenate([[0.0, 1.0], np.sqrt(rng.random(P - 2))])
    th = 2 * np.pi * rng.random(P)
    c = rng.standard_normal((n.size, B)) / (n + 1.0)[:, None]
    return n.astype(np.int32), m.astype(np.int32), r, th, c


def _run_both(lib, n, m, r, th, c, prec):
    import torch

    import paper_2409_19156_amd as zp

    dev = torch.device("cuda:0")
    M, P, B = n.size, r.size, c.shape[1]
    td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    rd, thd, cd = td(r), td(th), td(c)
    f_ref = torch.full((P, B), np.nan, dtype=torch.float64, device=dev)
    f_new = torch.full((P, B), np.nan, dtype=torch.float64, device=dev)
    full, _, _ = zp.series_sizes(M, P, B, prec)
    ws = torch.empty(full, dtype=torch.uint8, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    st = lib.zp_series_fwd(n.ctypes.data, m.ctypes.data, M, rd.data_ptr(), thd.data_ptr(), P, cd.data_ptr(), B,
                           PRECS[prec], f_ref.data_ptr(), None, ws.data_ptr(), ws.numel(), stream)
    assert st == 0, lib.zp_last_error()
    st = lib.zp_series_fwd_noalloc(n.ctypes.data, m.ctypes.data, M, rd.data_ptr(), thd.data_ptr(), P, cd.data_ptr(),
                                   B, PRECS[prec], f_new.data_ptr(), stream)
    assert st == 0, lib.zp_last_error()
    torch.cuda.synchronize()
    return f_ref.cpu().numpy(), f_new.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_noalloc_matches_workspace_forward(prec):
    from paper_2409_19156_amd import _lib

    lib = _lib.load()
    # 1: n <= 64 (2145 modes), 9000 points x 64 sets: several chunks of the array
    # 2: a smaller, different mode list and size (new tables)
    # 3: the second list again on other points (tables reused)
    for step, (nmax, P, B, seed) in enumerate([(64, 9000, 64, 1), (12, 333, 5, 2), (12, 700, 3, 3)]):
        n, m, r, th, c = _case(nmax, P, B, seed)
        print(f"noalloc {prec} call {step + 1}: n <= {nmax}, M {n.size}, P {P}, B {B}", flush=True)
        ref, got = _run_both(lib, n, m, r, th, c, prec)
        assert np.all(np.isfinite(ref))
        assert np.array_equal(got, ref), f"call {step + 1}: max |diff| {np.abs(got - ref).max():.3g}"


def test_noalloc_rejects_size_beyond_array():
    import torch

    from paper_2409_19156_amd import _lib

    lib = _lib.load()
    n, m, r, th, _ = _case(64, 256, 1, 4)
    B = 4096  # the coefficient buffer alone, 8 * 2176 * 4096 bytes, exceeds 64 MiB
    dev = torch.device("cuda:0")
    rd = torch.from_numpy(r).to(dev)
    thd = torch.from_numpy(th).to(dev)
    cd = torch.zeros((n.size, B), dtype=torch.float64, device=dev)
    f = torch.full((r.size, B), 7.0, dtype=torch.float64, device=dev)
    st = lib.zp_series_fwd_noalloc(n.ctypes.data, m.ctypes.data, n.size, rd.data_ptr(), thd.data_ptr(), r.size,
                                   cd.data_ptr(), B, 0, f.data_ptr(), None)
    assert st == ERR_WS
    assert b"exceed the fixed scratch" in lib.zp_last_error()
    torch.cuda.synchronize()
    assert bool((f == 7.0).all()), "nothing may be written on error"
