"""The C ABI (include/zp.h) on the CPU: the library loads, exports every
declared symbol, and rejects bad arguments on the host before any HIP call.

No test here launches device work: error paths return before the first HIP
call, and empty problems (M, P or B zero) are no-ops.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2409_19156_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

OK, ERR_MODE, ERR_ARG, ERR_ORDER, ERR_WS, ERR_HIP, ERR_PREC = range(7)
FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: every call below fails validation first


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _declared():
    text = open(os.path.join(ROOT, "include", "zp.h")).read()
    return sorted(set(re.findall(r"\b(zp_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert set(declared) == set(_lib.EXPORTS), declared
    for name in declared:
        assert hasattr(lib, name), name


def test_abi_version_and_status_strings(lib):
    assert lib.zp_abi_version() == 1
    for code in range(7):
        assert lib.zp_status_string(code)
    assert b"unknown" in lib.zp_status_string(99)


def _modes(n, m):
    n = np.ascontiguousarray(n, dtype=np.int32)
    m = np.ascontiguousarray(m, dtype=np.int32)
    return n, m


@pytest.mark.parametrize("n,m", [([-1], [0]), ([3], [0]), ([2], [4]), ([5], [-6]), ([1001], [1]), ([4, 7], [0, 2])])
def test_invalid_modes(lib, n, m):
    n, m = _modes(n, m)
    assert lib.zp_radial(n.ctypes.data, m.ctypes.data, n.size, FAKE, 4, 0, FAKE, None) == ERR_MODE
    assert b"violates" in lib.zp_last_error()
    assert lib.zp_radial_direct(n.ctypes.data, m.ctypes.data, n.size, FAKE, 4, 0, FAKE, None) == ERR_MODE
    assert lib.zp_radial_zernike_recursion(n.ctypes.data, m.ctypes.data, n.size, FAKE, 4, 0, FAKE, None) == ERR_MODE
    assert lib.zp_basis(n.ctypes.data, m.ctypes.data, n.size, FAKE, FAKE, 4, 1, FAKE, None) == ERR_MODE
    assert lib.zp_basis_polar(n.ctypes.data, m.ctypes.data, n.size, FAKE, 2, FAKE, 2, 1, FAKE, None) == ERR_MODE
    assert lib.zp_series_fwd(n.ctypes.data, m.ctypes.data, n.size, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, None, FAKE,
                             1 << 20, None) == ERR_MODE
    assert lib.zp_series_bwd(n.ctypes.data, m.ctypes.data, n.size, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, None, FAKE,
                             FAKE, FAKE, FAKE, 1 << 20, None) == ERR_MODE
    assert lib.zp_series_jvp(n.ctypes.data, m.ctypes.data, n.size, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, FAKE, FAKE,
                             FAKE, FAKE, 1 << 20, None) == ERR_MODE
    assert lib.zp_series_fwd_noalloc(n.ctypes.data, m.ctypes.data, n.size, FAKE, FAKE, 4, FAKE, 2, 0, FAKE,
                                     None) == ERR_MODE


def test_order_mask_prec_and_sizes(lib):
    n, m = _modes([2, 3], [0, -1])
    nd, md = n.ctypes.data, m.ctypes.data
    for bad in (-1, 4, 7):
        assert lib.zp_radial(nd, md, 2, FAKE, 4, bad, FAKE, None) == ERR_ORDER
        assert lib.zp_radial_direct(nd, md, 2, FAKE, 4, bad, FAKE, None) == ERR_ORDER
        assert lib.zp_radial_zernike_recursion(nd, md, 2, FAKE, 4, bad, FAKE, None) == ERR_ORDER
    big, bm = _modes([61, 2], [1, 0])
    assert lib.zp_radial_zernike_recursion(big.ctypes.data, bm.ctypes.data, 2, FAKE, 4, 0, FAKE, None) == ERR_ARG
    assert b"n <= 60" in lib.zp_last_error()
    for mask in (0, 32, 33):
        assert lib.zp_basis(nd, md, 2, FAKE, FAKE, 4, mask, FAKE, None) == ERR_ARG
    assert lib.zp_radial(nd, md, -1, FAKE, 4, 0, FAKE, None) == ERR_ARG
    assert lib.zp_radial(nd, md, 2, FAKE, -4, 0, FAKE, None) == ERR_ARG
    assert lib.zp_radial(nd, md, 2, None, 4, 0, FAKE, None) == ERR_ARG
    assert lib.zp_radial(nd, md, 2, FAKE, 4, 0, None, None) == ERR_ARG
    assert lib.zp_radial(None, md, 2, FAKE, 4, 0, FAKE, None) == ERR_ARG
    assert lib.zp_basis(nd, md, 2, FAKE, None, 4, 1, FAKE, None) == ERR_ARG
    # polar grids: sizes, mask and pointers are checked first
    assert lib.zp_basis_polar(nd, md, 2, FAKE, -1, FAKE, 4, 1, FAKE, None) == ERR_ARG
    assert lib.zp_basis_polar(nd, md, 2, FAKE, 3, FAKE, -4, 1, FAKE, None) == ERR_ARG
    assert lib.zp_basis_polar(nd, md, 2, FAKE, 1 << 40, FAKE, 1 << 40, 1, FAKE, None) == ERR_ARG
    assert lib.zp_basis_polar(nd, md, 2, FAKE, 3, FAKE, 4, 0, FAKE, None) == ERR_ARG
    assert lib.zp_basis_polar(nd, md, 2, FAKE, 3, None, 4, 1, FAKE, None) == ERR_ARG
    assert lib.zp_basis_polar(nd, md, 2, FAKE, 3, FAKE, 4, 1, None, None) == ERR_ARG
    assert lib.zp_basis_polar(nd, md, 2, None, 0, None, 4, 31, None, None) == OK
    for prec in (-1, 3):
        assert lib.zp_series_fwd(nd, md, 2, FAKE, FAKE, 4, FAKE, 2, prec, FAKE, None, FAKE, 1 << 20, None) == ERR_PREC
    assert lib.zp_series_fwd(nd, md, 2, FAKE, FAKE, -4, FAKE, 2, 0, FAKE, None, FAKE, 1 << 20, None) == ERR_ARG
    assert lib.zp_series_fwd(nd, md, 2, FAKE, FAKE, 4, FAKE, -2, 0, FAKE, None, FAKE, 1 << 20, None) == ERR_ARG
    # the allocation-free forward: precision, sizes and null pointers are checked first
    for prec in (-1, 3):
        assert lib.zp_series_fwd_noalloc(nd, md, 2, FAKE, FAKE, 4, FAKE, 2, prec, FAKE, None) == ERR_PREC
    assert lib.zp_series_fwd_noalloc(nd, md, 2, FAKE, FAKE, -4, FAKE, 2, 0, FAKE, None) == ERR_ARG
    assert lib.zp_series_fwd_noalloc(nd, md, 2, FAKE, FAKE, 4, FAKE, -2, 0, FAKE, None) == ERR_ARG
    for i in (3, 4, 6, 9):
        args = [nd, md, 2, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, None]
        args[i] = None
        assert lib.zp_series_fwd_noalloc(*args) == ERR_ARG
    # workspace: null / misaligned / too small (all host-side)
    assert lib.zp_series_fwd(nd, md, 2, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, None, None, 1 << 20, None) == ERR_ARG
    assert lib.zp_series_fwd(nd, md, 2, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, None, ctypes.c_void_p(0x10008), 1 << 20,
                             None) == ERR_ARG
    assert lib.zp_series_fwd(nd, md, 2, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, None, FAKE, 16, None) == ERR_WS
    assert lib.zp_series_bwd(nd, md, 2, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, None, FAKE, FAKE, FAKE, FAKE, 16,
                             None) == ERR_WS
    # forward mode: bad precision, null output, point tangent without c, small workspace
    assert lib.zp_series_jvp(nd, md, 2, FAKE, FAKE, 4, FAKE, 2, 5, FAKE, None, None, FAKE, FAKE, 1 << 20,
                             None) == ERR_PREC
    assert lib.zp_series_jvp(nd, md, 2, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, None, None, None, FAKE, 1 << 20,
                             None) == ERR_ARG
    assert lib.zp_series_jvp(nd, md, 2, FAKE, FAKE, 4, None, 2, 0, None, FAKE, None, FAKE, FAKE, 1 << 20,
                             None) == ERR_ARG
    assert lib.zp_series_jvp(nd, md, 2, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, None, None, FAKE, FAKE, 16,
                             None) == ERR_WS


def test_stream_fill_arguments(lib):
    assert lib.zp_stream_fill(FAKE, -1, 0.0, 1, None) == ERR_ARG
    assert lib.zp_stream_fill(None, 8, 0.0, 1, None) == ERR_ARG
    assert lib.zp_stream_fill(ctypes.c_void_p(0x10008), 8, 0.0, 0, None) == ERR_ARG
    assert lib.zp_stream_fill(None, 0, 0.0, 1, None) == OK


def test_empty_problems_are_noops(lib):
    n, m = _modes([2], [0])
    e = np.zeros(0, dtype=np.int32)
    assert lib.zp_radial(e.ctypes.data, e.ctypes.data, 0, FAKE, 4, 3, FAKE, None) == OK
    assert lib.zp_radial(n.ctypes.data, m.ctypes.data, 1, None, 0, 3, None, None) == OK
    assert lib.zp_basis(n.ctypes.data, m.ctypes.data, 1, None, None, 0, 31, None, None) == OK
    assert lib.zp_series_fwd(n.ctypes.data, m.ctypes.data, 1, FAKE, FAKE, 4, FAKE, 0, 0, FAKE, None, FAKE, 0,
                             None) == OK
    assert lib.zp_series_fwd_noalloc(n.ctypes.data, m.ctypes.data, 1, FAKE, FAKE, 4, FAKE, 0, 0, FAKE, None) == OK
    assert lib.zp_series_fwd_noalloc(e.ctypes.data, e.ctypes.data, 0, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, None) == OK


def test_size_queries(lib):
    full, mn, cb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    for prec in (0, 1, 2):
        assert lib.zp_series_workspace(2145, 65536, 1024, prec, ctypes.byref(full), ctypes.byref(mn)) == OK
        assert 0 < mn.value <= full.value
        assert full.value % 256 == 0 and mn.value % 256 == 0
        assert lib.zp_series_cache_bytes(2145, 65536, prec, ctypes.byref(cb)) == OK
        # at least Z (FP64, or FP32 for the FP32 and bf16 contractions) plus two derivative planes
        per = {0: 8 + 16, 1: 4 + 8, 2: 4 + 8}[prec]
        assert cb.value >= 2145 * 65536 * per
    assert lib.zp_series_workspace(-1, 4, 4, 0, ctypes.byref(full), None) == ERR_ARG
    assert lib.zp_series_workspace(4, 4, 4, 9, ctypes.byref(full), None) == ERR_PREC
    assert lib.zp_series_cache_bytes(4, 4, 0, None) == ERR_ARG


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    """The Python binding has no fallback: a missing libzp.so is an error."""
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load()


def test_series3d_validation(lib):
    n, m = _modes([2, 3, 2], [0, -1, 0])
    l = np.ascontiguousarray([0, 1, -1], dtype=np.int32)
    nd, md, ld = n.ctypes.data, m.ctypes.data, l.ctypes.data
    full, mn, cb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.zp_series3d_workspace(nd, md, ld, 3, 100, 8, 2, 0, ctypes.byref(full), ctypes.byref(mn)) == OK
    assert 0 < mn.value <= full.value and full.value % 256 == 0
    # two distinct (n, m) pairs: the cache is the planar cache of those two
    ref = ctypes.c_size_t()
    assert lib.zp_series3d_cache_bytes(nd, md, ld, 3, 100, 0, ctypes.byref(cb)) == OK
    assert lib.zp_series_cache_bytes(2, 100, 0, ctypes.byref(ref)) == OK and cb.value == ref.value
    bad_l = np.ascontiguousarray([0, 1, 1048577], dtype=np.int32)
    args = (FAKE, FAKE, 4, FAKE, 2, FAKE, 2)
    assert lib.zp_series3d_fwd(nd, md, bad_l.ctypes.data, 3, *args, 0, FAKE, None, FAKE, 1 << 20, None) == ERR_MODE
    assert b"ZP_L_MAX" in lib.zp_last_error()
    bad_n, _ = _modes([2, 4, 2], [0, -1, 0])
    assert lib.zp_series3d_fwd(bad_n.ctypes.data, md, ld, 3, *args, 0, FAKE, None, FAKE, 1 << 20, None) == ERR_MODE
    assert lib.zp_series3d_bwd(bad_n.ctypes.data, md, ld, 3, *args, 0, FAKE, None, FAKE, FAKE, FAKE, FAKE, FAKE,
                               1 << 20, None) == ERR_MODE
    assert lib.zp_series3d_fwd(nd, md, None, 3, *args, 0, FAKE, None, FAKE, 1 << 20, None) == ERR_ARG
    assert lib.zp_series3d_fwd(nd, md, ld, 3, *args, 7, FAKE, None, FAKE, 1 << 20, None) == ERR_PREC
    assert lib.zp_series3d_fwd(nd, md, ld, 3, FAKE, FAKE, 4, None, 2, FAKE, 2, 0, FAKE, None, FAKE, 1 << 20,
                               None) == ERR_ARG
    assert lib.zp_series3d_fwd(nd, md, ld, 3, *args, 0, FAKE, None, FAKE, 16, None) == ERR_WS
    assert lib.zp_series3d_fwd(nd, md, ld, 3, FAKE, FAKE, 4, FAKE, -2, FAKE, 2, 0, FAKE, None, FAKE, 1 << 20,
                               None) == ERR_ARG
    # empty problems are no-ops
    assert lib.zp_series3d_fwd(nd, md, ld, 3, FAKE, FAKE, 4, FAKE, 0, FAKE, 2, 0, FAKE, None, FAKE, 0, None) == OK
    assert lib.zp_series3d_fwd(nd, md, ld, 0, FAKE, FAKE, 4, FAKE, 2, FAKE, 2, 0, FAKE, None, FAKE, 0, None) == OK


def test_analysis_grid_matches_oracle_rule(oracle_mod):
    """zp_analysis_grid is host code: its Gauss-Legendre rule against numpy's
    (accurate to ~1e-15 for up to a few tens of nodes) and, at 50 and 300
    nodes, where numpy's rule loses digits near the ends, against nodes and
    weights refined by Newton's method in mpmath at 40 digits."""
    import mpmath as mp

    import paper_2409_19156_amd as zp

    for nr, nt in [(1, 1), (2, 5), (7, 3), (26, 101)]:
        r, th, w = zp.analysis_grid(nr, nt)
        ro, tho, wo = oracle_mod.analysis_grid(nr, nt)
        assert np.abs(r - ro).max() <= 4e-16 and np.abs(th - tho).max() <= 1e-15
        assert np.abs(w - wo).max() <= 1e-14 * np.abs(wo).max()
        assert abs(w.sum() - np.pi) <= 1e-14
    mp.mp.dps = 40
    for N, i in [(50, 0), (50, 24), (50, 49), (300, 0), (300, 1), (300, 77), (300, 149), (300, 150), (300, 298),
                 (300, 299)]:
        r, _, w = zp.analysis_grid(N, 1)
        x = 2 * mp.mpf(r[i]) ** 2 - 1
        for _ in range(4):
            p, q = mp.legendre(N, x), mp.legendre(N - 1, x)
            x -= p / (N * (x * p - q) / (x * x - 1))
        p, q = mp.legendre(N, x), mp.legendre(N - 1, x)
        dp = N * (x * p - q) / (x * x - 1)
        w_ref = 2 / ((1 - x * x) * dp * dp) / 4 * 2 * mp.pi
        assert abs(r[i] - mp.sqrt((1 + x) / 2)) <= 2.3e-16 * r[i], (N, i)  # one ulp
        assert abs(w[i] - w_ref) <= 2e-15 * w[i], (N, i)
        assert abs(w.sum() - np.pi) <= 1e-13


def test_analysis_grid_largest_rule_is_fast():
    """The largest accepted rule (4096 radial nodes) is built in well under a
    second of host time; its weights still sum to the disc's area."""
    import time

    import paper_2409_19156_amd as zp

    t0 = time.perf_counter()
    r, _, w = zp.analysis_grid(4096, 1)
    assert time.perf_counter() - t0 < 5.0
    assert np.all(np.diff(r) > 0) and 0 < r[0] and r[-1] < 1
    assert abs(w.sum() - np.pi) <= 1e-12


def test_analysis_validation(lib):
    n, m = _modes([2, 3], [0, -1])
    nd, md = n.ctypes.data, m.ctypes.data
    buf = np.zeros(8)
    p = buf.ctypes.data
    assert lib.zp_analysis_grid(0, 4, p, p, p) == ERR_ARG
    assert lib.zp_analysis_grid(2, 4, None, p, p) == ERR_ARG
    assert lib.zp_analysis_grid(4097, 1, p, p, p) == ERR_ARG  # above the radial node limit (O(nr^2) host work)
    full, mn = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.zp_series_analysis_workspace(2, 100, 3, 2, ctypes.byref(full), ctypes.byref(mn)) == OK
    assert 0 < mn.value <= full.value
    assert lib.zp_series_analysis_workspace(2, 100, 3, 9, ctypes.byref(full), None) == ERR_PREC
    bad, _ = _modes([2, 4], [0, -1])
    assert lib.zp_series_analysis(bad.ctypes.data, md, 2, FAKE, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, FAKE, 1 << 20,
                                  None) == ERR_MODE
    assert lib.zp_series_analysis(nd, md, 2, FAKE, FAKE, None, 4, FAKE, 2, 0, FAKE, FAKE, 1 << 20, None) == ERR_ARG
    assert lib.zp_series_analysis(nd, md, 2, FAKE, FAKE, FAKE, 4, FAKE, 2, 3, FAKE, FAKE, 1 << 20, None) == ERR_PREC
    assert lib.zp_series_analysis(nd, md, 2, FAKE, FAKE, FAKE, 4, FAKE, 2, 0, FAKE, FAKE, 16, None) == ERR_WS
    assert lib.zp_series_analysis(nd, md, 2, FAKE, FAKE, FAKE, 4, FAKE, 0, 0, FAKE, FAKE, 0, None) == OK
    # backward: c may be NULL only when grad_r and grad_theta are not requested
    assert lib.zp_series_bwd(nd, md, 2, FAKE, FAKE, 4, None, 2, 0, FAKE, None, None, FAKE, None, FAKE, 1 << 20,
                             None) == ERR_ARG
