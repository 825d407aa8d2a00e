"""MI355X (gfx950) Zernike polynomials: radial part, full basis, and the
differentiable Zernike series.

Thin binding over libzp.so (C ABI in include/zp.h).  Torch supplies device
memory and the current stream; every step of the computation runs in the
library's HIP kernels.  There is no CPU fallback: without the built library or
a GPU these functions raise.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from ._lib import ZpError

Z, DR, DR2, DR3, DTHETA = 1, 2, 4, 8, 16
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}

__all__ = ["radial", "radial_direct", "radial_zernike_recursion", "basis", "basis_polar", "stream_fill", "ZpError", "Z", "DR", "DR2", "DR3", "DTHETA", "PREC", "modes_i32"]


def modes_i32(n, m):
    """Host int32 copies of the mode arrays (they are metadata, like shapes)."""
    if isinstance(n, torch.Tensor):
        n = n.detach().cpu().numpy()
    if isinstance(m, torch.Tensor):
        m = m.detach().cpu().numpy()
    n = np.ascontiguousarray(n, dtype=np.int32).reshape(-1)
    m = np.ascontiguousarray(m, dtype=np.int32).reshape(-1)
    if n.shape != m.shape:
        raise ValueError("n and m must have the same length")
    return n, m


def _points(x: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if x.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    return x.reshape(-1).contiguous()


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def basis_polar(n, m, r: torch.Tensor, theta: torch.Tensor, mask: int = Z,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """``basis`` on the tensor grid of NR radii ``r`` times NT angles
    ``theta`` (point p = i * NT + j, angle fastest): float64
    [popcount(mask), M, NR * NT], equal to ``basis`` on the flattened points."""
    lib = _lib.load()
    nh, mh = modes_i32(n, m)
    r = _points(r, "r")
    theta = _points(theta, "theta")
    if theta.device != r.device:
        raise ValueError("r and theta must be on one device")
    M, NR, NT = nh.size, r.numel(), theta.numel()
    nout = bin(int(mask) & 31).count("1")
    shape = (max(nout, 1), M, NR * NT)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=r.device)
    elif out.shape != shape or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor [popcount(mask), M, NR * NT]")
    with torch.cuda.device(r.device):
        st = lib.zp_basis_polar(nh.ctypes.data, mh.ctypes.data, M, r.data_ptr(), NR, theta.data_ptr(), NT,
                                int(mask), out.data_ptr(), _stream(r.device))
    _lib.check(st, "zp_basis_polar")
    return out


def stream_fill(out: torch.Tensor, value: float = 0.0, nontemporal: bool = True) -> torch.Tensor:
    """out[:] = value by the library's streaming-write kernel (the benchmark's
    write-rate reference).  ``out``: contiguous float64 GPU tensor."""
    lib = _lib.load()
    if not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != torch.float64 or not out.is_contiguous():
        raise TypeError("out must be a contiguous float64 GPU tensor")
    with torch.cuda.device(out.device):
        st = lib.zp_stream_fill(out.data_ptr(), out.numel(), float(value), 1 if nontemporal else 0, _stream(out.device))
    _lib.check(st, "zp_stream_fill")
    return out


def radial(n, m, r: torch.Tensor, max_dr: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
    """d^j R_n^{|m|}(r) / dr^j for j = 0..max_dr.

    Returns a float64 tensor [max_dr+1, M, P] on r's device (plane j, mode i,
    point p).  ``out[j].T`` is the paper's (points x modes) array."""
    lib = _lib.load()
    nh, mh = modes_i32(n, m)
    r = _points(r, "r")
    M, P = nh.size, r.numel()
    if out is None:
        out = torch.empty((max_dr + 1, M, P), dtype=torch.float64, device=r.device)
    elif out.shape != (max_dr + 1, M, P) or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor [max_dr+1, M, P]")
    with torch.cuda.device(r.device):
        st = lib.zp_radial(nh.ctypes.data, mh.ctypes.data, M, r.data_ptr(), P, int(max_dr), out.data_ptr(),
                           _stream(r.device))
    _lib.check(st, "zp_radial")
    return out


def radial_direct(n, m, r: torch.Tensor, max_dr: int = 0) -> torch.Tensor:
    """Same outputs as ``radial`` but evaluated directly from the closed-form
    sum in FP64 (the paper's accuracy comparator; loses digits as n - |m|
    grows).  For accuracy comparisons only."""
    lib = _lib.load()
    nh, mh = modes_i32(n, m)
    r = _points(r, "r")
    M, P = nh.size, r.numel()
    out = torch.empty((max_dr + 1, M, P), dtype=torch.float64, device=r.device)
    with torch.cuda.device(r.device):
        st = lib.zp_radial_direct(nh.ctypes.data, mh.ctypes.data, M, r.data_ptr(), P, int(max_dr), out.data_ptr(),
                                  _stream(r.device))
    _lib.check(st, "zp_radial_direct")
    return out


def radial_zernike_recursion(n, m, r: torch.Tensor, max_dr: int = 0) -> torch.Tensor:
    """Same outputs as ``radial`` by the Zernike recursion (Eq.
    zernike-recursion) over the whole (n, |m|) triangle; n <= 60.  For accuracy
    comparisons only."""
    lib = _lib.load()
    nh, mh = modes_i32(n, m)
    r = _points(r, "r")
    M, P = nh.size, r.numel()
    out = torch.empty((max_dr + 1, M, P), dtype=torch.float64, device=r.device)
    with torch.cuda.device(r.device):
        st = lib.zp_radial_zernike_recursion(nh.ctypes.data, mh.ctypes.data, M, r.data_ptr(), P, int(max_dr),
                                             out.data_ptr(), _stream(r.device))
    _lib.check(st, "zp_radial_zernike_recursion")
    return out


def basis(n, m, r: torch.Tensor, theta: torch.Tensor, mask: int = Z, out: torch.Tensor | None = None) -> torch.Tensor:
    """Z_n^m(r, theta) and the derivatives selected by ``mask`` (Z, DR, DR2,
    DR3, DTHETA bits).  Returns float64 [popcount(mask), M, P]."""
    lib = _lib.load()
    nh, mh = modes_i32(n, m)
    r = _points(r, "r")
    theta = _points(theta, "theta")
    if theta.numel() != r.numel():
        raise ValueError("r and theta must have the same number of points")
    M, P = nh.size, r.numel()
    nout = bin(int(mask) & 31).count("1")
    shape = (max(nout, 1), M, P)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=r.device)
    elif out.shape != shape or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor [popcount(mask), M, P]")
    with torch.cuda.device(r.device):
        st = lib.zp_basis(nh.ctypes.data, mh.ctypes.data, M, r.data_ptr(), theta.data_ptr(), P, int(mask),
                          out.data_ptr(), _stream(r.device))
    _lib.check(st, "zp_basis")
    return out


# ------------------------------------------------------------------ series --

def _prec_code(prec) -> int:
    if isinstance(prec, str):
        if prec not in PREC:
            raise ValueError(f"prec must be one of {sorted(PREC)}")
        return PREC[prec]
    return int(prec)


def series_sizes(M: int, P: int, B: int, prec="fp64"):
    """(workspace bytes for one pass, minimum workspace bytes, basis-cache bytes)."""
    import ctypes

    lib = _lib.load()
    full = ctypes.c_size_t()
    mn = ctypes.c_size_t()
    cb = ctypes.c_size_t()
    _lib.check(lib.zp_series_workspace(M, P, B, _prec_code(prec), ctypes.byref(full), ctypes.byref(mn)),
               "zp_series_workspace")
    _lib.check(lib.zp_series_cache_bytes(M, P, _prec_code(prec), ctypes.byref(cb)), "zp_series_cache_bytes")
    return full.value, mn.value, cb.value


def _budget(mem_budget):
    import os

    if mem_budget is not None:
        return int(mem_budget)
    return int(os.environ.get("ZP_MEM_BUDGET_BYTES", str(32 << 30)))


def _workspace(M, P, B, prec, budget, device):
    full, mn, _ = series_sizes(M, P, B, prec)
    nbytes = full if full <= budget else max(mn, budget)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _coef(c: torch.Tensor, M: int) -> torch.Tensor:
    if not isinstance(c, torch.Tensor) or not c.is_cuda or c.dtype != torch.float64:
        raise TypeError("c must be a float64 GPU tensor [M, B]")
    if c.dim() != 2 or c.shape[0] != M:
        raise ValueError(f"c must have shape [M={M}, B]")
    return c.contiguous()


def series_forward(n, m, r, theta, c, prec="fp64", cache: torch.Tensor | None = None,
                   ws: torch.Tensor | None = None, mem_budget=None) -> torch.Tensor:
    """f[p, b] = sum_k c[k, b] Z_k(r_p, theta_p).  If ``cache`` (uint8, from
    ``series_sizes``) is given, the basis is kept in it for ``series_backward``."""
    lib = _lib.load()
    nh, mh = modes_i32(n, m)
    r, theta = _points(r, "r"), _points(theta, "theta")
    M, P = nh.size, r.numel()
    c = _coef(c, M)
    B = c.shape[1]
    f = torch.empty((P, B), dtype=torch.float64, device=r.device)
    if M == 0 or P == 0 or B == 0:  # an empty sum (the library call is a no-op)
        return f.zero_()
    if ws is None:
        ws = _workspace(M, P, B, prec, _budget(mem_budget), r.device)
    with torch.cuda.device(r.device):
        st = lib.zp_series_fwd(nh.ctypes.data, mh.ctypes.data, M, r.data_ptr(), theta.data_ptr(), P, c.data_ptr(), B,
                               _prec_code(prec), f.data_ptr(), cache.data_ptr() if cache is not None else None,
                               ws.data_ptr(), ws.numel(), _stream(r.device))
    _lib.check(st, "zp_series_fwd")
    return f


def series_backward(n, m, r, theta, c, g, prec="fp64", cache: torch.Tensor | None = None,
                    need=(True, True, True), ws: torch.Tensor | None = None, mem_budget=None):
    """(dL/dc, dL/dr, dL/dtheta) for upstream gradient g = dL/df [P, B]; entries
    not in ``need`` are returned as None."""
    lib = _lib.load()
    nh, mh = modes_i32(n, m)
    r, theta = _points(r, "r"), _points(theta, "theta")
    M, P = nh.size, r.numel()
    c = _coef(c, M)
    B = c.shape[1]
    g = g.contiguous()
    if g.shape != (P, B) or g.dtype != torch.float64:
        raise ValueError("g must be float64 [P, B]")
    dev = r.device
    gc = torch.empty((M, B), dtype=torch.float64, device=dev) if need[0] else None
    gr = torch.empty(P, dtype=torch.float64, device=dev) if need[1] else None
    gt = torch.empty(P, dtype=torch.float64, device=dev) if need[2] else None
    if M == 0 or P == 0 or B == 0:
        return tuple(None if x is None else x.zero_() for x in (gc, gr, gt))
    if ws is None:
        ws = _workspace(M, P, B, prec, _budget(mem_budget), dev)
    ptr = (lambda t: t.data_ptr() if t is not None else None)
    with torch.cuda.device(dev):
        st = lib.zp_series_bwd(nh.ctypes.data, mh.ctypes.data, M, r.data_ptr(), theta.data_ptr(), P, c.data_ptr(), B,
                               _prec_code(prec), g.data_ptr(), ptr(cache), ptr(gc), ptr(gr), ptr(gt), ws.data_ptr(),
                               ws.numel(), _stream(dev))
    _lib.check(st, "zp_series_bwd")
    return gc, gr, gt


def series_jvp(n, m, r, theta, c, tc=None, tr=None, ttheta=None, prec="fp64", ws: torch.Tensor | None = None,
               mem_budget=None) -> torch.Tensor:
    """Forward-mode derivative of ``series_forward`` along tangents (tc, tr,
    ttheta) of (c, r, theta); any tangent may be None."""
    lib = _lib.load()
    nh, mh = modes_i32(n, m)
    r, theta = _points(r, "r"), _points(theta, "theta")
    M, P = nh.size, r.numel()
    c = _coef(c, M)
    B = c.shape[1]
    tf = torch.empty((P, B), dtype=torch.float64, device=r.device)
    if tc is not None:
        tc = _coef(tc, M)
        if tc.shape != c.shape:
            raise ValueError("tc must have the shape of c")
    if tr is not None:
        tr = _points(tr, "tr")
    if ttheta is not None:
        ttheta = _points(ttheta, "ttheta")
    if M == 0 or P == 0 or B == 0:
        return tf.zero_()
    if ws is None:
        ws = _workspace(M, P, B, prec, _budget(mem_budget), r.device)
    ptr = (lambda t: t.data_ptr() if t is not None else None)
    with torch.cuda.device(r.device):
        st = lib.zp_series_jvp(nh.ctypes.data, mh.ctypes.data, M, r.data_ptr(), theta.data_ptr(), P, c.data_ptr(), B,
                               _prec_code(prec), ptr(tc), ptr(tr), ptr(ttheta), tf.data_ptr(), ws.data_ptr(),
                               ws.numel(), _stream(r.device))
    _lib.check(st, "zp_series_jvp")
    return tf


def series_backward2(n, m, r, theta, c, g, uc=None, ur=None, ut=None, prec="fp64", need=(True, True, True, True),
                     ws: torch.Tensor | None = None, mem_budget=None):
    """Adjoint of ``series_backward`` (second-order derivatives): for cotangents
    (uc, ur, ut) of its outputs (dL/dc, dL/dr, dL/dtheta), returns the
    derivatives of <uc, dL/dc> + <ur, dL/dr> + <ut, dL/dtheta> with respect to
    (g, c, r, theta); entries not in ``need`` are None, missing cotangents
    count as zero."""
    import ctypes

    lib = _lib.load()
    nh, mh = modes_i32(n, m)
    r, theta = _points(r, "r"), _points(theta, "theta")
    M, P = nh.size, r.numel()
    c = _coef(c, M)
    B = c.shape[1]
    g = g.contiguous()
    if g.shape != (P, B) or g.dtype != torch.float64:
        raise ValueError("g must be float64 [P, B]")
    if uc is not None:
        uc = _coef(uc, M)
    ur = _points(ur, "ur") if ur is not None else None
    ut = _points(ut, "ut") if ut is not None else None
    dev = r.device
    outs = [torch.empty(shape, dtype=torch.float64, device=dev) if want else None
            for want, shape in zip(need, ((P, B), (M, B), (P,), (P,)))]
    if M == 0 or P == 0 or B == 0:
        return tuple(None if x is None else x.zero_() for x in outs)
    if ws is None:
        full, mn = ctypes.c_size_t(), ctypes.c_size_t()
        _lib.check(lib.zp_series_bwd2_workspace(M, P, B, _prec_code(prec), ctypes.byref(full), ctypes.byref(mn)),
                   "zp_series_bwd2_workspace")
        budget = _budget(mem_budget)
        nbytes = full.value if full.value <= budget else max(mn.value, budget)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    ptr = (lambda t: t.data_ptr() if t is not None else None)
    with torch.cuda.device(dev):
        st = lib.zp_series_bwd2(nh.ctypes.data, mh.ctypes.data, M, r.data_ptr(), theta.data_ptr(), P, c.data_ptr(), B,
                                _prec_code(prec), g.data_ptr(), ptr(uc), ptr(ur), ptr(ut), *(ptr(x) for x in outs),
                                ws.data_ptr(), ws.numel(), _stream(dev))
    _lib.check(st, "zp_series_bwd2")
    return tuple(outs)


class _SeriesBackward(torch.autograd.Function):
    """(c, r, theta, g) -> (dL/dc, dL/dr, dL/dtheta) of the series, itself
    differentiable through zp_series_bwd2 (double backward)."""

    @staticmethod
    def forward(ctx, c, r, theta, g, modes, prec, cache, budget, need):
        nh, mh = modes
        ctx.set_materialize_grads(False)
        ctx.modes, ctx.prec, ctx.budget = modes, prec, budget
        ctx.save_for_backward(c, r, theta, g)
        return series_backward(nh, mh, r, theta, c, g, prec, cache=cache, need=need, mem_budget=budget)

    @staticmethod
    def backward(ctx, uc, ur, ut):
        c, r, theta, g = ctx.saved_tensors
        nh, mh = ctx.modes
        nc, nr, nt, ng = ctx.needs_input_grad[:4]
        if uc is None and ur is None and ut is None:
            return (None,) * 9
        og, oc, orr, ot = series_backward2(nh, mh, r, theta, c, g, uc, ur, ut, ctx.prec, need=(ng, nc, nr, nt),
                                           mem_budget=ctx.budget)
        return oc, orr, ot, og, None, None, None, None, None


class ZernikeSeries(torch.autograd.Function):
    """f = Z(r, theta)^T c with a hand-written adjoint (zp_series_bwd), its
    own adjoint for second derivatives (zp_series_bwd2), and a forward-mode
    rule (zp_series_jvp).

    The basis (Z, dZ/dr, dZ/dtheta) is kept from the forward when its size is
    within the memory budget, and recomputed chunk by chunk in the backward
    otherwise."""

    @staticmethod
    def forward(ctx, c, r, theta, n, m, prec="fp64", mem_budget=None):
        nh, mh = modes_i32(n, m)
        M, P, B = nh.size, r.numel(), c.shape[1]
        budget = _budget(mem_budget)
        _, _, cache_bytes = series_sizes(M, P, B, prec)
        cache = None
        if M and P and B and cache_bytes <= budget:
            cache = torch.empty(cache_bytes, dtype=torch.uint8, device=r.device)
        f = series_forward(nh, mh, r, theta, c, prec, cache=cache, mem_budget=budget)
        ctx.modes = (nh, mh)
        ctx.prec = prec
        ctx.budget = budget
        ctx.cache = cache
        ctx.save_for_backward(c, r, theta)
        ctx.save_for_forward(c, r, theta)
        return f

    @staticmethod
    def backward(ctx, g):
        c, r, theta = ctx.saved_tensors
        need = tuple(bool(x) for x in ctx.needs_input_grad[:3])
        gc, gr, gt = _SeriesBackward.apply(c, r, theta, g.contiguous(), ctx.modes, ctx.prec, ctx.cache, ctx.budget,
                                           need)
        if gr is not None:
            gr = gr.view_as(r)
        if gt is not None:
            gt = gt.view_as(theta)
        return gc, gr, gt, None, None, None, None

    @staticmethod
    def jvp(ctx, tc, tr, ttheta, *unused):
        c, r, theta = ctx.saved_tensors
        nh, mh = ctx.modes
        return series_jvp(nh, mh, r, theta, c, tc=tc, tr=tr, ttheta=ttheta, prec=ctx.prec, mem_budget=ctx.budget)


def series(c, r, theta, n, m, prec="fp64", mem_budget=None):
    """Differentiable Zernike series f[p, b] = sum_k c[k, b] Z_k(r_p, theta_p)."""
    return ZernikeSeries.apply(c, r, theta, n, m, prec, mem_budget)


__all__ += ["series_sizes", "series_forward", "series_backward", "series_backward2", "series_jvp", "ZernikeSeries",
            "series"]


# ------------------------------------------------------------- analysis --

def analysis_grid(nr: int, nt: int):
    """Host quadrature rule on the unit disc (numpy float64 r, theta, w of
    nr * nt points, theta fastest): Gauss-Legendre in r^2 times the
    trapezoidal rule in theta.  Exact for modes n <= L with
    nr >= ceil((L+1)/2), nt >= 2L+1."""
    lib = _lib.load()
    P = int(nr) * int(nt)
    r, th, w = (np.empty(max(P, 1), dtype=np.float64) for _ in range(3))
    _lib.check(lib.zp_analysis_grid(int(nr), int(nt), r.ctypes.data, th.ctypes.data, w.ctypes.data),
               "zp_analysis_grid")
    return r[:P], th[:P], w[:P]


def series_analysis(n, m, r, theta, w, f, prec="fp64", ws: torch.Tensor | None = None,
                    mem_budget=None) -> torch.Tensor:
    """Coefficients c[k, b] = (1/N_k) sum_p w_p Z_k(r_p, theta_p) f[p, b] from
    samples f [P, B] with quadrature weights w [P] (N_k = integral of Z_k^2)."""
    import ctypes

    lib = _lib.load()
    nh, mh = modes_i32(n, m)
    r, theta, w = _points(r, "r"), _points(theta, "theta"), _points(w, "w")
    M, P = nh.size, r.numel()
    if not isinstance(f, torch.Tensor) or f.dtype != torch.float64 or f.dim() != 2 or f.shape[0] != P:
        raise ValueError("f must be a float64 GPU tensor [P, B]")
    f = f.contiguous()
    B = f.shape[1]
    c = torch.empty((M, B), dtype=torch.float64, device=r.device)
    if M == 0 or B == 0:
        return c
    if ws is None:
        full, mn = ctypes.c_size_t(), ctypes.c_size_t()
        _lib.check(lib.zp_series_analysis_workspace(M, P, B, _prec_code(prec), ctypes.byref(full), ctypes.byref(mn)),
                   "zp_series_analysis_workspace")
        budget = _budget(mem_budget)
        nbytes = full.value if full.value <= budget else max(mn.value, budget)
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=r.device)
    with torch.cuda.device(r.device):
        st = lib.zp_series_analysis(nh.ctypes.data, mh.ctypes.data, M, r.data_ptr(), theta.data_ptr(), w.data_ptr(),
                                    P, f.data_ptr(), B, _prec_code(prec), c.data_ptr(), ws.data_ptr(), ws.numel(),
                                    _stream(r.device))
    _lib.check(st, "zp_series_analysis")
    return c


__all__ += ["analysis_grid", "series_analysis"]


# ---------------------------------------------------- three-dimensional --

def modes3_i32(n, m, l):
    nh, mh = modes_i32(n, m)
    if isinstance(l, torch.Tensor):
        l = l.detach().cpu().numpy()
    lh = np.ascontiguousarray(l, dtype=np.int32).reshape(-1)
    if lh.shape != nh.shape:
        raise ValueError("n, m and l must have the same length")
    return nh, mh, lh


def series3d_sizes(n, m, l, P: int, Q: int, B: int, prec="fp64"):
    """(workspace bytes for one pass, minimum workspace bytes, basis-cache bytes)
    of the three-dimensional series."""
    import ctypes

    lib = _lib.load()
    nh, mh, lh = modes3_i32(n, m, l)
    full, mn, cb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _lib.check(lib.zp_series3d_workspace(nh.ctypes.data, mh.ctypes.data, lh.ctypes.data, nh.size, P, Q, B,
                                         _prec_code(prec), ctypes.byref(full), ctypes.byref(mn)),
               "zp_series3d_workspace")
    _lib.check(lib.zp_series3d_cache_bytes(nh.ctypes.data, mh.ctypes.data, lh.ctypes.data, nh.size, P,
                                           _prec_code(prec), ctypes.byref(cb)), "zp_series3d_cache_bytes")
    return full.value, mn.value, cb.value


def _workspace3(nh, mh, lh, P, Q, B, prec, budget, device):
    full, mn, _ = series3d_sizes(nh, mh, lh, P, Q, B, prec)
    nbytes = full if full <= budget else max(mn, budget)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def series3d_forward(n, m, l, r, theta, phi, c, prec="fp64", cache: torch.Tensor | None = None,
                     ws: torch.Tensor | None = None, mem_budget=None) -> torch.Tensor:
    """f[p, q, b] = sum_j c[j, b] Z_{n_j m_j}(r_p, theta_p) F_{l_j}(phi_q), with
    F_l(phi) = cos(l phi) (l >= 0) or sin(|l| phi) (l < 0).  Modes sharing (n, m)
    share one Zernike evaluation."""
    lib = _lib.load()
    nh, mh, lh = modes3_i32(n, m, l)
    r, theta, phi = _points(r, "r"), _points(theta, "theta"), _points(phi, "phi")
    J, P, Q = nh.size, r.numel(), phi.numel()
    c = _coef(c, J)
    B = c.shape[1]
    f = torch.empty((P, Q, B), dtype=torch.float64, device=r.device)
    if J == 0 or P == 0 or Q == 0 or B == 0:
        return f.zero_()
    if ws is None:
        ws = _workspace3(nh, mh, lh, P, Q, B, prec, _budget(mem_budget), r.device)
    with torch.cuda.device(r.device):
        st = lib.zp_series3d_fwd(nh.ctypes.data, mh.ctypes.data, lh.ctypes.data, J, r.data_ptr(), theta.data_ptr(), P,
                                 phi.data_ptr(), Q, c.data_ptr(), B, _prec_code(prec), f.data_ptr(),
                                 cache.data_ptr() if cache is not None else None, ws.data_ptr(), ws.numel(),
                                 _stream(r.device))
    _lib.check(st, "zp_series3d_fwd")
    return f


def series3d_backward(n, m, l, r, theta, phi, c, g, prec="fp64", cache: torch.Tensor | None = None,
                      need=(True, True, True, True), ws: torch.Tensor | None = None, mem_budget=None):
    """(dL/dc, dL/dr, dL/dtheta, dL/dphi) for g = dL/df [P, Q, B]; entries not
    in ``need`` are None."""
    lib = _lib.load()
    nh, mh, lh = modes3_i32(n, m, l)
    r, theta, phi = _points(r, "r"), _points(theta, "theta"), _points(phi, "phi")
    J, P, Q = nh.size, r.numel(), phi.numel()
    c = _coef(c, J)
    B = c.shape[1]
    g = g.contiguous()
    if g.shape != (P, Q, B) or g.dtype != torch.float64:
        raise ValueError("g must be float64 [P, Q, B]")
    dev = r.device
    outs = [torch.empty(shape, dtype=torch.float64, device=dev) if want else None
            for want, shape in zip(need, ((J, B), (P,), (P,), (Q,)))]
    if J == 0 or P == 0 or Q == 0 or B == 0:
        return tuple(None if x is None else x.zero_() for x in outs)
    if ws is None:
        ws = _workspace3(nh, mh, lh, P, Q, B, prec, _budget(mem_budget), dev)
    ptr = (lambda t: t.data_ptr() if t is not None else None)
    with torch.cuda.device(dev):
        st = lib.zp_series3d_bwd(nh.ctypes.data, mh.ctypes.data, lh.ctypes.data, J, r.data_ptr(), theta.data_ptr(), P,
                                 phi.data_ptr(), Q, c.data_ptr(), B, _prec_code(prec), g.data_ptr(), ptr(cache),
                                 *(ptr(x) for x in outs), ws.data_ptr(), ws.numel(), _stream(dev))
    _lib.check(st, "zp_series3d_bwd")
    return tuple(outs)


class ZernikeSeries3D(torch.autograd.Function):
    """f = sum_j c_j Z_{n_j m_j}(r, theta) F_{l_j}(phi) on a (polar points) x
    (phi) grid, with the hand-written adjoint zp_series3d_bwd.  The basis of
    the distinct (n, m) pairs is kept from the forward when it fits the
    memory budget."""

    @staticmethod
    def forward(ctx, c, r, theta, phi, n, m, l, prec="fp64", mem_budget=None):
        nh, mh, lh = modes3_i32(n, m, l)
        J, P, Q, B = nh.size, r.numel(), phi.numel(), c.shape[1]
        budget = _budget(mem_budget)
        cache = None
        if J and P and Q and B:
            _, _, cache_bytes = series3d_sizes(nh, mh, lh, P, Q, B, prec)
            if cache_bytes <= budget:
                cache = torch.empty(cache_bytes, dtype=torch.uint8, device=r.device)
        f = series3d_forward(nh, mh, lh, r, theta, phi, c, prec, cache=cache, mem_budget=budget)
        ctx.modes = (nh, mh, lh)
        ctx.prec = prec
        ctx.budget = budget
        ctx.cache = cache
        ctx.save_for_backward(c, r, theta, phi)
        return f

    @staticmethod
    def backward(ctx, g):
        c, r, theta, phi = ctx.saved_tensors
        nh, mh, lh = ctx.modes
        need = ctx.needs_input_grad[:4]
        gc, gr, gt, gp = series3d_backward(nh, mh, lh, r, theta, phi, c, g, ctx.prec, cache=ctx.cache, need=need,
                                           mem_budget=ctx.budget)
        gr = gr.view_as(r) if gr is not None else None
        gt = gt.view_as(theta) if gt is not None else None
        gp = gp.view_as(phi) if gp is not None else None
        return gc, gr, gt, gp, None, None, None, None, None


def series3d(c, r, theta, phi, n, m, l, prec="fp64", mem_budget=None):
    """Differentiable three-dimensional spectral series f[p, q, b]."""
    return ZernikeSeries3D.apply(c, r, theta, phi, n, m, l, prec, mem_budget)


__all__ += ["series3d_sizes", "series3d_forward", "series3d_backward", "ZernikeSeries3D", "series3d"]
