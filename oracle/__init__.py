"""Reference implementation (the oracle) of the Zernike radial, basis and series
computations, for checking the GPU library.

TEST INFRASTRUCTURE ONLY: only the test-suite, the smoke check and the CPU
baseline of the benchmark may import this package.  The product library never
does, and this package imports nothing from it.

* ``radial`` / ``basis``  -- quad-precision (binary128) C code in ``zpo.c``
  following the paper: Eq. (jacobi-relation), Eq. (jacobi) for P_0 and P_1,
  Eq. (jacobi-recursion) for the chain, the derivative identity with the
  Pochhammer symbol (Sec. 2), Algorithm 1's loop structure, and Eq.
  (zernike-poly) for the angular factor.
* ``series_*`` -- the Zernike series f = sum_k c_k Z_k (Eq. zernike-poly
  summed over modes) and its exact adjoint, as plain float64 matrix products
  on the oracle basis rounded to double.
* ``series_basis2`` / ``series_bwd2`` -- second derivatives of the basis
  (d2Z/dr2 from the quad oracle; d2Z/(dr dtheta) and d2Z/dtheta2 = -m^2 Z
  from the quad radial derivative and long-double trigonometry) and the
  adjoint of ``series_bwd`` (double backward), written out term by term.
* ``analysis_grid`` / ``analysis`` -- coefficients from samples by
  quadrature, c_k = (1/N_k) sum_p w_p Z_k(p) f_p with N_k the integral of
  Z_k^2 over the unit disc (orthogonality of the basis); the rule is
  Gauss-Legendre in r^2 (numpy's routine) times the trapezoidal rule in theta.
* ``fourier`` / ``series3d_*`` -- the three-dimensional spectral series of the
  paper's duplicated-mode use (Sec. 3, footnote): modes (n, m, l), value
  sum_j c_j R_n^m(r) F_m(theta) F_l(phi) with F the Fourier basis, evaluated
  over the full (duplicated) mode list with no deduplication, and its adjoint.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ZP_ORACLE_LIB names a prebuilt copy to load instead (the sanitizer test
# builds one with AddressSanitizer); build() then compiles nothing.
_SO = os.environ.get("ZP_ORACLE_LIB") or os.path.join(_HERE, "libzpo.so")
_lib = None

MASK_Z, MASK_DR, MASK_DR2, MASK_DR3, MASK_DTHETA = 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile ``zpo.c`` into ``libzpo.so`` (gcc, OpenMP, libquadmath)."""
    import subprocess

    src = os.path.join(_HERE, "zpo.c")
    if os.environ.get("ZP_ORACLE_LIB"):
        return _SO
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", src, "-lquadmath", "-lm", "-o", tmp],
            check=True,
        )
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.zpo_radial.argtypes = [i32p, i32p, ctypes.c_int64, f64p, ctypes.c_int64, ctypes.c_int,
                                   f64p, f64p, ctypes.c_int]
        lib.zpo_basis.argtypes = [i32p, i32p, ctypes.c_int64, f64p, f64p, ctypes.c_int64,
                                  ctypes.c_uint32, f64p, f64p, ctypes.c_int]
        lib.zpo_jacobi_chain.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, f64p, f64p]
        lib.zpo_jacobi_explicit.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            f64p, f64p]
        lib.zpo_max_threads.argtypes = []
        for f in (lib.zpo_radial, lib.zpo_basis, lib.zpo_jacobi_chain, lib.zpo_jacobi_explicit,
                  lib.zpo_max_threads):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


_ERR = {1: "invalid mode (n < 0, |m| > n or n - |m| odd)", 2: "bad argument", 3: "out of memory"}


def max_threads() -> int:
    return _load().zpo_max_threads()


def radial(n, m, r, max_dr: int, with_lo: bool = False, nthreads: int = 0):
    """R_n^{|m|}(r) and its r-derivatives up to ``max_dr``.

    Returns ``hi`` of shape [max_dr+1, M, P] (and ``lo`` if ``with_lo``): the
    binary128 result as hi + lo.
    """
    n, m, r = _i32(n), _i32(m), _f64(r)
    M, P = n.size, r.size
    hi = np.zeros((max_dr + 1, M, P))
    lo = np.zeros_like(hi) if with_lo else None
    rc = _load().zpo_radial(_ptr(n, ctypes.c_int32), _ptr(m, ctypes.c_int32), M, _ptr(r, ctypes.c_double), P,
                            max_dr, _ptr(hi, ctypes.c_double),
                            _ptr(lo, ctypes.c_double) if with_lo else None, nthreads)
    if rc:
        raise ValueError(f"oracle radial: {_ERR.get(rc, rc)}")
    return (hi, lo) if with_lo else hi


def basis(n, m, r, theta, mask: int, with_lo: bool = False, nthreads: int = 0):
    """Z, dZ/dr, d2Z/dr2, d3Z/dr3, dZ/dtheta selected by ``mask`` bits 0..4.

    Returns [popcount(mask), M, P] (hi, and lo if asked)."""
    n, m, r, theta = _i32(n), _i32(m), _f64(r), _f64(theta)
    M, P = n.size, r.size
    if theta.size != P:
        raise ValueError("r and theta must have the same length")
    nout = bin(mask & 31).count("1")
    hi = np.zeros((nout, M, P))
    lo = np.zeros_like(hi) if with_lo else None
    rc = _load().zpo_basis(_ptr(n, ctypes.c_int32), _ptr(m, ctypes.c_int32), M, _ptr(r, ctypes.c_double),
                           _ptr(theta, ctypes.c_double), P, mask, _ptr(hi, ctypes.c_double),
                           _ptr(lo, ctypes.c_double) if with_lo else None, nthreads)
    if rc:
        raise ValueError(f"oracle basis: {_ERR.get(rc, rc)}")
    return (hi, lo) if with_lo else hi


def jacobi_chain(kmax: int, a: int, b: int, x_hi: float, x_lo: float = 0.0):
    """P_k^{(a,b)}(x), k = 0..kmax, by Eq. (jacobi) seeds + Eq. (jacobi-recursion)."""
    hi = np.zeros(kmax + 1)
    lo = np.zeros(kmax + 1)
    rc = _load().zpo_jacobi_chain(kmax, a, b, x_hi, x_lo, _ptr(hi, ctypes.c_double), _ptr(lo, ctypes.c_double))
    if rc:
        raise ValueError(f"oracle jacobi_chain: {_ERR.get(rc, rc)}")
    return hi, lo


def jacobi_explicit(k: int, a: int, b: int, x: float):
    """P_k^{(a,b)}(x) by the explicit sum of Eq. (jacobi)."""
    hi = ctypes.c_double()
    lo = ctypes.c_double()
    rc = _load().zpo_jacobi_explicit(k, a, b, x, ctypes.byref(hi), ctypes.byref(lo))
    if rc:
        raise ValueError(f"oracle jacobi_explicit: {_ERR.get(rc, rc)}")
    return hi.value, lo.value


# ---------------------------------------------------------------- series --
#
# f[p, b] = sum_k Z[k, p] c[k, b]      (the Zernike series at every point, for
#                                       every coefficient set b)
# Given an upstream gradient g[p, b] of a scalar loss L with dL/df = g:
#   dL/dc[k, b]   = sum_p Z[k, p] g[p, b]
#   dL/dr[p]      = sum_b g[p, b] sum_k dZ/dr[k, p] c[k, b]
#   dL/dtheta[p]  = sum_b g[p, b] sum_k dZ/dtheta[k, p] c[k, b]
# (each point's r and theta enter only that point's row of f).

def series_basis(n, m, r, theta, nthreads: int = 0):
    """Oracle basis planes (Z, dZ/dr, dZ/dtheta), each [M, P], rounded to double."""
    return basis(n, m, r, theta, MASK_Z | MASK_DR | MASK_DTHETA, nthreads=nthreads)


def series_basis2(n, m, r, theta, nthreads: int = 0):
    """(d2Z/dr2, d2Z/(dr dtheta), d2Z/dtheta2), each [M, P]."""
    n = np.asarray(n)
    m = np.asarray(m)
    Zrr = basis(n, m, r, theta, MASK_DR2, nthreads=nthreads)[0]
    dR = radial(n, m, r, 1, nthreads=nthreads)[1]  # dR/dr [M, P]
    a = np.abs(m).astype(np.longdouble)[:, None]
    arg = a * np.asarray(theta, dtype=np.float64).astype(np.longdouble)[None, :]
    # d/dtheta of cos(a theta) = -a sin(a theta); of sin(a theta) = a cos(a theta)
    dtrig = np.where(m[:, None] >= 0, -a * np.sin(arg), a * np.cos(arg))
    Zrt = (dR.astype(np.longdouble) * dtrig).astype(np.float64)
    Z = basis(n, m, r, theta, MASK_Z, nthreads=nthreads)[0]
    Ztt = -(np.abs(m).astype(np.float64) ** 2)[:, None] * Z
    return Zrr, Zrt, Ztt


def series_fwd(Z, c):
    """f = Z^T c with Z [M, P] and c [M, B]: returns [P, B]."""
    return np.asarray(Z).T @ np.asarray(c)


def series_bwd(Z, Zr, Zt, c, g):
    """Adjoint of ``series_fwd`` with respect to c, r and theta."""
    Z, Zr, Zt, c, g = (np.asarray(a) for a in (Z, Zr, Zt, c, g))
    grad_c = Z @ g
    grad_r = np.einsum("pb,pb->p", g, Zr.T @ c)
    grad_t = np.einsum("pb,pb->p", g, Zt.T @ c)
    return grad_c, grad_r, grad_t


def fourier(l, phi, deriv: int = 0):
    """Fourier factor F_l(phi) = cos(l phi) for l >= 0 and sin(|l| phi) for
    l < 0 (the convention of Eq. zernike-poly for the angle), or its first
    phi-derivative.  The product l*phi and the trigonometric functions are
    taken in long double; returns float64 [len(l), len(phi)]."""
    l = np.asarray(l, dtype=np.int64).reshape(-1, 1)
    ph = np.asarray(phi, dtype=np.float64).reshape(1, -1)
    a = np.abs(l).astype(np.longdouble)
    arg = a * ph.astype(np.longdouble)
    cs, sn = np.cos(arg), np.sin(arg)
    if deriv == 0:
        out = np.where(l >= 0, cs, sn)
    else:  # d/dphi cos(a phi) = -a sin(a phi); d/dphi sin(a phi) = a cos(a phi)
        out = np.where(l >= 0, -a * sn, a * cs)
    return out.astype(np.float64)


def series3d_fwd(Z, F, c):
    """f[p, q, b] = sum_j Z[j, p] F[j, q] c[j, b]: Z is the basis of the full
    mode list [J, P], F the Fourier factors [J, Q], c [J, B]."""
    return np.einsum("jp,jq,jb->pqb", np.asarray(Z), np.asarray(F), np.asarray(c), optimize=True)


def series3d_bwd(Z, Zr, Zt, F, dF, c, g):
    """Adjoint of ``series3d_fwd`` for an upstream gradient g [P, Q, B], with
    respect to c, r, theta and phi (dF = dF/dphi)."""
    Z, Zr, Zt, F, dF, c, g = (np.asarray(a) for a in (Z, Zr, Zt, F, dF, c, g))
    grad_c = np.einsum("jp,jq,pqb->jb", Z, F, g, optimize=True)
    grad_r = np.einsum("pqb,jp,jq,jb->p", g, Zr, F, c, optimize=True)
    grad_t = np.einsum("pqb,jp,jq,jb->p", g, Zt, F, c, optimize=True)
    grad_phi = np.einsum("pqb,jp,jq,jb->q", g, Z, dF, c, optimize=True)
    return grad_c, grad_r, grad_t, grad_phi


def series_bwd2(Z, Zr, Zt, Zrr, Zrt, Ztt, c, g, uc, ur, ut):
    """Adjoint of ``series_bwd``: with L2 = <uc, grad_c> + <ur, grad_r> +
    <ut, grad_t>, returns (dL2/dg, dL2/dc, dL2/dr, dL2/dtheta)."""
    Z, Zr, Zt, Zrr, Zrt, Ztt, c, g, uc, ur, ut = (np.asarray(a) for a in (Z, Zr, Zt, Zrr, Zrt, Ztt, c, g, uc, ur, ut))
    # grad_c = Z g;  grad_r[p] = sum_b g[p,b] (Zr^T c)[p,b];  grad_t likewise with Zt
    out_g = Z.T @ uc + ur[:, None] * (Zr.T @ c) + ut[:, None] * (Zt.T @ c)
    out_c = (Zr * ur[None, :] + Zt * ut[None, :]) @ g
    Hu = g @ uc.T  # [P, M]
    Hc = g @ c.T
    out_r = np.einsum("kp,pk->p", Zr, Hu) + ur * np.einsum("kp,pk->p", Zrr, Hc) + ut * np.einsum("kp,pk->p", Zrt, Hc)
    out_t = np.einsum("kp,pk->p", Zt, Hu) + ur * np.einsum("kp,pk->p", Zrt, Hc) + ut * np.einsum("kp,pk->p", Ztt, Hc)
    return out_g, out_c, out_r, out_t


def mode_norms(n, m):
    """N_k = integral of Z_k^2 over the unit disc: the radial integral
    1 / (2 (n + 1)) times pi (m != 0) or 2 pi (m = 0)."""
    n = np.asarray(n, dtype=np.float64)
    m = np.asarray(m)
    return np.where(m == 0, 2.0, 1.0) * np.pi / (2.0 * (n + 1.0))


def analysis_grid(nr: int, nt: int):
    """Quadrature on the disc: Gauss-Legendre nodes x in t = r^2 = (1 + x)/2,
    times nt equispaced angles; point p = i * nt + j.  Returns (r, theta, w)."""
    x, wx = np.polynomial.legendre.leggauss(nr)
    t = (1.0 + x) / 2.0
    th = 2.0 * np.pi * np.arange(nt) / nt
    r = np.repeat(np.sqrt(t), nt)
    theta = np.tile(th, nr)
    # r dr = dt / 2 and dt = dx / 2; the angle contributes 2 pi / nt
    w = np.repeat(wx / 4.0 * (2.0 * np.pi / nt), nt)
    return r, theta, w


def analysis(Z, n, m, w, f):
    """c[k, b] = (1 / N_k) sum_p w_p Z[k, p] f[p, b]."""
    return (np.asarray(Z) @ (np.asarray(w)[:, None] * np.asarray(f))) / mode_norms(n, m)[:, None]
