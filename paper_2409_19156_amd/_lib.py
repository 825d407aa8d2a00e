"""ctypes loader for libzp.so (the C ABI declared in include/zp.h).

The library is built in-tree by ``paper_2409_19156_amd.build.build()``.  There
is no fallback: if the shared library is missing, importing the binding's
compute functions raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# ZP_LIBZP names another build of the same library to load (the sanitizer
# test's AddressSanitizer build of the host code).
LIB_PATH = os.environ.get("ZP_LIBZP") or os.path.join(_HERE, "libzp.so")

ZP_OK = 0
STATUS_NAMES = {0: "ZP_OK", 1: "ZP_ERR_MODE", 2: "ZP_ERR_ARG", 3: "ZP_ERR_ORDER", 4: "ZP_ERR_WORKSPACE",
                5: "ZP_ERR_HIP", 6: "ZP_ERR_PREC"}

# Every symbol include/zp.h declares.
EXPORTS = ("zp_radial", "zp_radial_direct", "zp_radial_zernike_recursion", "zp_basis", "zp_basis_polar", "zp_series_workspace", "zp_series_cache_bytes", "zp_series_fwd",
           "zp_series_bwd", "zp_series_jvp", "zp_series_bwd2_workspace", "zp_series_bwd2", "zp_series3d_workspace",
           "zp_series3d_cache_bytes", "zp_series3d_fwd", "zp_series3d_bwd", "zp_analysis_grid",
           "zp_series_analysis_workspace", "zp_series_analysis", "zp_series_fwd_noalloc", "zp_stream_fill", "zp_status_string", "zp_last_error", "zp_cache_clear",
           "zp_abi_version")


class ZpError(RuntimeError):
    def __init__(self, status: int, fn: str, detail: str):
        self.status = status
        super().__init__(f"{fn}: {STATUS_NAMES.get(status, status)}: {detail}")


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libzp.so not built at {LIB_PATH}; run paper_2409_19156_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    szp = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "zp_radial": [vp, vp, i64, vp, i64, i32, vp, vp],
        "zp_radial_direct": [vp, vp, i64, vp, i64, i32, vp, vp],
        "zp_radial_zernike_recursion": [vp, vp, i64, vp, i64, i32, vp, vp],
        "zp_basis": [vp, vp, i64, vp, vp, i64, u32, vp, vp],
        "zp_basis_polar": [vp, vp, i64, vp, i64, vp, i64, u32, vp, vp],
        "zp_series_workspace": [i64, i64, i64, i32, szp, szp],
        "zp_series_cache_bytes": [i64, i64, i32, szp],
        "zp_series_fwd": [vp, vp, i64, vp, vp, i64, vp, i64, i32, vp, vp, vp, sz, vp],
        "zp_series_bwd": [vp, vp, i64, vp, vp, i64, vp, i64, i32, vp, vp, vp, vp, vp, vp, sz, vp],
        "zp_series_jvp": [vp, vp, i64, vp, vp, i64, vp, i64, i32, vp, vp, vp, vp, vp, sz, vp],
        "zp_series_bwd2_workspace": [i64, i64, i64, i32, szp, szp],
        "zp_series_bwd2": [vp, vp, i64, vp, vp, i64, vp, i64, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp],
        "zp_series3d_workspace": [vp, vp, vp, i64, i64, i64, i64, i32, szp, szp],
        "zp_series3d_cache_bytes": [vp, vp, vp, i64, i64, i32, szp],
        "zp_series3d_fwd": [vp, vp, vp, i64, vp, vp, i64, vp, i64, vp, i64, i32, vp, vp, vp, sz, vp],
        "zp_series3d_bwd": [vp, vp, vp, i64, vp, vp, i64, vp, i64, vp, i64, i32, vp, vp, vp, vp, vp, vp, vp, sz, vp],
        "zp_analysis_grid": [i64, i64, vp, vp, vp],
        "zp_series_analysis_workspace": [i64, i64, i64, i32, szp, szp],
        "zp_series_analysis": [vp, vp, i64, vp, vp, vp, i64, vp, i64, i32, vp, vp, sz, vp],
        "zp_series_fwd_noalloc": [vp, vp, i64, vp, vp, i64, vp, i64, i32, vp, vp],
        "zp_stream_fill": [vp, i64, ctypes.c_double, i32, vp],
    }
    for name, args in sig.items():
        if not hasattr(lib, name):
            continue  # reported by the export test
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.zp_status_string.argtypes = [ctypes.c_int]
    lib.zp_status_string.restype = ctypes.c_char_p
    lib.zp_last_error.argtypes = []
    lib.zp_last_error.restype = ctypes.c_char_p
    lib.zp_cache_clear.argtypes = []
    lib.zp_cache_clear.restype = None
    lib.zp_abi_version.argtypes = []
    lib.zp_abi_version.restype = ctypes.c_int32
    _lib = lib
    return lib


def check(status: int, fn: str) -> None:
    if status != ZP_OK:
        lib = load()
        detail = lib.zp_last_error().decode() or lib.zp_status_string(status).decode()
        raise ZpError(status, fn, detail)
