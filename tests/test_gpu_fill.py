"""zp_stream_fill, the streaming-write reference of the benchmark: every
element written, nothing past the end, for even and odd lengths, with
non-temporal and plain stores."""
from __future__ import annotations

import ctypes

import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 1001, 65536, (1 << 20) + 3])
@pytest.mark.parametrize("nt", [1, 0])
def test_stream_fill_writes_exactly_n(n, nt):
    from paper_2409_19156_amd import _lib

    lib = _lib.load()
    buf = torch.full((n + 16,), -7.0, dtype=torch.float64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.zp_stream_fill(buf.data_ptr(), n, 2.5, nt, stream) == 0, lib.zp_last_error()
    torch.cuda.synchronize()
    assert bool((buf[:n] == 2.5).all())
    assert bool((buf[n:] == -7.0).all())
