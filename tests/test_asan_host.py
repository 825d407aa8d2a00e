"""Host code under AddressSanitizer (CPU only).

The oracle (oracle/zpo.c) and the host side of libzp (argument validation,
plan construction, size queries of the C ABI) are rebuilt with
AddressSanitizer, and the oracle pin tests and the C-ABI tests run against
those builds in a child process with the sanitizer runtime preloaded.  Any
out-of-bounds access or use after free aborts the child with a report.  No
GPU is used: the C-ABI tests only reach host code (validation errors and
no-op sizes return before the first HIP call), and the device code of the
sanitized libzp is built as usual (the sanitizer applies to host code only).
"""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2409_19156_amd", "csrc")


def _asan_runtime() -> str:
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not path or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("AddressSanitizer runtime not found")
    return path


@pytest.fixture(scope="module")
def asan_builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("asan")
    oracle_so = str(d / "libzpo_asan.so")
    subprocess.run(["gcc", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-fopenmp", "-fPIC",
                    "-shared", os.path.join(ROOT, "oracle", "zpo.c"), "-lquadmath", "-lm", "-o", oracle_so],
                   check=True)
    from paper_2409_19156_amd import build as zb

    zp_so = str(d / "libzp_asan.so")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in zb.HIPCC_FLAGS if f not in ("-O3",)]
    cmd = [hipcc, *flags, "-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
           "-fno-omit-frame-pointer", "-o", zp_so, *[os.path.join(CSRC, s) for s in zb.SOURCES]]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    return oracle_so, zp_so


def test_oracle_and_c_abi_under_address_sanitizer(asan_builds):
    oracle_so, zp_so = asan_builds
    env = dict(os.environ)
    env.update(LD_PRELOAD=_asan_runtime(), ZP_ORACLE_LIB=oracle_so, ZP_LIBZP=zp_so,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    files = ["tests/test_abi.py", "tests/test_oracle_pins.py", "tests/test_oracle_series_pins.py",
             "tests/test_oracle_series3d_pins.py", "tests/test_oracle_analysis_pins.py"]
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", *files],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (res.stdout + res.stderr)[-4000:]
    assert res.returncode == 0, tail
    assert "AddressSanitizer" not in res.stderr, tail
    # the child really ran the sanitized builds
    probe = subprocess.run([sys.executable, "-c", "import oracle, paper_2409_19156_amd._lib as L; "
                            "print(oracle._SO); print(L.LIB_PATH)"], cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=120)
    assert oracle_so in probe.stdout and zp_so in probe.stdout, probe.stdout + probe.stderr
