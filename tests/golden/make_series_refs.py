"""Write the oracle's values on fixed samples of the two timed series workloads,
for the error report of the benchmark (which does not run the oracle itself).

    python tests/golden/make_series_refs.py

Each file holds the sample (point and set indices), a digest of the workload's
inputs (so a changed generator is detected) and the oracle's f, grad_c,
grad_r and grad_theta on that sample:
  f[ps][:, bs_f], grad_c[:, bs_c], grad_r[ps], grad_theta[ps].
Only the oracle and the seeded input generators are called.
"""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def workload_digest(wl) -> str:
    h = hashlib.sha256()
    for a in (wl.n, wl.m, wl.r, wl.theta, wl.c, wl.g):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def sample(wl, npts: int, nsets_f: int, nsets_c: int, seed: int):
    rng = np.random.default_rng(seed)
    ps = np.sort(rng.choice(wl.P, npts, replace=False))
    ps[0], ps[-1] = int(np.argmin(wl.r)), int(np.argmax(wl.r))  # the innermost and outermost points
    ps = np.unique(ps)
    bs_f = np.sort(rng.choice(wl.B, nsets_f, replace=False))
    bs_c = np.sort(rng.choice(wl.B, nsets_c, replace=False))
    return ps, bs_f, bs_c


def write(wl, name: str, npts: int, nsets_f: int, nsets_c: int, seed: int):
    import oracle

    ps, bs_f, bs_c = sample(wl, npts, nsets_f, nsets_c, seed)
    Z = oracle.basis(wl.n, wl.m, wl.r, wl.theta, oracle.MASK_Z)[0]
    gc = Z @ wl.g[:, bs_c]
    del Z
    Zs, Zrs, Zts = oracle.series_basis(wl.n, wl.m, wl.r[ps], wl.theta[ps])
    f = oracle.series_fwd(Zs, wl.c[:, bs_f])
    _, gr, gt = oracle.series_bwd(Zs, Zrs, Zts, wl.c, wl.g[ps])
    path = os.path.join(HERE, name)
    np.savez_compressed(path, digest=np.array(workload_digest(wl)), ps=ps, bs_f=bs_f, bs_c=bs_c, f=f, grad_c=gc,
                        grad_r=gr, grad_theta=gt)
    print(path, os.path.getsize(path), "bytes")


def main():
    import zp_workloads as W

    write(W.series_n64(), "series_n64_oracle_sample.npz", 128, 64, 8, seed=99)
    write(W.series_n40(), "series_n40_oracle_sample.npz", 256, 64, 16, seed=98)


if __name__ == "__main__":
    main()
