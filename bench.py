"""Benchmark: FP64 Zernike basis entries/s on the L = M = 50 polar-grid workload
(1326 ANSI modes n <= 50 at 64 Chebyshev-Gauss-Lobatto radii x 128 theta =
8192 points; outputs Z, dZ/dr, d2Z/dr2, d3Z/dr3, dZ/dtheta), plus the
mixed-precision vs FP64 speedup of the Zernike series forward + backward.

One step = one zp_basis call over the whole grid (inputs resident in HBM).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
FP64_PEAK_TFS = 78.6  # MI355X FP64 MFMA (dense), published

# Measured HBM traffic of the basis kernel on this workload: two rocprofv3
# --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch, median of 5) of
#   bench.py --steps 3 --warmup 1 --no-series --no-spectral3d --no-radial --no-ad --no-cpu-baseline
# scaled by what the same counters read for a plain 1 GiB device copy
#   bench.py --copy-calibration-mb 1024
# (FETCH_SIZE 524299.5 KiB for 1048576 KiB read: x2.0; WRITE_SIZE 1048576 KiB
# for 1048576 KiB written: x1.0).  Valid only for the kernel sources it was
# taken on; reported as null once they change.
TRAFFIC = {"sources": ("paper_2409_19156_amd/csrc/chain_kernel.hip", "paper_2409_19156_amd/csrc/zp_internal.hpp"),
           "sha256": "3a57c2c967d0012d97e8508ab1e3eae43f26d23c1440cfc79c5f75ec5123ffa2",
           "fetch_kib": 469.0, "fetch_scale": 1048576.0 / 524299.8,
           "write_kib": 424769.9, "write_scale": 1.0}


def measured_traffic():
    import hashlib

    h = hashlib.sha256()
    for f in TRAFFIC["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC["sha256"]:
        return None
    return (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"] + TRAFFIC["write_kib"] * TRAFFIC["write_scale"]) * 1024.0


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-series", action="store_true")
    ap.add_argument("--no-spectral3d", action="store_true")
    ap.add_argument("--no-radial", action="store_true")
    ap.add_argument("--no-ad", action="store_true")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB, 5 times (for scaling "
                         "hardware byte counters), then exit")
    ap.add_argument("--cpu-sample-points", type=int, default=0,
                    help="points of the workload the oracle is timed on (0: all)")
    return ap.parse_args()


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, sample_points: int):
    """The oracle (quad precision, OpenMP over points), untuned, on a bounded
    sample of the same workload's points; scaled to entries/s.  Timed with all
    the threads OpenMP gives it (the reported value) and with one thread on a
    smaller strided sample."""
    import oracle

    oracle.build(force=False)
    threads = oracle.max_threads()
    if sample_points <= 0:
        # The whole grid takes the oracle ~1-2 s on a 16-thread host share: time
        # all of it (a bounded sample is only needed for larger grids).
        sample_points = wl.P
    idx = np.linspace(0, wl.P - 1, sample_points).astype(np.int64)
    t0 = time.perf_counter()
    oracle.basis(wl.n, wl.m, wl.r[idx], wl.theta[idx], wl.mask)
    dt = time.perf_counter() - t0
    entries = wl.M * 5 * sample_points
    one = max(1, sample_points // 8)
    idx1 = np.linspace(0, wl.P - 1, one).astype(np.int64)
    t0 = time.perf_counter()
    oracle.basis(wl.n, wl.m, wl.r[idx1], wl.theta[idx1], wl.mask, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": entries / dt, "unit": "entries/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample_points} of {wl.P} grid points (evenly strided), all {wl.M} modes, 5 outputs; "
                      f"{dt:.1f} s",
            "single_thread": {"value": wl.M * 5 * one / dt1, "unit": "entries/s", "cores": 1,
                              "sample": f"{one} of {wl.P} grid points (evenly strided); {dt1:.1f} s"},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count()}


def _errors(got, ref):
    """Error measures of one output tensor against the oracle: max-norm and
    Frobenius-norm relative errors, and the largest elementwise relative error
    over the entries whose magnitude exceeds 1e-3 of the largest."""
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    d = np.abs(got - ref)
    big = np.abs(ref) > 1e-3 * np.abs(ref).max()
    return {"inf": float(d.max() / np.abs(ref).max()),
            "fro": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "elem": float((d[big] / np.abs(ref[big])).max())}


def _oracle_sample(name: str, wl):
    """The oracle's values on a fixed sample of a series workload, written by
    tests/golden/make_series_refs.py (the benchmark does not run the oracle
    outside its CPU-baseline leg).  None if the file is missing or was made
    from other inputs."""
    import hashlib

    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    d = np.load(path, allow_pickle=False)
    h = hashlib.sha256()
    for a in (wl.n, wl.m, wl.r, wl.theta, wl.c, wl.g):
        h.update(np.ascontiguousarray(a).tobytes())
    if str(d["digest"]) != h.hexdigest():
        return None
    return {k: d[k] for k in d.files}


def _sample_errors(ref, f, gc, gr, gt):
    """Errors of the GPU outputs (numpy) on the stored oracle sample."""
    ps = ref["ps"]
    got = (f[ps][:, ref["bs_f"]], gc[:, ref["bs_c"]], gr[ps], gt[ps])
    return {k: _errors(a, ref[k]) for k, a in zip(("f", "grad_c", "grad_r", "grad_theta"), got)}


def series_leg(steps: int, warmup: int):
    """FP64 vs mixed-precision Zernike series on the n <= 64 workload (2145
    modes, 65536 disc points, 1024 coefficient sets): the forward alone, then
    forward + backward; each precision's error per output against the oracle
    on a fixed sample (f on 128 points x 64 sets, grad_r and grad_theta on the
    128 points, grad_c for all modes on 8 sets).  Then one GPU's share of an
    eight-way split by points (P/8 points), forward + backward."""
    import torch

    import paper_2409_19156_amd as zp
    import zp_workloads as W

    wl = W.series_n64()
    dev = torch.device("cuda:0")
    r, th = torch.from_numpy(wl.r).to(dev), torch.from_numpy(wl.theta).to(dev)
    c, g = torch.from_numpy(wl.c).to(dev), torch.from_numpy(wl.g).to(dev)
    out = {}
    stream = torch.cuda.current_stream(dev)
    oref = _oracle_sample("series_n64_oracle_sample.npz", wl)
    ps = wl.P // 8
    for prec in ("fp64", "fp32", "bf16x3"):
        full, _, cb = zp.series_sizes(wl.M, wl.P, wl.B, prec)
        ws = torch.empty(full, dtype=torch.uint8, device=dev)
        cache = torch.empty(cb, dtype=torch.uint8, device=dev)

        res = []

        def step():  # forward + backward; keeps the last outputs in res
            f = zp.series_forward(wl.n, wl.m, r, th, c, prec, cache=cache, ws=ws)
            res[:] = (f,) + zp.series_backward(wl.n, wl.m, r, th, c, g, prec, cache=cache, ws=ws)

        def fwd():
            zp.series_forward(wl.n, wl.m, r, th, c, prec, cache=cache, ws=ws)

        def timed(fn):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / steps

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ms_fwd = timed(fwd)
        ms = timed(step)
        entry = {"ms_fwd_bwd": ms, "ms_fwd": ms_fwd, "gemm_gflop": 3 * 2.0 * wl.P * wl.M * wl.B / 1e9}
        entry["algorithmic_tflops"] = entry["gemm_gflop"] / ms
        if oref is not None:
            entry["err_vs_oracle"] = _sample_errors(oref, *(x.cpu().numpy() for x in res))
        full_rows = [x[:ps].clone() for x in (res[0], res[2], res[3])]  # f, grad_r, grad_theta of the shard
        del ws, cache, res[:]
        torch.cuda.empty_cache()

        # One GPU's share of an eight-way split by points: the first P/8 points,
        # all modes and sets.  f, grad_r and grad_theta of those points must
        # equal the full run's; grad_c is that GPU's partial sum before the
        # all-reduce.
        full, _, cb = zp.series_sizes(wl.M, ps, wl.B, prec)
        ws = torch.empty(full, dtype=torch.uint8, device=dev)
        cache = torch.empty(cb, dtype=torch.uint8, device=dev)
        rs, ts, gs = r[:ps], th[:ps], g[:ps]

        def step_shard():
            f = zp.series_forward(wl.n, wl.m, rs, ts, c, prec, cache=cache, ws=ws)
            res[:] = (f,) + zp.series_backward(wl.n, wl.m, rs, ts, c, gs, prec, cache=cache, ws=ws)

        for _ in range(warmup):
            step_shard()
        torch.cuda.synchronize()
        ms_s = timed(step_shard)
        gflop_s = 3 * 2.0 * ps * wl.M * wl.B / 1e9
        same = all(bool(torch.equal(a, b)) for a, b in zip(full_rows, (res[0], res[2], res[3])))
        entry["shard_8way"] = {"points": ps, "ms_fwd_bwd": ms_s, "algorithmic_tflops": gflop_s / ms_s,
                               "per_point_outputs_equal_full_run": same}
        out[prec] = entry
        del ws, cache, res[:], full_rows
        torch.cuda.empty_cache()
    out["speedup_bf16x3_vs_fp64"] = out["fp64"]["ms_fwd_bwd"] / out["bf16x3"]["ms_fwd_bwd"]
    out["speedup_fp32_vs_fp64"] = out["fp64"]["ms_fwd_bwd"] / out["fp32"]["ms_fwd_bwd"]
    out["workload"] = "series_n64: ANSI n<=64 (2145 modes), 65536 disc points, 1024 sets, fwd+bwd (c, r, theta)"
    out["err_sample"] = ("oracle (stored) on 128 fixed points x 64 sets (f), the same points (grad_r, grad_theta), "
                         "8 sets x all modes (grad_c)" if oref is not None else "oracle sample missing")
    out["shard_8way"] = ("one GPU's share of an 8-way split by points (the first P/8 points, all modes and sets), "
                         "forward + backward without the all-reduce of grad_c; its f, grad_r and grad_theta are "
                         "compared with the full run's rows for those points")
    return out


def series_n40_leg(steps: int, warmup: int):
    """The FP64 differentiable series on the n <= 40 workload (861 modes, 16384
    disc points, 256 sets): forward + backward through the autograd function,
    with the contraction work (three GEMMs of 2PMB) as a fraction of the FP64
    MFMA peak, and the error of every output against the oracle on a fixed
    sample (f on 256 points x 64 sets, grad_r and grad_theta on the 256
    points, grad_c for all modes on 16 sets)."""
    import torch

    import paper_2409_19156_amd as zp
    import zp_workloads as W

    wl = W.series_n40()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    r0, th0 = torch.from_numpy(wl.r).to(dev), torch.from_numpy(wl.theta).to(dev)
    c0, g = torch.from_numpy(wl.c).to(dev), torch.from_numpy(wl.g).to(dev)
    res = []

    def step():
        c, r, th = (x.detach().requires_grad_() for x in (c0, r0, th0))
        f = zp.series(c, r, th, wl.n, wl.m, "fp64")
        f.backward(g)
        res[:] = (f.detach(), c.grad, r.grad, th.grad)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    gflop = 3 * 2.0 * wl.P * wl.M * wl.B / 1e9
    oref = _oracle_sample("series_n40_oracle_sample.npz", wl)
    errs = _sample_errors(oref, *(x.cpu().numpy() for x in res)) if oref is not None else "oracle sample missing"
    return {"workload": "series_n40: ANSI n<=40 (861 modes), 16384 disc points, 256 sets, FP64, forward + "
                        "autograd backward (c, r, theta)",
            "ms_fwd_bwd": ms, "gemm_gflop": gflop, "algorithmic_tflops": gflop / ms,
            "frac_of_fp64_mfma_peak": gflop / ms / FP64_PEAK_TFS, "err_vs_oracle": errs}


def radial_legs(steps: int, warmup: int):
    """The radial-only configurations: n <= 16 at 1002 points with orders 0..3
    (launch-bound: entries/s only) and the n <= 200 stress set (10 201 pairs,
    100 000 clustered points, orders 0..2: 3.06e9 entries, 24.5 GB written per
    launch)."""
    import torch

    import paper_2409_19156_amd as zp
    import zp_workloads as W

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {}
    for wl in (W.radial_n16(), W.radial_n200()):
        r = torch.from_numpy(wl.r).to(dev)
        buf = torch.empty((wl.max_dr + 1, wl.M, wl.P), dtype=torch.float64, device=dev)
        for _ in range(warmup):
            zp.radial(wl.n, wl.m, r, wl.max_dr, out=buf)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            zp.radial(wl.n, wl.m, r, wl.max_dr, out=buf)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        entries = buf.numel()
        nbytes = entries * 8 + wl.P * 8
        out[wl.name] = {"modes": wl.M, "points": wl.P, "orders": wl.max_dr + 1, "entries": entries,
                        "ms_per_launch": ms, "entries_per_s": entries / (ms * 1e-3),
                        "GBs": nbytes / (ms * 1e-3) / 1e9, "frac_of_hbm_peak": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del buf
        torch.cuda.empty_cache()
    return out


def ad_analysis_leg(steps: int, warmup: int):
    """Forward-mode and second-order derivatives of the series on the n <= 64
    workload (2145 modes, 65 536 points, 1024 sets), and the analysis transform
    on a 256 x 512 quadrature grid (131 072 points, 1024 sets), per precision.
    Algorithmic contraction work: JVP 2 x 2PMB (the stacked K = 2M), second-order
    adjoint 4 x 2PMB (split-K, two column-dots, and the JVP's 2), analysis 2PMB."""
    import torch

    import paper_2409_19156_amd as zp
    import zp_workloads as W

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    wl = W.series_n64()
    r, th = torch.from_numpy(wl.r).to(dev), torch.from_numpy(wl.theta).to(dev)
    c, g = torch.from_numpy(wl.c).to(dev), torch.from_numpy(wl.g).to(dev)
    rng = np.random.default_rng(7)
    tc = torch.from_numpy(rng.standard_normal(wl.c.shape) / (wl.n + 1.0)[:, None]).to(dev)
    tr = torch.from_numpy(rng.standard_normal(wl.P)).to(dev)
    tt = torch.from_numpy(rng.standard_normal(wl.P)).to(dev)
    ra, tha, wa = zp.analysis_grid(256, 512)
    ra, tha, wa = (torch.from_numpy(x).to(dev) for x in (ra, tha, wa))
    fa = torch.from_numpy(rng.standard_normal((ra.numel(), wl.B))).to(dev)
    unit = 2.0 * wl.P * wl.M * wl.B / 1e9

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    out = {"workload": "series_n64 (JVP, second-order adjoint); analysis on 256 x 512 Gauss-Legendre x trapezoid "
                       "points, 1024 sets"}
    for prec in ("fp64", "bf16x3"):
        ms_jvp = timed(lambda: zp.series_jvp(wl.n, wl.m, r, th, c, tc, tr, tt, prec))
        ms_b2 = timed(lambda: zp.series_backward2(wl.n, wl.m, r, th, c, g, tc, tr, tt, prec))
        ms_an = timed(lambda: zp.series_analysis(wl.n, wl.m, ra, tha, wa, fa, prec))
        an_gf = 2.0 * ra.numel() * wl.M * wl.B / 1e9
        out[prec] = {"ms_jvp": ms_jvp, "jvp_tflops": 2 * unit / ms_jvp, "ms_bwd2": ms_b2,
                     "bwd2_tflops": 4 * unit / ms_b2, "ms_analysis": ms_an, "analysis_tflops": an_gf / ms_an}
        torch.cuda.empty_cache()
    return out


def spectral3d_leg(steps: int, warmup: int):
    """Three-dimensional spectral series with duplicated modes (561 (n, m) pairs
    x 33 values of l = 18 513 modes; 32 768 polar points x 64 toroidal planes):
    forward + backward of the deduplicated path per precision, and the forward
    of the planar series over the full duplicated mode list (coefficients
    c_j F_{l_j}(phi_q) prepared beforehand) as the comparison."""
    import torch

    import paper_2409_19156_amd as zp
    import zp_workloads as W

    w = W.spectral3d_L32()
    dev = torch.device("cuda:0")
    P, Q, B = w.r.size, w.phi.size, w.c.shape[1]
    r, th, ph = (torch.from_numpy(x).to(dev) for x in (w.r, w.theta, w.phi))
    c, g = torch.from_numpy(w.c).to(dev), torch.from_numpy(w.g).to(dev)
    stream = torch.cuda.current_stream(dev)
    U = int(np.unique(np.stack([w.n, w.m]), axis=1).shape[1])

    def timed(fn):
        for _ in range(warmup):
            res = fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            res = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, res

    out, ref = {"workload": f"spectral3d_L32: {w.J} modes = {U} (n, m) pairs x 33 l; {P} polar points "
                            f"(128 CGL radii x 256 theta) x {Q} phi planes; {B} set; fwd+bwd (c, r, theta, phi)",
                "modes": w.J, "distinct_pairs": U}, None
    for prec in ("fp64", "bf16x3"):
        full, _, cb = zp.series3d_sizes(w.n, w.m, w.l, P, Q, B, prec)
        ws = torch.empty(full, dtype=torch.uint8, device=dev)
        cache = torch.empty(cb, dtype=torch.uint8, device=dev)

        def step():
            f = zp.series3d_forward(w.n, w.m, w.l, r, th, ph, c, prec, cache=cache, ws=ws)
            return (f,) + zp.series3d_backward(w.n, w.m, w.l, r, th, ph, c, g, prec, cache=cache, ws=ws)

        ms, res = timed(step)
        ms_f, _ = timed(lambda: zp.series3d_forward(w.n, w.m, w.l, r, th, ph, c, prec, cache=cache, ws=ws))
        entry = {"ms_fwd_bwd": ms, "ms_fwd": ms_f, "gemm_gflop_dedup": 3 * 2.0 * P * U * Q * B / 1e9}
        if prec == "fp64":
            ref = [x.clone() for x in res]
        else:
            errs = [((a - b).abs().max() / b.abs().max()).item() for a, b in zip(res, ref)]
            entry["rel_err_vs_fp64"] = dict(zip(("f", "grad_c", "grad_r", "grad_theta", "grad_phi"), errs))
        out[prec] = entry
        del ws, cache
        torch.cuda.empty_cache()
    # the same forward as a planar series over the duplicated list
    a = np.abs(w.l)[:, None] * w.phi[None, :]
    F = np.where(w.l[:, None] >= 0, np.cos(a), np.sin(a))
    cq = torch.from_numpy((w.c[:, None, :] * F[:, :, None]).reshape(w.J, Q * B)).to(dev)
    full, _, _ = zp.series_sizes(w.J, P, Q * B, "fp64")
    ws = torch.empty(full, dtype=torch.uint8, device=dev)
    ms_dup, f_dup = timed(lambda: zp.series_forward(w.n, w.m, r, th, cq, "fp64", ws=ws))
    out["fp64_duplicated_planar_ms_fwd"] = ms_dup
    out["dedup_speedup_fwd_fp64"] = ms_dup / out["fp64"]["ms_fwd"]
    out["dedup_vs_duplicated_rel_diff"] = ((f_dup.view(P, Q, B) - ref[0]).abs().max() / ref[0].abs().max()).item()
    del ws
    torch.cuda.empty_cache()
    return out


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py measures a single GPU only (asked for --gpus {args.gpus}): the library runs one process "
              "per GPU with no collectives", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration_mb:
        n = args.copy_calibration_mb << 20
        src = torch.ones(n // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n, "copy_calibration_bytes_written": n, "calls": 5}))
        return

    import paper_2409_19156_amd as zp
    import zp_workloads as W

    wl = W.basis_L50()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    r = torch.from_numpy(wl.r).to(dev)
    th = torch.from_numpy(wl.theta).to(dev)
    out = torch.empty((5, wl.M, wl.P), dtype=torch.float64, device=dev)
    entries = wl.M * wl.P * 5
    bytes_per_launch = entries * 8 + wl.P * 16  # outputs written + r, theta read

    t0 = time.perf_counter()
    zp.basis(wl.n, wl.m, r, th, 31, out=out)
    torch.cuda.synchronize()
    first_call_ms = (time.perf_counter() - t0) * 1e3
    for _ in range(args.warmup):
        zp.basis(wl.n, wl.m, r, th, 31, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        zp.basis(wl.n, wl.m, r, th, 31, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall) * 1e3
    ms = ev0.elapsed_time(ev1) / args.steps
    value = entries / (ms * 1e-3)
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9

    # The same basis through the polar-grid entry point (64 radii x 128 angles):
    # bitwise the same output, one radial recurrence per lane instead of two.
    rr, tt = W.cgl_polar_axes(64, 128)
    rrd, ttd = torch.from_numpy(rr).to(dev), torch.from_numpy(tt).to(dev)
    for _ in range(args.warmup):
        zp.basis_polar(wl.n, wl.m, rrd, ttd, 31, out=out)
    ev0.record(stream)
    for _ in range(args.steps):
        zp.basis_polar(wl.n, wl.m, rrd, ttd, 31, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_polar = ev0.elapsed_time(ev1) / args.steps

    # Reference streaming-write rate on the same buffer: the library's trivial
    # fill kernel (one 16-byte store per lane), non-temporal and plain; the
    # faster of the two is the measured write peak.
    fill_rates = {}
    for nt in (1, 0):
        for _ in range(3):
            zp.stream_fill(out, 0.0, nontemporal=bool(nt))
        ev0.record(stream)
        for _ in range(20):
            zp.stream_fill(out, 0.0, nontemporal=bool(nt))
        ev1.record(stream)
        torch.cuda.synchronize()
        fill_rates["nontemporal" if nt else "plain"] = out.numel() * 8 / (ev0.elapsed_time(ev1) / 20 * 1e-3) / 1e9
    fill_gbs = max(fill_rates.values())

    res = {
        "metric": "Zernike basis entries/s FP64 (L=M=50) & series fwd+bwd speedup at stated err",
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "basis_L50: ANSI n<=50 (1326 modes) on 64 CGL radii x 128 theta (8192 points), "
                               "outputs Z, dZ/dr, d2Z/dr2, d3Z/dr3, dZ/dtheta",
                   "modes": wl.M, "points": wl.P, "outputs": 5, "entries": entries},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "chain_kernel<3, true, false, 2, false, false, false>", "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": ms * 1e3, "measured_fill_GBs": fill_gbs, "fill_GBs": fill_rates,
                     "frac_of_measured_fill": achieved / fill_gbs},
        "basis_polar": {"entry": "zp_basis_polar (64 radii x 128 angles, same output)", "ms": ms_polar,
                        "entries_per_s": entries / (ms_polar * 1e-3),
                        "frac_of_hbm_peak": bytes_per_launch / (ms_polar * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "frac_of_measured_fill": bytes_per_launch / (ms_polar * 1e-3) / 1e9 / fill_gbs},
        "first_call_ms": first_call_ms,
        "timed_wall_ms": wall_ms,
    }
    if not args.no_series:
        res["series"] = series_leg(steps=max(3, min(args.steps, 10)), warmup=2)
        # small problem: enough warm-up for the clocks to settle (the first 20
        # passes after 3 warm-ups ran ~10% slower than the next 40)
        res["series_n40"] = series_n40_leg(steps=max(3, min(args.steps, 50)), warmup=20)
    if not args.no_spectral3d:
        res["spectral3d"] = spectral3d_leg(steps=max(3, min(args.steps, 20)), warmup=10)
    if not args.no_radial:
        res["radial"] = radial_legs(steps=max(3, min(args.steps, 10)), warmup=2)
        for leg in res["radial"].values():  # against the write rate measured above as well
            leg["frac_of_measured_fill"] = leg["GBs"] / fill_gbs
    if not args.no_ad:
        res["ad_analysis"] = ad_analysis_leg(steps=max(3, min(args.steps, 5)), warmup=1)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_points)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
