#!/usr/bin/env python3
"""Throughput of the star-M t-SVDM-II hot path on one MI355X.

Workload (default): the climate-like tensor 512 (lat) x 1024 (lon) x 256
(time), FP32 in HBM, M = orthonormal DCT-II along time, t-SVDM-II with
relative tolerance 1e-3.  One step = transform -> slice SVDs -> rank
selection -> factor packing -> reconstruction with back-transform -> FP64
error report.  The mixed-precision path (FP32 MFMA transform, FP32 Jacobi
with FP64 angles/convergence/energies) is the reported value; the plain FP64
path is timed beside it on the same FP32 input (its up-cast is inside the
step).  Metric: input GB/s = m*p*n*4 bytes / step time.

Prints one JSON line (see the design doc for every field).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"hbm_GBs": 8000.0, "f32_TF": 157.3, "f64_TF": 78.6}
METRIC = "input GB/s through t-SVDM-II (mixed-prec vs FP64 GPU) at stated rel. error"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_src_sha():
    h = hashlib.sha256()
    for f in ("jacobi.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2605_16058_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_steps(op, A, steps, warmup, torch):
    for _ in range(warmup):
        res = op(A)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = op(A)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return res, (t1 - t0) * 1e3 / steps


def jacobi_roofline(stats, m, p, esize, dtype_peak_tf):
    launches, ms, pg, pr, width = stats
    L, r = max(m, p), min(m, p)
    Wd = width
    f_gram = 2.0 * Wd * Wd * L
    f_rot = f_gram + 2.0 * Wd * Wd * (L + r)
    b_gram = Wd * L * esize
    b_rot = b_gram + 2.0 * Wd * (L + r) * esize
    flops = pg * f_gram + pr * f_rot
    nbytes = pg * b_gram + pr * b_rot
    t = ms * 1e-3
    ai = flops / max(nbytes, 1.0)
    ridge = dtype_peak_tf * 1e12 / (PEAK["hbm_GBs"] * 1e9)
    per_launch_ms = ms / max(launches, 1)
    if ai >= ridge:
        ach = flops / t / 1e12
        return {"bound": "mfma", "achieved": round(ach, 3), "peak": dtype_peak_tf,
                "unit": "TFLOP/s", "frac": round(ach / dtype_peak_tf, 4), "traffic": None,
                "kernel": "jacobi_round", "launches": int(launches),
                "avg_launch_ms": round(per_launch_ms, 4),
                "flops_per_launch": flops / max(launches, 1),
                "bytes_per_launch": nbytes / max(launches, 1), "ai_flop_per_byte": round(ai, 2)}
    ach = nbytes / t / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK["hbm_GBs"], "unit": "GB/s",
            "frac": round(ach / PEAK["hbm_GBs"], 4), "traffic": None, "kernel": "jacobi_round",
            "launches": int(launches), "avg_launch_ms": round(per_launch_ms, 4),
            "flops_per_launch": flops / max(launches, 1),
            "bytes_per_launch": nbytes / max(launches, 1), "ai_flop_per_byte": round(ai, 2)}


def load_traffic(key, sha):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f).get(key)
    except (OSError, ValueError):
        return None
    if not d or d.get("src_sha") != sha:
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(m, p, n_sample, eps):
    """The FP64 oracle, as it stands, on the first n_sample time steps of the
    same recipe (a bounded sample of the workload)."""
    import numpy as np
    import threadpoolctl

    import oracle
    import synth

    A = synth.climate_like(m, p, n_sample, rng=np.random.default_rng(2))
    M = synth.dct2_matrix(n_sample)
    t0 = time.perf_counter()
    res = oracle.tsvdm_ii(A.astype(np.float64), M, eps)
    dt = time.perf_counter() - t0
    threads = max((i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()), default=1)
    gbs = m * p * n_sample * 4 / dt / 1e9
    return {"value": round(gbs, 5), "unit": "GB/s", "cores": int(threads), "kind": "oracle",
            "sample": f"climate-like {m}x{p}x{n_sample} (first {n_sample} of 256 time steps), "
                      f"DCT-II {n_sample}, t-SVDM-II tol {eps}, FP64 NumPy/LAPACK; "
                      f"{dt:.2f} s wall, rel_err {res['rel_error']:.3e}",
            "seconds": round(dt, 3)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f32", choices=["f32", "bf16x3", "bf16"])
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--shape", default="512,1024,256")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 comparison path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=32)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM counters)")
    a = ap.parse_args(argv)

    if a.calibrate_copy:
        import torch
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4, "repeats": 3}), flush=True)
        return 0

    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); every box here has a "
              "single GPU and the multi-GPU layout is a design note, not a built path.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_2605_16058_amd import _lib, ops
    from paper_2605_16058_amd.pipeline import TSVDM

    m, p, n = (int(x) for x in a.shape.split(","))
    log(f"generating climate-like {m}x{p}x{n} FP32")
    A = synth.climate_like(m, p, n, rng=np.random.default_rng(2))
    M = synth.dct2_matrix(n)
    Ad = torch.from_numpy(np.ascontiguousarray(A.transpose(2, 1, 0))).cuda().permute(2, 1, 0)
    del A
    in_bytes = m * p * n * 4

    lib = _lib.load()
    op_mix = TSVDM((m, p, n), M, mode="II", eps=a.eps, precision=a.precision, block=a.block)
    log(f"mixed ({a.precision}) warmup {a.warmup}, steps {a.steps}")
    for _ in range(a.warmup):
        op_mix(Ad)
    torch.cuda.synchronize()
    lib.tsvdm_stats_reset()
    lib.tsvdm_stats_enable(1)
    res_mix, ms_mix = time_steps(op_mix, Ad, a.steps, 0, torch)
    lib.tsvdm_stats_enable(0)
    import ctypes
    launches, ms, pg, pr, width = (ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64(),
                                   ctypes.c_int64(), ctypes.c_int32())
    lib.tsvdm_stats_get(ctypes.byref(launches), ctypes.byref(ms), ctypes.byref(pg),
                        ctypes.byref(pr), ctypes.byref(width))
    stats = (launches.value, ms.value, pg.value, pr.value, width.value)
    log(f"mixed: {ms_mix:.2f} ms/step; jacobi stats {stats}")
    roof = jacobi_roofline(stats, m, p, 4, PEAK["f32_TF"])
    sha = kernel_src_sha()
    roof["src_sha"] = sha
    tr = load_traffic(f"jacobi_round_f32_{m}x{p}x{n}", sha)
    if tr is not None:
        roof["traffic"] = tr
    status_mix = int(res_mix.svd_status.item())
    rel_mix = res_mix.rel_error()
    sum_rho_mix = int(res_mix.offsets[-1].item())

    out_f64 = {}
    if not a.no_f64:
        op64 = TSVDM((m, p, n), M, mode="II", eps=a.eps, precision="f64", block=a.block)
        log(f"fp64 warmup {a.warmup}, steps {a.steps}")
        res64, ms64 = time_steps(op64, Ad, a.steps, a.warmup, torch)
        log(f"fp64: {ms64:.2f} ms/step")
        d = ops.tsvdm_error(res64.A_rec, res_mix.A_rec)
        e = d.double().cpu()
        nA = float(res64.err[1].cpu())
        out_f64 = {
            "fp64_GBs": round(in_bytes / (ms64 * 1e-3) / 1e9, 3),
            "fp64_ms_per_step": round(ms64, 3),
            "speedup_vs_fp64": round(ms64 / ms_mix, 3),
            "fp64_rel_error": res64.rel_error(),
            "fp64_sum_rho": int(res64.offsets[-1].item()),
            "fp64_svd_status": int(res64.svd_status.item()),
            "mixed_vs_fp64_rel_diff": math.sqrt(float(e[0]) / nA) if nA > 0 else 0.0,
        }
        del res64, op64
        torch.cuda.empty_cache()

    cpu = None
    if not a.no_cpu_baseline:
        log(f"cpu baseline: oracle on {m}x{p}x{a.cpu_sample_n}")
        cpu = cpu_baseline(m, p, a.cpu_sample_n, a.eps)

    value = in_bytes / (ms_mix * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_mix, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.precision == "f32" else a.precision,
        "data": "synthetic",
        "config": {"workload": f"climate-like {m}x{p}x{n} FP32, DCT-II, t-SVDM-II tol {a.eps}",
                   "m": m, "p": p, "n": n, "eps": a.eps, "precision": a.precision},
        "rel_error": rel_mix,
        "sum_rho": sum_rho_mix,
        "svd_status": status_mix,
        **out_f64,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
