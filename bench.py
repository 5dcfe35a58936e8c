#!/usr/bin/env python3
"""Throughput of the star-M t-SVDM hot path on one MI355X.

Default workload (the reported line): the climate-like tensor 512 (lat) x
1024 (lon) x 256 (time), FP32 in HBM, M = orthonormal DCT-II along time,
t-SVDM-II with relative tolerance 1e-3.  One step = transform -> slice SVDs ->
rank selection -> factor packing -> reconstruction with back-transform -> FP64
error report.  The mixed-precision path (FP32 MFMA transform, FP32 Jacobi with
FP64 angles/convergence/energies) gives the value; the plain FP64 path is
timed beside it on the same FP32 input (its up-cast is inside the step).
Metric: input GB/s = m*p*n*4 bytes / step time.

Other workloads (--workload): ragged (512 uneven tensors through one batch
plan), turbulence (2048x1024x256, transform precision sweep), cayley
(gradient steps on a Cayley-parameterised M).  Each prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
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
    for f in ("jacobi.hip", "precond.hip", "angle.h", "common.h"):
        with open(os.path.join(ROOT, "paper_2605_16058_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_stats(lib):
    v = [ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(),
         ctypes.c_double(), ctypes.c_double()]
    lib.tsvdm_stats_get(*[ctypes.byref(x) for x in v])
    k = ["launches", "ms", "pairs_gram", "pairs_rot", "pair_width", "flops", "bytes"]
    return dict(zip(k, [x.value for x in v]))


def jacobi_roofline(st, peak_tf):
    """Roofline entry of jacobi_round for workloads without a single shape
    (the batch): the kernel's own per-pair flops and bytes from the
    library's counters over the event-timed launches (the caller adds the
    method's flops)."""
    t = st["ms"] * 1e-3
    launches = max(st["launches"], 1)
    ai = st["flops"] / max(st["bytes"], 1.0)
    ridge = peak_tf * 1e12 / (PEAK["hbm_GBs"] * 1e9)
    common = {"traffic": None, "kernel": "jacobi_round", "launches": int(st["launches"]),
              "avg_launch_ms": round(st["ms"] / launches, 4),
              "flops_per_launch": st["flops"] / launches,
              "bytes_per_launch": st["bytes"] / launches, "ai_flop_per_byte": round(ai, 2),
              "pair_width": st["pair_width"], "pairs_rotating": st["pairs_rot"],
              "pairs_gram_only": st["pairs_gram"]}
    if ai >= ridge:
        ach = st["flops"] / t / 1e12
        return {"bound": "mfma", "achieved": round(ach, 3), "peak": peak_tf, "unit": "TFLOP/s",
                "frac": round(ach / peak_tf, 4), **common}
    ach = st["bytes"] / t / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK["hbm_GBs"], "unit": "GB/s",
            "frac": round(ach / PEAK["hbm_GBs"], 4), **common}


def svd_work(m, p, n, rho_sum):
    """Algorithmic flops of the slice SVDs by the Householder-bidiagonalisation
    convention: 4 L r^2 - (4/3) r^3 per slice for the singular values plus
    4 (L + r) r rho_i for the retained vectors (L = max(m, p), r = min(m, p))."""
    L, r = max(m, p), min(m, p)
    return n * (4.0 * L * r * r - 4.0 / 3.0 * r ** 3), 4.0 * (L + r) * r * rho_sum


def path_roofline(m, p, n, rho_sum, eb, peak_tf, transform, ms_per_step):
    """Roofline time of the whole step, T_roof = sum over stages of
    max(bytes / HBM peak, flops / compute peak), and its fraction of the
    measured step.  Stages: forward transform (FP32 in, eb out), slice SVD
    values (read A-hat) and retained vectors (write the packed factors),
    low-rank product (read factors, write C-hat), back-transform (read C-hat,
    write FP32 A_rho), error sums (read A and A_rho).  eb: bytes per element
    of the compute type."""
    N = float(m) * p * n
    tf = 2.5 * math.log2(n) if transform == "dct" else 2.0 * n   # flops per element
    f_val, f_vec = svd_work(m, p, n, rho_sum)
    fac = rho_sum * (m + p + 1) * eb
    stages = {
        "transform": (N * (4 + eb), N * tf),
        "svd_values": (N * eb, f_val),
        "svd_vectors": (fac, f_vec),
        "lowrank": (rho_sum * (m + p) * eb + N * eb, 2.0 * m * p * rho_sum),
        "back_transform": (N * (eb + 4), N * tf),
        "error": (N * 8, 3.0 * N),
    }
    t = {k: max(b / (PEAK["hbm_GBs"] * 1e9), f / (peak_tf * 1e12)) * 1e3 for k, (b, f) in stages.items()}
    t_roof = sum(t.values())
    return {"t_roof_ms": round(t_roof, 4), "path_frac": round(t_roof / ms_per_step, 4),
            "stage_ms": {k: round(v, 4) for k, v in t.items()},
            "algorithmic_bytes": N * 4 * 2 + fac}


def svd_roofline(st, steps, m, p, n, rho_sum, peak_tf, traffic_per_launch, alg_bytes_step):
    """Roofline entry of the dominant kernel (jacobi_round).  achieved = the
    slice SVDs' algorithmic flops (svd_work) per launch over the launch time
    measured with HIP events on the library's stream; the kernel's own flop
    count (Gram plus rotation of every pair it processed) is kept beside it
    as impl_*.  traffic: counter bytes per launch (or None); traffic_ratio:
    counter bytes per step over the whole path's algorithmic bytes (read A,
    write A_rho, write the factors)."""
    launches = max(st["launches"], 1)
    t_launch = st["ms"] * 1e-3 / launches
    per_step = launches / steps
    f_val, f_vec = svd_work(m, p, n, rho_sum)
    alg = (f_val + f_vec) / per_step
    ach = alg / t_launch / 1e12
    impl = st["flops"] / launches
    out = {"bound": "mfma", "achieved": round(ach, 3), "peak": peak_tf, "unit": "TFLOP/s",
           "frac": round(ach / peak_tf, 4), "traffic": traffic_per_launch,
           "kernel": "jacobi_round", "launches": int(st["launches"]),
           "launches_per_step": round(per_step, 2), "avg_launch_ms": round(t_launch * 1e3, 4),
           "algorithmic_flops_per_launch": alg,
           "impl_flops_per_launch": impl, "impl_bytes_per_launch": st["bytes"] / launches,
           "impl_achieved": round(impl / t_launch / 1e12, 3),
           "impl_frac": round(impl / t_launch / 1e12 / peak_tf, 4),
           "pair_width": st["pair_width"], "pairs_rotating": st["pairs_rot"],
           "pairs_gram_only": st["pairs_gram"]}
    out["traffic_ratio"] = (round(traffic_per_launch * per_step / alg_bytes_step, 2)
                            if traffic_per_launch else None)
    return out


def climate_golden(m, p, n, eps):
    """The oracle's stored full-size results for this workload, or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "climate_fullsize.npz")
    if (m, p, n) != (512, 1024, 256) or not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as f:
        g = {k: f[k] for k in f.files}
    return g if float(g["eps"]) == eps else None


def vs_golden(res, g, A_host):
    """Rank differences and sampled-tube error against the oracle's stored
    result at the tolerance the run selected with (None if not stored)."""
    import numpy as np
    tag = None
    for key in g:
        if key.startswith("eps") and float(g[key]) == res.eps_sel:
            tag = key[3:]
            break
    if tag is None:
        return None
    rho = res.rho.cpu().numpy().astype(np.int64)
    pos = g["tube_pos"]
    got = np.stack([res.A_rec[int(a), int(b), :].double().cpu().numpy() for a, b in pos])
    nt = np.array([np.linalg.norm(A_host[int(a), int(b), :].astype(np.float64)) for a, b in pos])
    return {"eps_sel": res.eps_sel, "sum_abs_rank_diff": int(np.abs(rho - g[f"rho{tag}"]).sum()),
            "oracle_sum_rho": int(g[f"rho{tag}"].sum()),
            "oracle_rel_error": float(g[f"rel_error{tag}"]),
            "max_tube_rel_diff": float(np.max(np.linalg.norm(got - g[f"tubes{tag}"], axis=1) / nt)),
            "tubes": int(len(pos))}


def threshold_margin(res):
    """min(tau - nearest smaller square, nearest larger square - tau) / tau
    over the run's own squared singular values."""
    import numpy as np
    tau = float(res.stats[0].item())
    v = np.sort(res.s2.double().cpu().numpy().ravel())
    if not np.isfinite(tau) or tau <= 0:
        return None
    lo = v[v < tau].max() if np.any(v < tau) else -np.inf
    hi = v[v > tau].min() if np.any(v > tau) else np.inf
    return float(min(tau - lo, hi - tau) / tau)


def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"affinity_cpus": len(os.sched_getaffinity(0)), "model": model}


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


def blas_threads():
    import threadpoolctl
    return max((i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()), default=1)


def to_device(A, torch):
    """(m, p, n) Fortran-ordered numpy array -> column-major device tensor."""
    import numpy as np
    return torch.from_numpy(np.ascontiguousarray(A.transpose(2, 1, 0))).cuda().permute(2, 1, 0)


def timed(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) * 1e3 / steps


# ---------------------------------------------------------------------------
# climate (default)
# ---------------------------------------------------------------------------

def tune_single(a, Ad, M, precision, tuned, transform="dense"):
    """(block, tile) for one tensor: --block if given, else the autotuner's."""
    if a.block or a.no_tune:
        return a.block, 0
    from paper_2605_16058_amd import autotune
    t0 = time.perf_counter()
    ch = autotune.tune_tsvdm(Ad, M, mode="II", eps=a.eps, precision=precision,
                             transform=transform)
    tuned[precision] = {"block": ch.block, "tile": ch.tile,
                        "seconds": round(time.perf_counter() - t0, 2),
                        "measured_ms": {k: {str(c): round(v, 3) for c, v in t.items()}
                                        for k, t in ch.times.items()}}
    log(f"autotune {precision}: {tuned[precision]}")
    return ch.block, ch.tile


def cpu_baseline_climate(m, p, n_sample, eps):
    """The FP64 oracle, as it stands, on the first n_sample time steps of the
    same recipe (a bounded sample of the workload)."""
    import numpy as np

    import oracle
    import synth

    A = synth.climate_like(m, p, n_sample, rng=np.random.default_rng(2))
    M = synth.dct2_matrix(n_sample)
    t0 = time.perf_counter()
    res = oracle.tsvdm_ii(A.astype(np.float64), M, eps)
    dt = time.perf_counter() - t0
    return {"value": round(m * p * n_sample * 4 / dt / 1e9, 5), "unit": "GB/s",
            "cores": int(blas_threads()), "kind": "oracle",
            "sample": f"climate-like {m}x{p}x{n_sample} (the same recipe, first {n_sample} of 256 "
                      f"time steps), DCT-II {n_sample}, t-SVDM-II tol {eps}, the FP64 oracle as it "
                      f"stands (NumPy/LAPACK; cores = its BLAS threads); {dt:.2f} s wall, "
                      f"rel_err {res['rel_error']:.3e}",
            "seconds": round(dt, 3), "host": host_cpu()}


def transform_timing(a, Ad, M, torch, tf):
    """Forward transform alone, FP32 in and out: the FFT DCT (HBM bound:
    one read and one write of every element) beside the dense MFMA product,
    HIP events on the current stream."""
    from paper_2605_16058_amd import autotune, ops
    m, p, n = Ad.shape
    out = {}
    Y = ops.colmajor_empty(m, p, n, torch.float32, Ad.device)
    by = 2 * m * p * n * 4
    if n >= 2 and n <= 1024 and (n & (n - 1)) == 0:
        t = autotune.time_ms(lambda: ops.tsvdm_transform_dct(Ad, 3, compute="f32", out=Y), reps=5)
        out["dct_fft_ms"] = round(t, 4)
        out["dct_fft_GBs"] = round(by / (t * 1e-3) / 1e9, 1)
        out["dct_fft_hbm_frac"] = round(by / (t * 1e-3) / 1e9 / PEAK["hbm_GBs"], 4)
    Md = ops.device_matrix(M)
    ws = ops.Workspace(Ad.device)
    t = autotune.time_ms(lambda: ops.tsvdm_transform(Ad, Md, compute="f32", out_dtype=torch.float32,
                                                     out=Y, ws=ws), reps=5)
    out["dense_ttm_ms"] = round(t, 4)
    out["dense_ttm_TFs"] = round(2.0 * m * p * n * n / (t * 1e-3) / 1e12, 1)
    out["used"] = tf
    del Y
    log(f"transform timing: {out}")
    return out


def transform_only(a):
    """The dense transform Y = A x_3 M alone, back to back: the rate of the
    kernel by itself, for comparison with the stand-alone timing inside a
    benchmark run (which follows the timed steps)."""
    import numpy as np
    import torch

    import synth
    from paper_2605_16058_amd import autotune, ops
    m, p, n = (int(x) for x in a.shape.split(","))
    g = np.random.default_rng(5)
    Ad = ops.colmajor_empty(m, p, n, torch.float32, "cuda")
    Ad.copy_(torch.from_numpy(g.standard_normal((m, p, n)).astype(np.float32)))
    Md = ops.device_matrix(synth.haar_orthogonal(n, g))
    ws = ops.Workspace(Ad.device)
    out = {"workload": f"dense mode-3 transform {m}x{p}x{n}, Haar M, default tiles"}
    flops = 2.0 * m * p * n * n
    for compute, dt, peak in (("f32", torch.float32, PEAK["f32_TF"]), ("f64", torch.float64, PEAK["f64_TF"])):
        Y = ops.colmajor_empty(m, p, n, dt, "cuda")
        t = autotune.time_ms(lambda: ops.tsvdm_transform(Ad, Md, compute=compute, out_dtype=dt, out=Y, ws=ws),
                             reps=10, warmup=2)
        out[compute] = {"ms": round(t, 4), "TFLOP_s": round(flops / (t * 1e-3) / 1e12, 1),
                        "frac": round(flops / (t * 1e-3) / 1e12 / peak, 4)}
        del Y
    print(json.dumps(out), flush=True)
    return 0


def bench_climate(a, torch, lib):
    import numpy as np

    import synth
    from paper_2605_16058_amd import ops
    from paper_2605_16058_amd.pipeline import TSVDM

    m, p, n = (int(x) for x in a.shape.split(","))
    log(f"generating climate-like {m}x{p}x{n} FP32")
    A = synth.climate_like(m, p, n, rng=np.random.default_rng(2))
    M = synth.dct2_matrix(n)
    Ad = to_device(A, torch)
    in_bytes = m * p * n * 4
    gold = climate_golden(m, p, n, a.eps)

    # the DCT-II is applied by FFT (tsvdm_transform_dct) where the FFT covers
    # the precision (FP32 / FP64); the BF16 forms are transform precisions of
    # the dense product
    tf = a.transform if a.precision == "f32" else "dense"
    tuned = {}
    ch = tune_single(a, Ad, M, a.precision, tuned, tf)
    op_mix = TSVDM((m, p, n), M, mode="II", eps=a.eps, precision=a.precision, block=ch[0],
                   tile=ch[1], transform=tf)
    log(f"mixed ({a.precision}) warmup {a.warmup}, steps {a.steps}; guard {op_mix.guard}")
    for _ in range(a.warmup):
        op_mix(Ad)
    lib.tsvdm_stats_reset()
    lib.tsvdm_stats_enable(1)
    res_mix, ms_mix = timed(lambda: op_mix(Ad), a.steps, torch)
    lib.tsvdm_stats_enable(0)
    st = read_stats(lib)
    log(f"mixed: {ms_mix:.2f} ms/step; jacobi stats {st}")
    sha = kernel_src_sha()
    rho_mix = int(res_mix.offsets[-1].item())
    path = path_roofline(m, p, n, rho_mix, 4, PEAK["f32_TF"], tf, ms_mix)
    roof = svd_roofline(st, a.steps, m, p, n, rho_mix, PEAK["f32_TF"],
                        load_traffic(f"jacobi_round_f32_{m}x{p}x{n}", sha), path["algorithmic_bytes"])
    roof["src_sha"] = sha

    transform_info = transform_timing(a, Ad, M, torch, tf)

    out_f64 = {}
    if not a.no_f64:
        tf64 = a.transform
        ch64 = tune_single(a, Ad, M, "f64", tuned, tf64)
        op64 = TSVDM((m, p, n), M, mode="II", eps=a.eps, precision="f64", block=ch64[0],
                     tile=ch64[1], transform=tf64)
        log(f"fp64 warmup {a.warmup}, steps {a.steps}")
        for _ in range(a.warmup):
            op64(Ad)
        lib.tsvdm_stats_reset()
        lib.tsvdm_stats_enable(1)
        res64, ms64 = timed(lambda: op64(Ad), a.steps, torch)
        lib.tsvdm_stats_enable(0)
        st64 = read_stats(lib)
        log(f"fp64: {ms64:.2f} ms/step; jacobi stats {st64}")
        rho64 = int(res64.offsets[-1].item())
        path64 = path_roofline(m, p, n, rho64, 8, PEAK["f64_TF"], tf64, ms64)
        # the FP64 path's round launches are of two instances (the FP32
        # first stage on the Gram factors, the FP64 rotation form on the
        # rotated slices); their counter traffic is in the profile summary
        roof64 = svd_roofline(st64, a.steps, m, p, n, rho64, PEAK["f64_TF"], None,
                              path64["algorithmic_bytes"])
        roof64["kernel"] = "jacobi_round (FP32 first stage + FP64 rotation form)"
        roof64["src_sha"] = sha
        d = ops.tsvdm_error(res64.A_rec, res_mix.A_rec).double().cpu()
        nA = float(res64.err[1].cpu())
        out_f64 = {
            "fp64_GBs": round(in_bytes / (ms64 * 1e-3) / 1e9, 3),
            "fp64_ms_per_step": round(ms64, 3),
            "speedup_vs_fp64": round(ms64 / ms_mix, 3),
            "fp64_rel_error": res64.rel_error(),
            "fp64_sum_rho": rho64,
            "fp64_svd_status": int(res64.svd_status.item()),
            "fp64_threshold_margin": threshold_margin(res64),
            "fp64_compression_ratio": round(m * p * n / max(rho64 * (m + p + 1), 1), 4),
            "mixed_vs_fp64_rel_diff": math.sqrt(float(d[0]) / nA) if nA > 0 else 0.0,
            "mixed_vs_fp64_sum_abs_rank_diff": int((res64.rho.long() - res_mix.rho.long()).abs().sum()),
            "fp64_path_roofline": path64,
            "fp64_roofline": roof64,
        }
        if gold is not None:
            out_f64["fp64_vs_oracle"] = vs_golden(res64, gold, A)
        del res64, op64
        torch.cuda.empty_cache()

    cpu = None
    if not a.no_cpu_baseline:
        log(f"cpu baseline: oracle on {m}x{p}x{a.cpu_sample_n}")
        cpu = cpu_baseline_climate(m, p, a.cpu_sample_n, a.eps)

    return {
        "metric": METRIC,
        "value": round(in_bytes / (ms_mix * 1e-3) / 1e9, 3),
        "unit": "GB/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_mix, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if a.precision == "f32" else a.precision,
        "data": "synthetic",
        "config": {"workload": f"climate-like {m}x{p}x{n} FP32, DCT-II"
                               f"{' (FFT)' if tf == 'dct' else ''}, t-SVDM-II tol {a.eps}",
                   "m": m, "p": p, "n": n, "eps": a.eps, "eps_selected": res_mix.eps_sel,
                   "guard": op_mix.guard, "selections": res_mix.selections,
                   "precision": a.precision, "transform": tf, "autotune": tuned},
        "transform": transform_info,
        "rel_error": res_mix.rel_error(),
        "stated_rel_error": a.eps,
        "sum_rho": rho_mix,
        "compression_ratio": round(m * p * n / max(rho_mix * (m + p + 1), 1), 4),
        "threshold_margin": threshold_margin(res_mix),
        "svd_status": int(res_mix.svd_status.item()),
        "vs_oracle": vs_golden(res_mix, gold, A) if gold is not None else None,
        **out_f64,
        "path_roofline": path,
        "roofline": roof,
        "cpu_baseline": cpu,
    }


# ---------------------------------------------------------------------------
# certified selection
# ---------------------------------------------------------------------------

def bench_certify(a, torch, lib):
    """t-SVDM-II with the certified selection (slices provably below the
    threshold skip their SVD) against the full selection, FP32 path, on the
    climate-like recipe with a quieter field (--noise, default 1e-4 of the
    RMS): same ranks required, both timed."""
    import numpy as np

    import synth
    from paper_2605_16058_amd.pipeline import TSVDM, TSVDMd

    if a.order6:
        dims = (73, 144, 17, 4, 365, 2)
        log(f"generating the order-6 climate-like tensor {dims}, noise {a.noise}")
        A = synth.climate6_like(*dims[:3], days=dims[4], years=dims[5], noise=a.noise,
                                rng=np.random.default_rng(12))
        Ms = [synth.dct2_matrix(x) for x in dims[2:]]
        Ad = to_device_nd(A, torch)
        n = int(np.prod(dims[2:]))
        desc = f"order-6 climate-like {'x'.join(map(str, dims))} FP32, DCT-II along modes 3-6"
        block = a.block or 16
        kw = dict(mode="II", eps=a.eps, precision="f32", block=block)
        plain = TSVDMd(dims, Ms, **kw)
        cert = TSVDMd(dims, Ms, certify=True, **kw)
    else:
        m, p, n = (int(x) for x in a.shape.split(","))
        log(f"generating climate-like {m}x{p}x{n} FP32, noise {a.noise}")
        A = synth.climate_like(m, p, n, noise=a.noise, rng=np.random.default_rng(2))
        M = synth.dct2_matrix(n)
        Ad = to_device(A, torch)
        desc = f"climate-like {m}x{p}x{n} FP32, DCT-II (FFT)"
        block = a.block or 32
        kw = dict(mode="II", eps=a.eps, precision="f32", block=block, transform="dct")
        plain = TSVDM((m, p, n), M, **kw)
        cert = TSVDM((m, p, n), M, certify=True, **kw)
    in_bytes = A.size * 4
    del A
    for _ in range(a.warmup):
        plain(Ad)
        cert(Ad)
    r_plain, ms_plain = timed(lambda: plain(Ad), a.steps, torch)
    r_cert, ms_cert = timed(lambda: cert(Ad), a.steps, torch)
    same = bool(torch.equal(r_plain.rho.cpu(), r_cert.rho.cpu()))
    computed = int(r_cert.computed.sum().item())
    log(f"plain {ms_plain:.2f} ms, certified {ms_cert:.2f} ms ({computed}/{n} slices computed, "
        f"{r_cert.passes} rounds), ranks equal {same}")
    return {
        "metric": "input GB/s through certified t-SVDM-II (FP32)",
        "value": round(in_bytes / (ms_cert * 1e-3) / 1e9, 3),
        "unit": "GB/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_cert, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{desc}, noise {a.noise} of the RMS, t-SVDM-II tol {a.eps}, "
                               "certified selection",
                   "block": block},
        "plain_GBs": round(in_bytes / (ms_plain * 1e-3) / 1e9, 3),
        "plain_ms_per_step": round(ms_plain, 3),
        "speedup_vs_plain": round(ms_plain / ms_cert, 3),
        "slices_computed": computed, "slices": n, "rounds": r_cert.passes,
        "ranks_equal": same, "sum_rho": int(r_cert.offsets[-1].item()),
        "rel_error": r_cert.rel_error(), "plain_rel_error": r_plain.rel_error(),
        "roofline": None, "cpu_baseline": None,
    }


# ---------------------------------------------------------------------------
# ragged batch
# ---------------------------------------------------------------------------

def bench_ragged(a, torch, lib):
    import numpy as np

    import synth
    from paper_2605_16058_amd.pipeline import BatchTSVDM

    log(f"generating ragged batch ({a.batch_count} tensors)")
    w = synth.ragged_batch(count=a.batch_count)
    in_bytes = sum(x.size for x in w.A) * 4
    Ts = [to_device(x, torch) for x in w.A]
    nslices = sum(x.shape[2] for x in w.A)
    out = {}
    res = {}
    tuned = {}
    for prec in ([a.precision] + ([] if a.no_f64 else ["f64"])):
        blocks = tiles = None
        if not a.no_tune and not a.block:
            from paper_2605_16058_amd import autotune
            t0 = time.perf_counter()
            blocks, tiles, rep = autotune.tune_batch(Ts, w.M, w.mode, ks=w.k, epss=w.eps,
                                                     precision=prec)
            tuned[prec] = {"seconds": round(time.perf_counter() - t0, 2),
                           "blocks": {str(bw): blocks.count(bw) for bw in sorted(set(blocks))},
                           "tiles": {str(tl): tiles.count(tl) for tl in sorted(set(tiles))},
                           "measured_ms": {k: {str(c): round(v, 3) for c, v in t.items()}
                                           for k, t in rep.items()}}
            log(f"autotune {prec}: {tuned[prec]}")
        b = BatchTSVDM(Ts, w.M, w.mode, ks=w.k, epss=w.eps, precision=prec, block=a.block,
                       blocks=blocks, tiles=tiles)
        for _ in range(a.warmup):
            b.run()
        if prec == a.precision:
            lib.tsvdm_stats_reset()
            lib.tsvdm_stats_enable(1)
        _, ms = timed(lambda: b.run(), a.steps, torch)
        if prec == a.precision:
            lib.tsvdm_stats_enable(0)
            st = read_stats(lib)
            out["roofline"] = jacobi_roofline(st, PEAK["f32_TF"])
            out["roofline"]["src_sha"] = kernel_src_sha()
        log(f"ragged {prec}: {ms:.2f} ms/step")
        status = int(b.status.item())
        errs = b.rel_errors()
        res[prec] = (ms, status, errs, [r.clone() for r in b.rho])
        if prec == a.precision:
            # the method's SVD flops of one batch run (SURVEY 8(d) convention,
            # ranks read back), spread over the launches of the timed runs
            alg = 0.0
            for x, rr in zip(w.A, b.rho):
                m_, p_, n_ = x.shape
                fv, fr = svd_work(m_, p_, n_, int(rr.sum().item()))
                alg += fv + fr
            rf = out["roofline"]
            per = alg * a.steps / max(rf["launches"], 1)
            t = rf["avg_launch_ms"] * 1e-3
            ach = per / t / 1e12
            rf.update({"impl_bound": rf["bound"], "impl_achieved": rf["achieved"],
                       "impl_peak": rf["peak"], "impl_unit": rf["unit"], "impl_frac": rf["frac"],
                       "bound": "mfma", "achieved": round(ach, 3), "peak": PEAK["f32_TF"],
                       "unit": "TFLOP/s", "frac": round(ach / PEAK["f32_TF"], 4),
                       "algorithmic_flops_per_launch": per})
        del b
        torch.cuda.empty_cache()
    ms_mix, status, errs, rho_mix = res[a.precision]
    line = {
        "metric": "input GB/s through a batch of t-SVDM-I/II on uneven tensors",
        "value": round(in_bytes / (ms_mix * 1e-3) / 1e9, 3), "unit": "GB/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_mix, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": a.precision, "data": "synthetic",
        "config": {"workload": f"{a.batch_count} tensors, m,p~U[32,384], n~U[8,96], CP rank 2..32 "
                               "+ 1e-2 noise, Haar M, even: t-SVDM-I k=16, odd: t-SVDM-II tol 1e-2",
                   "tensors": a.batch_count, "slices": nslices, "input_GB": round(in_bytes / 1e9, 3),
                   "autotune": tuned},
        "status": status,
        "max_rel_error_modeII": max(e for e, md in zip(errs, w.mode) if md == "II"),
        "mean_rel_error_modeI": float(np.mean([e for e, md in zip(errs, w.mode) if md == "I"])),
        "roofline": out.get("roofline"),
        "cpu_baseline": None,
    }
    if "f64" in res:
        ms64, st64, errs64, rho64 = res["f64"]
        line["fp64_GBs"] = round(in_bytes / (ms64 * 1e-3) / 1e9, 3)
        line["fp64_ms_per_step"] = round(ms64, 3)
        line["speedup_vs_fp64"] = round(ms64 / ms_mix, 3)
        line["sum_abs_rank_diff_vs_fp64"] = int(sum(int((r1.long() - r2.long()).abs().sum())
                                                    for r1, r2 in zip(rho_mix, rho64)))
    if not a.no_cpu_baseline:
        import oracle
        k = a.cpu_sample_tensors
        t0 = time.perf_counter()
        for A, M, md, kk, ee in list(zip(w.A, w.M, w.mode, w.k, w.eps))[:k]:
            if md == "I":
                oracle.tsvdm_i(A.astype(np.float64), M, kk)
            else:
                oracle.tsvdm_ii(A.astype(np.float64), M, ee)
        dt = time.perf_counter() - t0
        sb = sum(x.size for x in w.A[:k]) * 4
        line["cpu_baseline"] = {"value": round(sb / dt / 1e9, 5), "unit": "GB/s",
                                "cores": int(blas_threads()), "kind": "oracle",
                                "sample": f"first {k} of the {a.batch_count} tensors "
                                          f"({sb / 1e9:.3f} GB FP32), {dt:.2f} s"}
    return line


# ---------------------------------------------------------------------------
# turbulence: transform precision sweep
# ---------------------------------------------------------------------------

def bench_turbulence(a, torch, lib):
    import numpy as np

    import synth
    from paper_2605_16058_amd import ops
    from paper_2605_16058_amd.pipeline import TSVDM

    shape = (2048, 1024, 256) if not a.small else (192, 128, 32)
    log(f"generating turbulence-like {shape}")
    w = synth.workload("turbulence", small=a.small)
    Ad = to_device(np.asfortranarray(w.A), torch)
    in_bytes = Ad.numel() * 4
    results = {}
    ref = None
    for prec in ["f64", "f32", "bf16x3", "bf16"]:
        op = TSVDM(shape, w.M, mode="II", eps=w.eps, precision=prec, block=a.block)
        for _ in range(a.warmup):
            op(Ad)
        res, ms = timed(lambda: op(Ad), a.steps, torch)
        rec = {"ms_per_step": round(ms, 2), "GBs": round(in_bytes / (ms * 1e-3) / 1e9, 3),
               "rel_error": res.rel_error(), "sum_rho": int(res.offsets[-1].item()),
               "svd_status": int(res.svd_status.item()), "guard": op.guard,
               "eps_selected": res.eps_sel, "selections": res.selections}
        if prec == "f64":
            ref = res
        else:
            d = ops.tsvdm_error(ref.A_rec, res.A_rec).double().cpu()
            nA = float(ref.err[1].cpu())
            rec["rel_diff_vs_fp64"] = math.sqrt(float(d[0]) / nA)
        results[prec] = rec
        log(f"turbulence {prec}: {rec}")
        if prec != "f64":
            del res
        del op
        torch.cuda.empty_cache()
    return {"metric": "input GB/s through t-SVDM-II per transform precision",
            "value": results["f32"]["GBs"], "unit": "GB/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": results["f32"]["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"turbulence-like {shape[0]}x{shape[1]}x{shape[2]} k^-5/3 "
                                   "field, Haar M, t-SVDM-II tol 1e-2"},
            "precisions": results, "roofline": None, "cpu_baseline": None}


# ---------------------------------------------------------------------------
# order-6 climate tensor (Section 4.1's reshaped time axis)
# ---------------------------------------------------------------------------

def to_device_nd(A, torch):
    """Fortran-ordered numpy array of any order -> column-major device tensor."""
    import numpy as np
    d = A.ndim
    rev = tuple(range(d - 1, -1, -1))
    return torch.from_numpy(np.ascontiguousarray(A.transpose(rev))).cuda().permute(*rev)


def bench_climate6(a, torch, lib):
    import numpy as np

    import synth
    from paper_2605_16058_amd import ops
    from paper_2605_16058_amd.pipeline import TSVDMd

    log("generating the order-6 climate-like tensor")
    w = synth.workload("climate6", small=a.small)
    dims = w.A.shape
    Ad = to_device_nd(w.A, torch)
    in_bytes = Ad.numel() * 4
    eps = w.eps
    n1, n2 = dims[0], dims[1]
    flat_dims = (n1, n2, dims[2], int(np.prod(dims[3:])))
    flat_M = [w.M[0], synth.dct2_matrix(flat_dims[3])]
    # the Jacobi block width of each path, timed on that path (the FP64
    # path's slice SVDs run other kernels than the FP32 path's)
    blocks = {"f32": a.block, "f64": a.block}
    tuned = {}
    for prec in ("f32",) + (() if a.no_f64 else ("f64",)):
        if blocks[prec] or a.no_tune:
            continue
        t = {}
        for b in (16, 32):
            op = TSVDMd(dims, w.M, mode="II", eps=eps, precision=prec, block=b)
            op(Ad)
            torch.cuda.synchronize()
            _, ms = timed(lambda: op(Ad), 1, torch)
            t[b] = round(ms, 2)
            del op
        blocks[prec] = min(t, key=t.get)
        tuned[prec] = {"block": blocks[prec], "measured_ms": t}
        log(f"{prec} block widths {t}: using {blocks[prec]}")

    def run(d_, Ms, prec, stats=False):
        op = TSVDMd(d_, Ms, mode="II", eps=eps, precision=prec, block=blocks[prec])
        # the same bytes viewed with other dimensions (column-major reshape)
        X = Ad.permute(*range(len(dims) - 1, -1, -1)).reshape(*reversed(d_)).permute(
            *range(len(d_) - 1, -1, -1))
        for _ in range(a.warmup):
            op(X)
        if stats:
            lib.tsvdm_stats_reset()
            lib.tsvdm_stats_enable(1)
        res, ms = timed(lambda: op(X), a.steps, torch)
        st = None
        if stats:
            lib.tsvdm_stats_enable(0)
            st = read_stats(lib)
        # the forward transforms alone
        Mdev = [ops.device_matrix(M) for M in Ms]
        comp, dt = ("f64", torch.float64) if prec == "f64" else ("f32", torch.float32)
        bufs = [ops.colmajor_empty_nd(d_, dt, "cuda") for _ in range(2)]

        def fwd():
            cur = X
            for j, kk in enumerate(range(3, len(d_) + 1)):
                out = bufs[j % 2]
                ops.tsvdm_transform_mode(cur, kk, Mdev[j], compute=comp, out_dtype=dt, out=out)
                cur = out
        fwd()
        _, ttm_ms = timed(fwd, a.steps, torch)
        del bufs
        return res, ms, ttm_ms, st

    log(f"order 6 {dims}, FP32 mixed")
    r6, ms6, ttm6, st = run(dims, w.M, "f32", stats=True)
    nsl = int(np.prod(dims[2:]))
    rho6 = int(r6.offsets[-1].item())
    # the FP32 path's slice SVDs: FP64 Gram, Cholesky and the in-LDS Jacobi
    # (min(n1, n2) <= 192) or the round kernel; roofline of that kernel by
    # the algorithmic SVD flops of the order-6 slices
    roof = svd_roofline(st, a.steps, n1, n2, nsl, rho6, PEAK["f32_TF"], None,
                        float(np.prod(dims)) * 8 + rho6 * (n1 + n2 + 1) * 4)
    roof["kernel"] = "pc_jacobi_lds" if min(n1, n2) <= 192 else "jacobi_round"
    roof["src_sha"] = kernel_src_sha()
    out = {}
    if not a.no_f64:
        log("order 6, FP64")
        r64, ms64, ttm64, _ = run(dims, w.M, "f64")
        d = ops.tsvdm_error(r64.A_rec, r6.A_rec).double().cpu()
        nA = float(r64.err[1].cpu())
        out = {"fp64_GBs": round(in_bytes / (ms64 * 1e-3) / 1e9, 3),
               "fp64_ms_per_step": round(ms64, 3), "speedup_vs_fp64": round(ms64 / ms6, 3),
               "fp64_rel_error": r64.rel_error(), "fp64_sum_rho": int(r64.offsets[-1].item()),
               "mixed_vs_fp64_rel_diff": math.sqrt(float(d[0]) / nA) if nA > 0 else 0.0}
        del r64
        torch.cuda.empty_cache()
    log(f"flat order 4 {flat_dims}, FP32 mixed")
    r4, ms4, ttm4, _ = run(flat_dims, flat_M, "f32")
    nslices = nsl
    rho4 = int(r4.offsets[-1].item())
    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        days = min(30, dims[4])
        sample = np.ascontiguousarray(w.A[:, :, :, :, :days, :1]).astype(np.float64)
        sample = np.asfortranarray(sample)
        Ms = [w.M[0], w.M[1], synth.dct2_matrix(days), np.eye(1)]
        t0 = time.perf_counter()
        oracle.tsvdm_d(sample, Ms, mode="II", eps=eps)
        dt_ = time.perf_counter() - t0
        sb = sample.size * 4
        cpu = {"value": round(sb / dt_ / 1e9, 5), "unit": "GB/s", "cores": int(blas_threads()),
               "kind": "oracle", "sample": f"the first {days} days of year 1 ({sample.shape}, DCT-II "
               f"along each mode >= 3, tol {eps}), {dt_:.2f} s"}
    return {
        "metric": "input GB/s through t-SVDM-II of an order-6 tensor (mixed-prec vs FP64 GPU)",
        "value": round(in_bytes / (ms6 * 1e-3) / 1e9, 3), "unit": "GB/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms6, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"order-6 climate-like {'x'.join(map(str, dims))} (lat, lon, level, "
                               f"time of day, day, year), DCT-II along modes 3-6, t-SVDM-II tol {eps}",
                   "slices": nslices, "autotune": tuned},
        "rel_error": r6.rel_error(), "sum_rho": rho6,
        "compression_ratio": round(float(np.prod(dims)) / max(rho6 * (n1 + n2 + 1), 1), 3),
        "ttm_forward_ms": round(ttm6, 3),
        **out,
        "flat_order4": {"dims": list(flat_dims), "GBs": round(in_bytes / (ms4 * 1e-3) / 1e9, 3),
                        "ms_per_step": round(ms4, 3), "ttm_forward_ms": round(ttm4, 3),
                        "rel_error": r4.rel_error(), "sum_rho": rho4,
                        "compression_ratio": round(float(np.prod(dims)) / max(rho4 * (n1 + n2 + 1), 1), 3),
                        "ttm_flop_ratio_vs_order6": round((flat_dims[2] + flat_dims[3]) / sum(dims[2:]), 2)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }


# ---------------------------------------------------------------------------
# cayley: gradient steps on the transform
# ---------------------------------------------------------------------------

def bench_cayley(a, torch, lib):
    import numpy as np

    import synth
    from paper_2605_16058_amd.pipeline import TruncLoss

    w = synth.workload("cayley", small=a.small)
    A = to_device(np.asfortranarray(w.A), torch)
    n = A.shape[2]
    K = torch.tensor(w.extra["K0"], device="cuda", dtype=torch.float64)
    I = torch.eye(n, dtype=torch.float64, device="cuda")

    def loss_and_grad(Kv):
        Kp = Kv.detach().clone().requires_grad_(True)
        Ks = 0.5 * (Kp - Kp.t())
        M = torch.linalg.solve(I - Ks, I + Ks)
        L = TruncLoss.apply(A, M, w.k)
        L.backward()
        return float(L.detach()), Kp.grad.detach()

    L0, g0 = loss_and_grad(K)
    eta = 0.05 / float(g0.norm())
    losses = [L0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.grad_steps):
        L, g = loss_and_grad(K)
        K = K - eta * g
        losses.append(L)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / a.grad_steps
    Ks = 0.5 * (K - K.t())
    M = torch.linalg.solve(I - Ks, I + Ks)
    ortho = float((M.t() @ M - I).abs().max())
    return {"metric": "gradient steps per second on the Cayley-parameterised transform",
            "value": round(1e3 / ms, 3), "unit": "steps/s", "n_gpus": 1,
            "steps": a.grad_steps, "warmup": 1, "ms_per_step": round(ms, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{tuple(A.shape)} CP rank 24 + 5% noise, k={w.k}, "
                                   "M = Cayley(K), lr 0.05/|grad0|"},
            "loss_first": losses[0], "loss_last": losses[-1],
            "loss_curve": [round(x, 6) for x in losses[:: max(1, len(losses) // 10)]],
            "max_orthogonality_drift": ortho, "roofline": None, "cpu_baseline": None}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="climate",
                    choices=["climate", "ragged", "turbulence", "cayley", "climate6", "certify"])
    ap.add_argument("--precision", default="f32", choices=["f32", "bf16x3", "bf16"])
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--shape", default="512,1024,256")
    ap.add_argument("--transform", default="dct", choices=["dct", "dense"],
                    help="climate: apply the DCT-II by FFT (dct) or as a dense MFMA product")
    ap.add_argument("--noise", type=float, default=1e-4,
                    help="certify: relative noise of the climate-like field")
    ap.add_argument("--order6", action="store_true",
                    help="certify: the order-6 climate-like tensor instead of the 3-way one")
    ap.add_argument("--no-f64", action="store_true", help="skip the FP64 comparison path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=64)
    ap.add_argument("--cpu-sample-tensors", type=int, default=16)
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--grad-steps", type=int, default=50)
    ap.add_argument("--small", action="store_true", help="test-size turbulence / cayley / climate6 inputs")
    ap.add_argument("--block", type=int, default=0, help="fixed Jacobi block width (skips tuning)")
    ap.add_argument("--no-tune", action="store_true", help="library defaults, no autotuner")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--transform-only", action="store_true",
                    help="only time the dense mode-3 transform on --shape (Haar M, default tiles, "
                         "FP32 and FP64, 10 calls each), as a kernel measured by itself")
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

    if a.transform_only:
        return transform_only(a)

    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); every box here has a "
              "single GPU and the multi-GPU layout is a design note, not a built path.",
              file=sys.stderr)
        return 2

    import torch

    from paper_2605_16058_amd import _lib

    lib = _lib.load()
    fn = {"climate": bench_climate, "ragged": bench_ragged, "turbulence": bench_turbulence,
          "cayley": bench_cayley, "climate6": bench_climate6, "certify": bench_certify}[a.workload]
    line = fn(a, torch, lib)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
