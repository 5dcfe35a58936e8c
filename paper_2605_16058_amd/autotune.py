"""Measured choice of the transform tile shape and the Jacobi block width.

Both knobs change only the speed, never the result (the Jacobi block width
changes the rotation order, so results agree to rounding, not bit for bit).
Candidates run on the caller's own device data through the C ABI and are
timed with HIP events on the current stream; nothing is predicted from a
model.  Shapes are grouped into buckets:

* transform: by n (rounded up to a power of two), since n sets the tile's
  slice width and the K loop; the row count only changes the tile count;
* Jacobi: by r = min(m, p) (rounded up to a power of two) and by whether the
  Jacobi vectors are rows or columns.

Winners are kept in a JSON cache keyed by device name, precision and bucket
(path: ``$TSVDM_AUTOTUNE_CACHE``, else
``~/.cache/paper_2605_16058_amd/autotune.json``; ``cache=False`` disables
it) and reused by later calls and processes.  A candidate replaces the
incumbent only when it is faster by more than ``margin`` (default 3%), so
timing noise does not flip choices.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import torch

# transform tiles (rows x slices): 64x64, 128x32, 256x16 (16 slices per
# wave), 128x64, 256x32 (32), 128x128, 256x64 (64), 64x64 as 2 x 2 waves of
# 32 x 32 (8); the FP64 form has no registers for waves of more than 32 slices
TTM_TILES = (1, 2, 3, 4, 5, 6, 7, 8)
TTM_TILES_F64 = (1, 2, 3, 4, 8)
JACOBI_BLOCKS = (16, 32)


def ttm_tiles(precision: str) -> tuple:
    """Transform tile candidates for one precision."""
    return TTM_TILES_F64 if precision == "f64" else TTM_TILES


def _pow2_ceil(x: int) -> int:
    x = max(int(x), 1)
    return 1 << (x - 1).bit_length()


def ttm_bucket(n: int) -> str:
    return f"n{min(_pow2_ceil(n), 256)}"


def jacobi_bucket(m: int, p: int) -> str:
    r = min(m, p)
    return f"r{min(_pow2_ceil(r), 4096)}{'rows' if m < p else 'cols'}"


def default_block(m: int, p: int) -> int:
    """The library's choice for block = 0 on one tensor."""
    return 32 if min(m, p) >= 256 else 16


def default_tile(n: int, precision: str = "f64") -> int:
    """The library's choice for tile = 0: by n, and for the FP32-operand
    precisions wider waves once n > 32."""
    if n <= 16:
        return 3
    if n <= 32:
        return 2
    if precision == "f64":
        return 8
    return 4 if n <= 64 else 6


class Cache:
    """JSON file of measured winners; ``path=None`` keeps them in memory."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            try:
                with open(path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    @staticmethod
    def default_path() -> str:
        return os.environ.get("TSVDM_AUTOTUNE_CACHE") or os.path.join(
            os.path.expanduser("~"), ".cache", "paper_2605_16058_amd", "autotune.json")

    @staticmethod
    def key(kind: str, precision: str, bucket: str) -> str:
        dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
        return f"{dev}|{kind}|{precision}|{bucket}"

    def get(self, kind, precision, bucket):
        v = self.data.get(self.key(kind, precision, bucket))
        return None if v is None else int(v["choice"])

    def put(self, kind, precision, bucket, choice, times):
        self.data[self.key(kind, precision, bucket)] = {
            "choice": int(choice), "ms": {str(k): round(v, 4) for k, v in times.items()}}
        if self.path:
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _cache(cache) -> Cache:
    if isinstance(cache, Cache):
        return cache
    if cache is False:
        return Cache(None)
    return Cache(Cache.default_path() if cache in (None, True) else str(cache))


def time_ms(fn, reps: int = 3, warmup: int = 1) -> float:
    """Median device time of fn() in ms, HIP events on the current stream."""
    for _ in range(warmup):
        fn()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def pick(times: dict, incumbent, margin: float = 0.03):
    """Fastest candidate, unless it beats the incumbent by no more than margin."""
    best = min(times, key=times.get)
    if incumbent in times and times[best] >= (1.0 - margin) * times[incumbent]:
        return incumbent
    return best


@dataclass
class Choice:
    block: int
    tile: int
    times: dict = field(default_factory=dict)


def tune_tsvdm(A, M, mode="II", k=None, eps=None, precision="f32", cache=None, reps=2,
               margin=0.03, transform="dense") -> Choice:
    """Block width and tile shape for one tensor shape, timed on t-SVDM runs of A.

    With transform="dct" (the FFT transform, which has no tile shape) only the
    block width is tuned, on runs with that transform."""
    from .pipeline import TSVDM
    m, p, n = A.shape
    c = _cache(cache)
    jb, tb = jacobi_bucket(m, p), ttm_bucket(n)
    block, tile = c.get("jacobi", precision, jb), c.get("ttm", precision, tb)
    times = {}
    if block is None:
        t = {}
        for b in JACOBI_BLOCKS:
            op = TSVDM(A.shape, M, mode=mode, k=k, eps=eps, precision=precision, block=b,
                       device=A.device, transform=transform)
            t[b] = time_ms(lambda: op(A), reps=reps)
        block = pick(t, default_block(m, p), margin)
        c.put("jacobi", precision, jb, block, t)
        times["jacobi"] = t
    if transform == "dct":
        tile = 0
    elif tile is None:
        from . import ops
        from .pipeline import PRECISIONS
        compute, dtype = PRECISIONS[precision]
        Md = ops.device_matrix(M, A.device)
        Y = ops.colmajor_empty(m, p, n, dtype, A.device)
        t = {}
        for s in ttm_tiles(precision):
            t[s] = time_ms(lambda: ops.tsvdm_transform(A, Md, compute=compute, out_dtype=dtype,
                                                       out=Y, tile=s), reps=max(reps, 5))
        tile = pick(t, default_tile(n, precision), margin)
        c.put("ttm", precision, tb, tile, t)
        times["ttm"] = t
    return Choice(block, tile, times)


def _sample(indices, limit):
    """Up to `limit` evenly spaced members of a list (deterministic)."""
    if len(indices) <= limit:
        return list(indices)
    step = len(indices) / limit
    return [indices[int(i * step)] for i in range(limit)]


def tune_batch(tensors, Ms, modes, ks=None, epss=None, precision="f32", cache=None,
               sample=64, reps=2, margin=0.03):
    """Per-tensor (blocks, tiles) for BatchTSVDM, chosen per bucket.

    The objective is the device time of whole batch runs over an evenly
    spaced sample of at most `sample` tensors, so each choice is judged the
    way the batch runs it: all buckets share every launch.  Jacobi buckets
    are tuned first (largest total work first), then transform buckets, one
    bucket at a time with the others held at their current choice.
    Returns (blocks, tiles, report) with report = {bucket: {candidate: ms}}.
    """
    from .pipeline import BatchTSVDM
    cnt = len(tensors)
    c = _cache(cache)
    ks = ks or [None] * cnt
    epss = epss or [None] * cnt
    jb = [jacobi_bucket(t.shape[0], t.shape[1]) for t in tensors]
    tb = [ttm_bucket(t.shape[2]) for t in tensors]
    idx = _sample(list(range(cnt)), sample)
    sub = [tensors[i] for i in idx]
    sub_M = [Ms[i] for i in idx]
    sub_modes = [modes[i] for i in idx]
    sub_k = [ks[i] for i in idx]
    sub_e = [epss[i] for i in idx]
    rmax = max(min(t.shape[0], t.shape[1]) for t in tensors)
    plan_block = 32 if rmax >= 256 else 16
    jchoice = {b: c.get("jacobi", precision, b) for b in set(jb)}
    tchoice = {b: c.get("ttm", precision, b) for b in set(tb)}
    todo_j = [b for b, v in jchoice.items() if v is None]
    todo_t = [b for b, v in tchoice.items() if v is None]
    for b in todo_j:
        jchoice[b] = plan_block
    for b in todo_t:
        tchoice[b] = default_tile(int(b[1:]), precision)
    report = {}

    def run_time():
        blocks = [jchoice[jb[i]] for i in idx]
        tiles = [tchoice[tb[i]] for i in idx]
        bt = BatchTSVDM(sub, sub_M, sub_modes, ks=sub_k, epss=sub_e, precision=precision,
                        blocks=blocks, tiles=tiles, device=sub[0].device)
        return time_ms(lambda: bt.run(host_poll=True), reps=reps)

    def work(b):
        return sum(min(t.shape[0], t.shape[1]) ** 2 * max(t.shape[0], t.shape[1]) * t.shape[2]
                   for t, key in zip(sub, (jb[i] for i in idx)) if key == b)

    for b in sorted(todo_j, key=work, reverse=True):
        if work(b) == 0:
            continue
        t = {}
        for cand in JACOBI_BLOCKS:
            jchoice[b] = cand
            t[cand] = run_time()
        jchoice[b] = pick(t, plan_block, margin)
        c.put("jacobi", precision, b, jchoice[b], t)
        report[b] = t
    for b in todo_t:
        if not any(tb[i] == b for i in idx):
            continue
        t = {}
        for cand in ttm_tiles(precision):
            tchoice[b] = cand
            t[cand] = run_time()
        tchoice[b] = pick(t, default_tile(int(b[1:]), precision), margin)
        c.put("ttm", precision, b, tchoice[b], t)
        report[b] = t
    blocks = [jchoice.get(jb[i]) or plan_block for i in range(cnt)]
    tiles = [tchoice.get(tb[i]) or 0 for i in range(cnt)]
    return blocks, tiles, report
