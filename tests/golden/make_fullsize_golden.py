"""Write the oracle's results for the full-size benchmark workloads.

Calls only the FP64 oracle (oracle/) and the seeded input generators
(synth/); nothing here touches the GPU path.  For each workload it stores
  S          r x n singular values of every frontal slice of A x_3 M
  rho, tau, J, discarded, total, rel_error, compression   t-SVDM-II at eps
  tube_pos   sampled (row, column) positions of the reconstruction
  tubes      A_rho(row, column, :) at those positions
and the same ranks, statistics and tubes at each extra tolerance listed in
EXTRA_EPS (the tighter tolerances a mixed-precision path selects with).

Usage:  python tests/golden/make_fullsize_golden.py climate [turbulence]
Runs for minutes: the oracle's mode-3 product is a plain double loop.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

# eps - delta for the FP32 (delta = 3e-5) and split-BF16 (delta = 1e-4) paths
EXTRA_EPS = {"climate": [1e-3 - 3e-5], "turbulence": [1e-2 - 3e-5, 1e-2 - 1e-4]}
TUBES = 64


def path(name: str) -> str:
    return os.path.join(HERE, f"{name}_fullsize.npz")


def make(name: str) -> str:
    t0 = time.time()
    w = synth.workload(name)
    A = np.asarray(w.A, dtype=np.float64)      # the FP32 input, as the GPU sees it
    m, p, n = A.shape
    print(f"[{name}] {m}x{p}x{n}: oracle t-SVDM-II at eps {w.eps}", flush=True)
    A_hat = O.to_transform_domain(A, w.M)
    print(f"[{name}] transform {time.time() - t0:.0f} s", flush=True)
    U, S, V = O.slice_svd(A_hat)
    del A_hat
    print(f"[{name}] slice SVDs {time.time() - t0:.0f} s", flush=True)
    g = np.random.default_rng(2024)
    pos = np.stack([g.integers(0, m, TUBES), g.integers(0, p, TUBES)], axis=1)
    out = {"S": S, "eps": np.float64(w.eps), "tube_pos": pos}
    for tag, eps in [("", w.eps)] + [(f"_x{j}", e) for j, e in enumerate(EXTRA_EPS.get(name, []))]:
        rho, info = O.ranks_tolerance(S, eps)
        A_rec = O.reconstruct(O.truncated_factors(U, S, V, rho), w.M, (m, p, n))
        out[f"rho{tag}"] = rho
        out[f"eps{tag}"] = np.float64(eps)
        for k in ("tau", "J", "discarded", "total"):
            out[f"{k}{tag}"] = np.float64(info[k])
        out[f"rel_error{tag}"] = np.float64(O.rel_error(A, A_rec))
        out[f"compression{tag}"] = np.float64(O.compression_ratio(m, p, n, rho))
        out[f"tubes{tag}"] = np.stack([A_rec[a, b, :] for a, b in pos])
        print(f"[{name}] eps {eps}: sum rho {int(rho.sum())}, rel error {out[f'rel_error{tag}']:.9e}, "
              f"{time.time() - t0:.0f} s", flush=True)
        del A_rec
    np.savez_compressed(path(name), **out)
    return path(name)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["climate"]:
        print(make(nm), flush=True)
