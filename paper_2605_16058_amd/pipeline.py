"""t-SVDM-I / t-SVDM-II end to end on one GPU, and the autograd wrapper.

The pipeline chains the C-ABI calls: transform (Algorithm 1's first step),
slice SVDs, rank selection (Section 3.3 / Algorithm 2), factor packing
(Section 3.4) and reconstruction with the back-transform (Section 2.1), then
the FP64 error report.  Torch only allocates device memory and provides the
stream.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

import torch

from . import ops
from ._lib import GRAM_JACOBI, GRAM_MAX_R

PRECISIONS = {
    # name: (TTM compute, Jacobi dtype)
    "f64": ("f64", torch.float64),
    "f32": ("f32", torch.float32),
    "bf16x3": ("bf16x3", torch.float32),
    "bf16": ("bf16", torch.float32),
}


# Stated bound on ||A_rec - A_rec(FP64)||_F / ||A||_F for each precision (the
# parity tests hold every path to it); plain BF16 has none (it is reported).
RECON_BOUND = {"f64": 0.0, "f32": 3e-5, "bf16x3": 1e-4, "bf16": None}


GUARDS = ("measure", "bound", "off")


def _guard_mode(guard):
    if guard is True:
        return "measure"
    if guard is False or guard is None:
        return "off"
    if guard not in GUARDS:
        raise ValueError(f"guard must be one of {GUARDS}")
    return guard


def selection_eps(eps, precision, guard="measure"):
    """The tolerance a t-SVDM-II run selects with first.  Algorithm 2 bounds
    the tail of the squared singular values the run computed: the truncation
    alone leaves an error below eps relative to ||A||.  A reduced-precision
    path adds its rounding, at most delta = RECON_BOUND[precision] relative
    to ||A||, so selecting with eps - delta keeps ||A - A_rec|| / ||A|| < eps
    by the triangle inequality: guard "bound" does that up front.  Guard
    "measure" (TSVDM, TSVDMd) selects with eps and checks the measured error
    afterwards (next_selection_eps); "off" selects with eps and checks
    nothing.  FP64 (delta = 0) and plain BF16 (no stated bound) select with
    eps under every guard."""
    g = _guard_mode(guard)
    d = RECON_BOUND[precision]
    if g != "bound" or not d:
        return float(eps)
    if float(eps) <= d:
        raise ValueError(f"eps must exceed the {precision} reconstruction bound {d}")
    return float(eps) - d


def next_selection_eps(eps, eps_cur, rel, stats, precision, rounds):
    """Guard "measure": the tolerance of the next selection after a run with
    tolerance eps_cur measured rel >= eps.  The excess of the measured error
    over the run's own prediction sqrt(discarded / total) is rounding; the
    next selection tightens eps_cur by twice that excess, and a third one
    falls back to eps - delta (the triangle-inequality bound)."""
    d = RECON_BOUND[precision] or 0.0
    st = stats.double().cpu()
    pred = float((st[1] / st[2]).sqrt()) if float(st[2]) > 0 else 0.0
    nxt = eps_cur - 2.0 * max(rel - pred, 0.0)
    if rounds >= 2 or not (0.0 < nxt < eps_cur):
        nxt = min(eps_cur, eps - d) if d else eps_cur * (1.0 - 1e-6)
    return max(nxt, 1e-300)




def resolve_svd(svd, precision, r, certify=False):
    """Slice SVD form: "jacobi" rotates the slice itself (any precision);
    "gram" (FP32 Jacobi dtype only, min(m, p) <= 1024) runs the Jacobi on
    the Cholesky factor of the slice's FP64 Gram matrix and forms the long-
    side factor by one product (tsvdm_slice_svd_gram); "precond" (FP64 path,
    min(m, p) <= 1024) rotates the slice by the Gram form's vectors, made
    orthonormal in FP64, and finishes with the rotation form, to its
    accuracy (tsvdm_slice_svd_precond).  "auto":
    "gram" on the reduced-precision paths where it applies, "precond" on the
    FP64 path where it applies, else "jacobi"."""
    if svd not in ("auto", "jacobi", "gram", "precond"):
        raise ValueError("svd must be 'auto', 'jacobi', 'gram' or 'precond'")
    fits = r <= GRAM_MAX_R and not certify
    ok = PRECISIONS[precision][1] == torch.float32 and fits
    ok64 = PRECISIONS[precision][1] == torch.float64 and fits
    if svd == "gram" and not ok:
        raise ValueError("svd='gram' needs an FP32 Jacobi path, min(m, p) <= 1024 and no certify")
    if svd == "precond" and not ok64:
        raise ValueError("svd='precond' needs the FP64 path, min(m, p) <= 1024 and no certify")
    if svd == "auto":
        return "gram" if ok else ("precond" if ok64 else "jacobi")
    return svd


@dataclass
class Result:
    A_rec: torch.Tensor
    rho: torch.Tensor
    offsets: torch.Tensor
    U_pk: torch.Tensor
    G_pk: torch.Tensor
    S_pk: torch.Tensor
    s2: torch.Tensor
    stats: torch.Tensor          # t-SVDM-II: tau, discarded, total, J
    err: torch.Tensor            # [sum (A - A_rec)^2, sum A^2]
    svd_status: torch.Tensor
    pack_status: torch.Tensor
    capacity: int
    computed: torch.Tensor | None = None   # certified selection: slices given an SVD
    passes: int = 0                         # certified selection: SVD rounds
    eps_sel: float | None = None            # t-SVDM-II: the tolerance selected with
    selections: int = 1                     # t-SVDM-II: selections made (guard "measure")

    def rel_error(self) -> float:
        e = self.err.double().cpu()
        return float((e[0] / e[1]).sqrt()) if e[1] > 0 else 0.0


class TSVDM:
    """Reusable operator for one shape, transform and precision.

    mode "I" keeps rank k on every slice, mode "II" uses the global relative
    tolerance eps.  capacity="max" sizes the packed factors for r*n triplets
    (no host synchronisation); "exact" reads sum(rho) back first (one sync),
    like the paper's exact-size allocation.  transform="dct" applies M, which
    must then be the orthonormal DCT-II (or None), by FFT (tsvdm_transform_dct)
    instead of the dense product: forward, and after the transform-domain
    low-rank product (tsvdm_lowrank) backward; precision f64 or f32 only.

    svd: "auto", "jacobi", "gram" or "precond" (see resolve_svd).  gram_jacobi: where
    the Gram form's Jacobi on the factor runs, "auto" (in LDS for
    min(m, p) <= 128, else the block rounds), "rounds" or "lds".

    guard (mode "II"; see selection_eps): "measure" (default) selects with
    eps and, if the measured relative error of the result is not below eps
    (rounding of a reduced-precision path on top of a truncation error just
    below eps), repeats the selection, packing and reconstruction with a
    tighter tolerance (next_selection_eps; the slice SVDs are not redone);
    "bound" selects with eps - delta at once; "off" checks nothing.
    Result.eps_sel is the tolerance of the result, Result.selections the
    number of selections made.

    certify=True (mode "II") runs the certified selection: only slices whose
    energy could reach the threshold get an SVD.  The first round computes
    the slices outside the lowest-energy set holding theta * eps^2 of the
    total (theta = 0.5); every other slice enters the selection as its
    energy, and if all those stand-ins fall strictly below the resulting tau,
    the ranks are those of the full method (the skipped slices get rank 0).
    Otherwise the stand-ins at or above tau get their SVD and the selection
    is repeated, at most max_passes rounds before the remaining slices are
    all computed.  Result.computed marks the slices given an SVD; s2 holds
    the energy stand-ins for the others.
    """

    def __init__(self, shape, M, mode="II", k=None, eps=None, precision="f64",
                 block=0, max_sweeps=0, tol=0.0, host_poll=True, capacity="max",
                 device="cuda", check_m=True, tile=0, transform="dense", certify=False,
                 theta=0.5, max_passes=3, guard="measure", svd="auto", gram_jacobi="auto"):
        self.m, self.p, self.n = (int(x) for x in shape)
        self.r = min(self.m, self.p)
        self.svd = resolve_svd(svd, precision, self.r, certify)
        if gram_jacobi not in GRAM_JACOBI:
            raise ValueError(f"gram_jacobi must be one of {list(GRAM_JACOBI)}")
        self.gram_jacobi = gram_jacobi
        # the certified selection chooses its ranks inside its SVD rounds:
        # it takes the up-front bound instead of measuring
        self.guard = _guard_mode(guard)
        if certify and self.guard == "measure":
            self.guard = "bound"
        if mode not in ("I", "II"):
            raise ValueError("mode must be 'I' or 'II'")
        if mode == "I" and (k is None or int(k) < 1):
            raise ValueError("mode I needs k >= 1")
        if mode == "II" and (eps is None or not (0.0 < float(eps) < 1.0)):
            raise ValueError("mode II needs 0 < eps < 1")
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {list(PRECISIONS)}")
        self.mode, self.k, self.eps = mode, k, eps
        self.precision = precision
        self.eps_sel = selection_eps(eps, precision, self.guard) if mode == "II" else None
        self.ttm_compute, self.dtype = PRECISIONS[precision]
        if transform not in ("dense", "dct"):
            raise ValueError("transform must be 'dense' or 'dct'")
        self.transform = transform
        if transform == "dct":
            if precision not in ("f64", "f32"):
                raise ValueError("transform='dct' needs precision f64 or f32")
            n = self.n
            if n < 2 or n > 1024 or (n & (n - 1)) != 0:
                raise ValueError("transform='dct' needs n a power of two in [2, 1024]")
            q = np.arange(n)[:, None]
            j = np.arange(n)[None, :]
            C = np.sqrt(2.0 / n) * np.cos(np.pi * q * (2 * j + 1) / (2 * n))
            C[0] /= np.sqrt(2.0)
            if M is None:
                M = C
            elif np.max(np.abs(np.asarray(M, np.float64) - C)) > 1e-12:
                raise ValueError("transform='dct' needs M to be the orthonormal DCT-II")
        self.c2 = ops.check_transform(M) if check_m else 1.0
        self.Mdev = ops.device_matrix(M, device)
        self.block, self.max_sweeps, self.tol, self.host_poll = block, max_sweeps, tol, host_poll
        self.tile = tile
        if certify and mode != "II":
            raise ValueError("certify applies to mode II")
        if not (0.0 < float(theta) <= 1.0) or int(max_passes) < 1:
            raise ValueError("theta must lie in (0, 1] and max_passes be >= 1")
        self.certify, self.theta, self.max_passes = bool(certify), float(theta), int(max_passes)
        self.capacity_mode = capacity
        self.device = device
        self.ws = ops.Workspace(device)

    def __call__(self, A: torch.Tensor) -> Result:
        A = ops.as_colmajor(A)
        if tuple(A.shape) != (self.m, self.p, self.n):
            raise ValueError("shape mismatch")
        m, p, n, r = self.m, self.p, self.n, self.r
        out_dt = self.dtype
        # 1. transform (FP32 -> FP64 up-cast fused into the TTM load)
        if self.transform == "dct":
            A_hat = ops.tsvdm_transform_dct(A, 3, inverse=False, compute=self.ttm_compute,
                                            out_dtype=self.dtype)
        else:
            A_hat = ops.tsvdm_transform(A, self.Mdev, transpose=False, scale=1.0,
                                        compute=self.ttm_compute, out_dtype=self.dtype, ws=self.ws,
                                        tile=self.tile)
        # 2. slice SVDs
        computed, passes, shift = None, 0, None
        if self.certify:
            W, s2, svd_status, rho, offsets, stats, computed, passes = self._certified(A_hat)
        elif self.svd == "gram":
            W, s2, shift, svd_status = ops.tsvdm_slice_svd_gram(
                A_hat, self.block, self.max_sweeps, self.tol, self.host_poll, ws=self.ws,
                jacobi=self.gram_jacobi)
        elif self.svd == "precond":
            # the orthogonalised vectors land in a new tensor, packed from below
            A_hat, W, s2, svd_status = ops.tsvdm_slice_svd_precond(
                A_hat, self.block, self.max_sweeps, self.tol, self.host_poll, ws=self.ws)
        else:
            W, s2, svd_status = ops.tsvdm_slice_svd(A_hat, self.block, self.max_sweeps, self.tol,
                                                    self.host_poll, ws=self.ws)
        eps_cur = self.eps_sel
        selections = 0
        back = self.ttm_compute if self.ttm_compute != "f64" else "f64"
        while True:
            selections += 1
            # 3. ranks (the certified selection made them with its SVD rounds)
            if self.mode == "I":
                rho, offsets = ops.tsvdm_truncate_rank(self.k, r, n, self.device)
                stats = torch.full((4,), float("nan"), dtype=torch.float64, device=self.device)
            elif not (self.certify and selections == 1):
                rho, offsets, stats = ops.tsvdm_truncate_tol(s2, eps_cur, ws=self.ws)
            if self.capacity_mode == "exact":
                cap = int(offsets[n].item())
            elif self.mode == "I":
                cap = min(int(self.k), r) * n
            else:
                cap = r * n
            # 4. factors
            if self.svd == "gram":
                U_pk, G_pk, S_pk, pack_status = ops.tsvdm_pack_gram(A_hat, W, s2, shift, rho, offsets,
                                                                    cap, ws=self.ws)
            else:
                U_pk, G_pk, S_pk, pack_status = ops.tsvdm_pack(A_hat, W, s2, rho, offsets, cap,
                                                               ws=self.ws)
            # 5. reconstruct + back-transform (M^{-1} = M^T / c^2)
            if self.transform == "dct":
                C_hat = ops.tsvdm_lowrank(U_pk, G_pk, rho, offsets, cap, (m, p, n))
                A_rec = ops.tsvdm_transform_dct(C_hat, 3, inverse=True, compute=back, out_dtype=out_dt)
                del C_hat
            else:
                A_rec = ops.tsvdm_reconstruct(U_pk, G_pk, rho, offsets, cap, self.Mdev, (m, p, n),
                                              scale=1.0 / self.c2, out_dtype=out_dt, compute=back,
                                              ws=self.ws, tile=self.tile)
            # 6. error report; guard "measure": the result must be below eps
            err = ops.tsvdm_error(A, A_rec, ws=self.ws)
            if self.mode != "II" or self.guard != "measure" or selections >= 3:
                break
            e = err.double().cpu()
            rel = float((e[0] / e[1]).sqrt()) if float(e[1]) > 0 else 0.0
            if rel < self.eps:
                break
            eps_cur = next_selection_eps(self.eps, eps_cur, rel, stats, self.precision, selections)
            del U_pk, G_pk, S_pk, A_rec
        del W
        return Result(A_rec, rho, offsets, U_pk, G_pk, S_pk, s2, stats, err, svd_status,
                      pack_status, cap, computed, passes, eps_cur, selections)

    def _certified(self, A_hat):
        return certified_svd(A_hat, self.eps_sel, self.theta, self.max_passes, self.block,
                             self.max_sweeps, self.tol, self.host_poll, self.ws)


def certified_svd(A_hat, eps, theta, max_passes, block, max_sweeps, tol, host_poll, ws):
    """Slice SVDs and t-SVDM-II ranks with the certified selection (see
    TSVDM): returns W, s2, status, rho, offsets, stats, computed, rounds."""
    n = A_hat.shape[2]
    dev = A_hat.device
    W, s2, svd_status = ops.tsvdm_slice_svd_outputs(A_hat)
    E = ops.tsvdm_slice_energy(A_hat)
    # round 1: everything outside the lowest-energy set holding theta eps^2
    run, _, _ = ops.tsvdm_truncate_tol(E.view(n, 1), eps * theta ** 0.5, ws=ws)
    computed = run.clone()
    spare = torch.empty_like(run)
    certified = torch.zeros(1, dtype=torch.int32, device=dev)
    passes = 0
    while True:
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        ops.tsvdm_slice_svd_subset(A_hat, run, W, s2, st, block, max_sweeps, tol, host_poll, ws=ws)
        svd_status = torch.minimum(svd_status, st)
        passes += 1
        ops.tsvdm_certify_lump(E, computed, s2)
        rho, offsets, stats = ops.tsvdm_truncate_tol(s2, eps, ws=ws)
        if passes > max_passes:
            break   # the forced round computed every remaining slice
        ops.tsvdm_certify_check(E, stats, computed, spare, passes == max_passes, certified)
        if int(certified.item()):
            break
        run, spare = spare, run
    return W, s2, svd_status, rho, offsets, stats, computed, passes


def tsvdm(A, M, mode="II", k=None, eps=None, precision="f64", **kw) -> Result:
    """One-shot t-SVDM-I (mode="I", k) or t-SVDM-II (mode="II", eps)."""
    op = TSVDM(tuple(A.shape), M, mode=mode, k=k, eps=eps, precision=precision,
               device=A.device, **kw)
    return op(A)


class TSVDMd:
    """t-SVDM-I / t-SVDM-II of an order-d tensor n_1 x n_2 x n_3 x ... x n_d
    (Section 2.1, footnote; Section 3.1): one transform M_k per mode k >= 3,
    applied mode by mode (tsvdm_transform_mode, one launch per mode), then the
    slice SVDs, rank selection and packing over the N = n_3...n_d frontal
    slices as for three modes, the transform-domain low-rank product
    (tsvdm_lowrank) and the back-transforms mode by mode.  For d = 3 it runs
    the same kernels as TSVDM.  Result: as TSVDM (s2, rho, offsets over the
    N slices in column-major order; A_rec of shape dims).
    """

    def __init__(self, dims, Ms, mode="II", k=None, eps=None, precision="f64", block=0,
                 max_sweeps=0, tol=0.0, host_poll=True, device="cuda", tile=0, certify=False,
                 theta=0.5, max_passes=3, guard="measure", svd="auto", gram_jacobi="auto"):
        self.dims = tuple(int(x) for x in dims)
        if certify and mode != "II":
            raise ValueError("certify applies to mode II")
        self.certify, self.theta, self.max_passes = bool(certify), float(theta), int(max_passes)
        if len(self.dims) < 3:
            raise ValueError("order d >= 3")
        if len(Ms) != len(self.dims) - 2:
            raise ValueError("one transform per mode k >= 3")
        if mode not in ("I", "II"):
            raise ValueError("mode must be 'I' or 'II'")
        if mode == "I" and (k is None or int(k) < 1):
            raise ValueError("mode I needs k >= 1")
        if mode == "II" and (eps is None or not (0.0 < float(eps) < 1.0)):
            raise ValueError("mode II needs 0 < eps < 1")
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {list(PRECISIONS)}")
        self.mode, self.k, self.eps, self.precision = mode, k, eps, precision
        self.guard = _guard_mode(guard)
        if certify and self.guard == "measure":
            self.guard = "bound"
        self.eps_sel = selection_eps(eps, precision, self.guard) if mode == "II" else None
        self.ttm_compute, self.dtype = PRECISIONS[precision]
        self.c2 = [ops.check_transform(M) for M in Ms]
        self.Mdev = [ops.device_matrix(M, device) for M in Ms]
        self.block, self.max_sweeps, self.tol, self.host_poll = block, max_sweeps, tol, host_poll
        self.tile, self.device = tile, device
        self.m, self.p = self.dims[0], self.dims[1]
        self.N = 1
        for x in self.dims[2:]:
            self.N *= x
        self.r = min(self.m, self.p)
        self.svd = resolve_svd(svd, precision, self.r, certify)
        if gram_jacobi not in GRAM_JACOBI:
            raise ValueError(f"gram_jacobi must be one of {list(GRAM_JACOBI)}")
        self.gram_jacobi = gram_jacobi
        self.ws = ops.Workspace(device)

    def __call__(self, A: torch.Tensor) -> Result:
        A = ops.as_colmajor_nd(A)
        if tuple(A.shape) != self.dims:
            raise ValueError("shape mismatch")
        d, m, p, N, r = len(self.dims), self.m, self.p, self.N, self.r
        dt, comp = self.dtype, self.ttm_compute
        bufs = [ops.colmajor_empty_nd(self.dims, dt, self.device) for _ in range(2 if d > 3 else 1)]
        # 1. transforms along modes 3..d
        cur = A
        for j, kk in enumerate(range(3, d + 1)):
            out = bufs[j % len(bufs)]
            ops.tsvdm_transform_mode(cur, kk, self.Mdev[j], transpose=False, scale=1.0, compute=comp,
                                     out_dtype=dt, out=out, ws=self.ws, tile=self.tile)
            cur = out
        A_hat = cur.permute(*range(d - 1, -1, -1)).reshape(N, p, m).permute(2, 1, 0)
        # 2. slice SVDs over the N frontal slices
        computed, passes, shift = None, 0, None
        if self.certify:
            W, s2, svd_status, rho, offsets, stats, computed, passes = certified_svd(
                A_hat, self.eps_sel, self.theta, self.max_passes, self.block, self.max_sweeps,
                self.tol, self.host_poll, self.ws)
        elif self.svd == "gram":
            W, s2, shift, svd_status = ops.tsvdm_slice_svd_gram(
                A_hat, self.block, self.max_sweeps, self.tol, self.host_poll, ws=self.ws,
                jacobi=self.gram_jacobi)
        elif self.svd == "precond":
            # the orthogonalised vectors land in a new tensor, packed from below
            A_hat, W, s2, svd_status = ops.tsvdm_slice_svd_precond(
                A_hat, self.block, self.max_sweeps, self.tol, self.host_poll, ws=self.ws)
        else:
            W, s2, svd_status = ops.tsvdm_slice_svd(A_hat, self.block, self.max_sweeps, self.tol,
                                                    self.host_poll, ws=self.ws)
        # buffers of the back path that never alias A_hat (a repeated
        # selection packs from it again)
        free = [b for b in bufs if b.data_ptr() != cur.data_ptr()]
        while len(free) < (1 if d == 3 else 2):
            free.append(ops.colmajor_empty_nd(self.dims, dt, self.device))
        eps_cur = self.eps_sel
        selections = 0
        while True:
            selections += 1
            # 3. ranks (the certified selection made them with its SVD rounds)
            if self.mode == "I":
                rho, offsets = ops.tsvdm_truncate_rank(self.k, r, N, self.device)
                stats = torch.full((4,), float("nan"), dtype=torch.float64, device=self.device)
                cap = min(int(self.k), r) * N
            else:
                if not (self.certify and selections == 1):
                    rho, offsets, stats = ops.tsvdm_truncate_tol(s2, eps_cur, ws=self.ws)
                cap = r * N
            # 4. factors
            if self.svd == "gram":
                U_pk, G_pk, S_pk, pack_status = ops.tsvdm_pack_gram(A_hat, W, s2, shift, rho, offsets,
                                                                    cap, ws=self.ws)
            else:
                U_pk, G_pk, S_pk, pack_status = ops.tsvdm_pack(A_hat, W, s2, rho, offsets, cap,
                                                               ws=self.ws)
            # 5. transform-domain low-rank product, then back-transforms mode by mode
            C3 = free[0].permute(*range(d - 1, -1, -1)).reshape(N, p, m).permute(2, 1, 0)
            ops.tsvdm_lowrank(U_pk, G_pk, rho, offsets, cap, (m, p, N), out=C3)
            A_rec = ops.colmajor_empty_nd(self.dims, dt, self.device)
            cb = free[0]
            back = list(range(3, d + 1))
            for j, kk in enumerate(back):
                last = j == len(back) - 1
                out = A_rec if last else (free[1] if cb.data_ptr() == free[0].data_ptr() else free[0])
                ops.tsvdm_transform_mode(cb, kk, self.Mdev[kk - 3], transpose=True,
                                         scale=1.0 / self.c2[kk - 3], compute=comp, out_dtype=dt, out=out,
                                         ws=self.ws, tile=self.tile)
                cb = out
            # 6. error report; guard "measure": the result must be below eps
            err = ops.tsvdm_error(A, A_rec, ws=self.ws)
            if self.mode != "II" or self.guard != "measure" or selections >= 3:
                break
            e = err.double().cpu()
            rel = float((e[0] / e[1]).sqrt()) if float(e[1]) > 0 else 0.0
            if rel < self.eps:
                break
            eps_cur = next_selection_eps(self.eps, eps_cur, rel, stats, self.precision, selections)
            del U_pk, G_pk, S_pk, A_rec
        del W
        return Result(A_rec, rho, offsets, U_pk, G_pk, S_pk, s2, stats, err, svd_status,
                      pack_status, cap, computed, passes, eps_cur, selections)


class BatchTSVDM:
    """Many independent tensors of any shapes through one batch plan.

    tensors: list of column-major device tensors (m_t, p_t, n_t), all of one
    dtype; Ms: list of n_t x n_t transforms; modes: "I"/"II" per tensor with
    ks / epss.  Each stage of the hot path is one launch over all tensors
    (see tsvdm_batch_plan_create); run() returns the device status word.
    keep_factors=True allocates packed factors per tensor (worst-case
    capacity) so they can be read back; otherwise they stay in the workspace.
    blocks / tiles: optional per-tensor Jacobi block widths and transform
    tile shapes (0 = the plan's choice), e.g. from autotune.tune_batch().
    guard: "bound" (default) or "off" (see selection_eps): one plan runs
    without host decisions, so the mode "II" tensors of a reduced-precision
    batch select with eps - delta up front; the tolerances are in eps_sel.
    """

    def __init__(self, tensors, Ms, modes, ks=None, epss=None, precision="f32", block=0,
                 max_sweeps=0, keep_factors=False, reconstruct=True, device="cuda",
                 blocks=None, tiles=None, guard="bound"):
        import ctypes

        from . import _lib
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {list(PRECISIONS)}")
        ttm_compute, dtype = PRECISIONS[precision]
        self.dtype = dtype
        cnt = len(tensors)
        ks = ks or [None] * cnt
        epss = epss or [None] * cnt
        blocks = blocks or [0] * cnt
        tiles = tiles or [0] * cnt
        self.tensors = [ops.as_colmajor(t) for t in tensors]
        in_dt = self.tensors[0].dtype
        if any(t.dtype != in_dt for t in self.tensors):
            raise TypeError("all tensors of a batch must share one dtype")
        self.Mdev, self.rho, self.offsets, self.stats, self.A_rec, self.err = [], [], [], [], [], []
        self.U_pk, self.G_pk, self.S_pk, self.capacity = [], [], [], []
        if _guard_mode(guard) == "measure":
            raise ValueError("a batch takes guard 'bound' or 'off'")
        self.eps_sel = [selection_eps(e, precision, guard) if md == "II" else None
                        for e, md in zip(epss, modes)]
        items = (_lib.BatchItem * cnt)()
        for t, (A, M, mode) in enumerate(zip(self.tensors, Ms, modes)):
            m, p, n = A.shape
            r = min(m, p)
            c2 = ops.check_transform(M)
            Md = ops.device_matrix(M, device)
            rho = torch.empty(n, dtype=torch.int32, device=device)
            off = torch.empty(n + 1, dtype=torch.int64, device=device)
            stats = torch.zeros(4, dtype=torch.float64, device=device)
            Arec = ops.colmajor_empty(m, p, n, dtype, device) if reconstruct else None
            err = torch.zeros(2, dtype=torch.float64, device=device) if reconstruct else None
            it = items[t]
            it.m, it.p, it.n = m, p, n
            it.A = A.data_ptr()
            it.M = Md.data_ptr()
            it.inv_scale = 1.0 / c2
            it.mode = 1 if mode == "I" else 2
            it.block = int(blocks[t])
            it.ttm_tile = int(tiles[t])
            it.reserved = 0
            it.k = int(ks[t] or 1)
            it.eps = float(self.eps_sel[t] or 0.5)
            it.rho, it.offsets, it.stats = rho.data_ptr(), off.data_ptr(), stats.data_ptr()
            if keep_factors:
                cap = (min(int(ks[t]), r) if mode == "I" else r) * n
                U = torch.empty(m * cap, dtype=dtype, device=device)
                G = torch.empty(p * cap, dtype=dtype, device=device)
                S = torch.empty(cap, dtype=dtype, device=device)
                it.U_pk, it.G_pk, it.S_pk, it.capacity = U.data_ptr(), G.data_ptr(), S.data_ptr(), cap
                self.U_pk.append(U); self.G_pk.append(G); self.S_pk.append(S)
                self.capacity.append(cap)
            else:
                it.U_pk = it.G_pk = it.S_pk = None
                it.capacity = 0
            it.A_rec = Arec.data_ptr() if Arec is not None else None
            it.err = err.data_ptr() if err is not None else None
            self.Mdev.append(Md); self.rho.append(rho); self.offsets.append(off)
            self.stats.append(stats); self.A_rec.append(Arec); self.err.append(err)
        self._items = items
        plan = ctypes.c_void_p()
        wsb = ctypes.c_size_t(0)
        _lib.call("tsvdm_batch_plan_create", ctypes.cast(items, ctypes.c_void_p), cnt,
                  ops._DT[in_dt], ops._DT[dtype], ops._COMPUTE[ttm_compute], int(block),
                  int(max_sweeps), ctypes.byref(plan), ctypes.byref(wsb))
        self.plan = plan
        self.ws = torch.empty(max(int(wsb.value), 256), dtype=torch.uint8, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)

    def run(self, host_poll=True, use_graph=False):
        import ctypes

        from . import _lib
        _lib.call("tsvdm_batch_run", self.plan, ctypes.c_void_p(self.ws.data_ptr()),
                  self.ws.numel(), int(bool(host_poll)), int(bool(use_graph)),
                  ctypes.c_void_p(self.status.data_ptr()), ops._stream())
        return self.status

    def rel_errors(self):
        out = []
        for e in self.err:
            e = e.double().cpu()
            out.append(float((e[0] / e[1]).sqrt()) if e[1] > 0 else 0.0)
        return out

    def __del__(self):
        try:
            from . import _lib
            if getattr(self, "plan", None) is not None and self.plan.value:
                _lib.load().tsvdm_batch_plan_destroy(self.plan)
                self.plan = None
        except Exception:
            pass


class TruncLoss(torch.autograd.Function):
    """L(A, M) = sum of the squared singular values dropped by a rank-k
    truncation of every slice of A x_3 M, with a hand-written adjoint
    (tsvdm_backward) for both A and M.  M is an n x n FP64 device tensor;
    compose it with any torch parameterisation (e.g. a Cayley map) to learn
    the transform.  The factors are recomputed in backward, not stored."""

    @staticmethod
    def forward(ctx, A, M, k):
        Mdev = M.detach().t().contiguous()  # column-major bytes
        loss, _, _, status = ops.tsvdm_backward(A.detach(), Mdev, int(k), 1.0,
                                                want_dA=False, want_dM=False)
        ctx.save_for_backward(A, M)
        ctx.k = int(k)
        return loss[0].to(torch.float64)

    @staticmethod
    def backward(ctx, g):
        A, M = ctx.saved_tensors
        Mdev = M.detach().t().contiguous()
        _, dA, dM, _ = ops.tsvdm_backward(A.detach(), Mdev, ctx.k, 1.0,
                                          want_dA=ctx.needs_input_grad[0],
                                          want_dM=ctx.needs_input_grad[1])
        gA = (dA * g.to(dA.dtype)) if dA is not None else None
        gM = (dM * g) if dM is not None else None
        return gA, gM, None
