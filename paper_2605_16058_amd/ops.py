"""Torch-facing wrappers of the C ABI (device memory and streams only).

Each function marshals torch tensors into the matching ``tsvdm_*`` call;
every arithmetic step runs in libtsvdm's HIP kernels.  Tensors use the
column-major layout of the paper (Section 3): an m x p x n tensor is a torch
view of shape (m, p, n) with strides (1, m, m*p), see ``colmajor_empty``.
"""
from __future__ import annotations

import ctypes
from ctypes import byref, c_double, c_void_p

import torch

from . import _lib
from ._lib import BF16, BF16X3, F32, F64

_DT = {torch.float64: F64, torch.float32: F32}
_COMPUTE = {"f64": F64, "f32": F32, "bf16": BF16, "bf16x3": BF16X3}


def _dt(t: torch.Tensor) -> int:
    try:
        return _DT[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype} (float64 or float32)") from None


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def colmajor_empty(m: int, p: int, n: int, dtype, device="cuda") -> torch.Tensor:
    """Uninitialised m x p x n tensor with strides (1, m, m*p)."""
    return torch.empty((n, p, m), dtype=dtype, device=device).permute(2, 1, 0)


def colmajor_empty_nd(dims, dtype, device="cuda") -> torch.Tensor:
    """Uninitialised tensor of shape dims with column-major strides (mode 1 fastest)."""
    d = len(dims)
    return torch.empty(tuple(reversed(dims)), dtype=dtype, device=device).permute(*range(d - 1, -1, -1))


def is_colmajor_nd(t: torch.Tensor) -> bool:
    stride = 1
    for size, st in zip(t.shape, t.stride()):
        if size != 1 and st != stride:
            return False
        stride *= size
    return True


def as_colmajor_nd(t: torch.Tensor) -> torch.Tensor:
    """t itself if column-major, else a column-major copy."""
    if is_colmajor_nd(t):
        return t
    out = colmajor_empty_nd(tuple(t.shape), t.dtype, t.device)
    out.copy_(t)
    return out


def is_colmajor(t: torch.Tensor) -> bool:
    m, p, n = t.shape
    return t.stride() == (1, m, m * p) or t.numel() <= 1


def as_colmajor(t: torch.Tensor) -> torch.Tensor:
    """Return t itself if it already has the column-major strides, else a
    column-major copy (the only case in which the wrappers copy data)."""
    if t.dim() != 3:
        raise ValueError("expected an m x p x n tensor")
    if is_colmajor(t):
        return t
    out = colmajor_empty(*t.shape, dtype=t.dtype, device=t.device)
    out.copy_(t)
    return out


class Workspace:
    """Grow-only device scratch buffer reused across calls on one stream."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf

    def args(self, nbytes: int):
        b = self.get(nbytes)
        return c_void_p(b.data_ptr()), ctypes.c_size_t(b.numel())


_default_ws = {}


def _ws(ws):
    if ws is not None:
        return ws
    dev = torch.cuda.current_device()
    if dev not in _default_ws:
        _default_ws[dev] = Workspace(f"cuda:{dev}")
    return _default_ws[dev]


def check_transform(M, tol: float = 1e-10) -> float:
    """Host check that M = c*Q with Q orthogonal; returns c^2."""
    Mh = torch.as_tensor(M, dtype=torch.float64).cpu()
    Mc = Mh.t().contiguous()  # column-major bytes of M
    c2 = c_double(0.0)
    _lib.call("tsvdm_check_transform", c_void_p(Mc.data_ptr()), Mh.shape[0], float(tol), byref(c2))
    return c2.value


def device_matrix(M, device="cuda") -> torch.Tensor:
    """n x n FP64 matrix as a column-major device buffer (transposed view)."""
    Mh = torch.as_tensor(M, dtype=torch.float64)
    return Mh.t().contiguous().to(device)


# ---------------------------------------------------------------- entry points

def tsvdm_transform(X, Mdev, transpose=False, scale=1.0, compute="f64", out_dtype=None,
                    out=None, ws=None, tile=0):
    """Y = X x_3 (scale * op(M)); Mdev from device_matrix().  tile: 0 = by n
    and compute, 1..8 = 64x64, 128x32, 256x16, 128x64, 256x32, 128x128,
    256x64 (rows x slices), 64x64 in 2 x 2 waves."""
    X = as_colmajor(X)
    m, p, n = X.shape
    odt = out_dtype or (torch.float64 if compute == "f64" else torch.float32)
    Y = out if out is not None else colmajor_empty(m, p, n, odt, X.device)
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_transform_workspace_size", n))
    _lib.call("tsvdm_transform", _ptr(X), _dt(X), _ptr(Y), _dt(Y), m, p, n, _ptr(Mdev),
              int(bool(transpose)), float(scale), _COMPUTE[compute], int(tile), wp, wn, _stream())
    return Y


def tsvdm_transform_mode(X, k, Mdev, transpose=False, scale=1.0, compute="f64", out_dtype=None,
                         out=None, ws=None, tile=0):
    """Y = X x_k (scale * op(M)) for a column-major order-d tensor X (3 <= k <= d)."""
    X = as_colmajor_nd(X)
    dims = tuple(int(x) for x in X.shape)
    odt = out_dtype or (torch.float64 if compute == "f64" else torch.float32)
    Y = out if out is not None else colmajor_empty_nd(dims, odt, X.device)
    if tuple(Y.shape) != dims or not is_colmajor_nd(Y):
        raise ValueError("out must be a column-major tensor of the input's shape")
    d = len(dims)
    dims_c = (ctypes.c_int64 * d)(*dims)
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_transform_workspace_size", dims[k - 1]))
    _lib.call("tsvdm_transform_mode", _ptr(X), _dt(X), _ptr(Y), _dt(Y), d, dims_c, int(k),
              _ptr(Mdev), int(bool(transpose)), float(scale), _COMPUTE[compute], int(tile), wp, wn,
              _stream())
    return Y


def tsvdm_transform_dct(X, k=3, inverse=False, compute="f64", out_dtype=None, out=None):
    """Y = X x_k C (or C^T with inverse) for the orthonormal DCT-II C, by FFT.

    X is a column-major tensor of order >= 3; n_k must be a power of two in
    [2, 1024].  compute ("f64" or "f32") is the FFT's arithmetic."""
    if compute not in ("f64", "f32"):
        raise ValueError("compute must be 'f64' or 'f32'")
    X = as_colmajor_nd(X)
    dims = tuple(int(x) for x in X.shape)
    odt = out_dtype or (torch.float64 if compute == "f64" else torch.float32)
    Y = out if out is not None else colmajor_empty_nd(dims, odt, X.device)
    if tuple(Y.shape) != dims or not is_colmajor_nd(Y):
        raise ValueError("out must be a column-major tensor of the input's shape")
    d = len(dims)
    dims_c = (ctypes.c_int64 * d)(*dims)
    _lib.call("tsvdm_transform_dct", _ptr(X), _dt(X), _ptr(Y), _dt(Y), d, dims_c, int(k),
              int(bool(inverse)), _COMPUTE[compute], _stream())
    return Y


def tsvdm_lowrank(U_pk, G_pk, rho, offsets, capacity, shape, out=None):
    """C-hat with slice i = U_i G_i (transform domain, no back-transform)."""
    m, p, n = shape
    dt = U_pk.dtype
    C = out if out is not None else colmajor_empty(m, p, n, dt, U_pk.device)
    _lib.call("tsvdm_lowrank", _ptr(U_pk), _ptr(G_pk), _DT[dt], m, p, n, _ptr(rho), _ptr(offsets),
              int(capacity), _ptr(C), _stream())
    return C


def tsvdm_slice_svd(A_hat, block=0, max_sweeps=0, tol=0.0, host_poll=True, ws=None):
    """In-place one-sided Jacobi on every slice.  Returns (W, s2, status)."""
    if not is_colmajor(A_hat):
        raise ValueError("A_hat must be column-major (it is overwritten in place)")
    m, p, n = A_hat.shape
    r = min(m, p)
    W = torch.empty((n, r, r), dtype=A_hat.dtype, device=A_hat.device)
    s2 = torch.empty((n, r), dtype=torch.float64, device=A_hat.device)
    status = torch.zeros(1, dtype=torch.int32, device=A_hat.device)
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_slice_svd_workspace_size", m, p, n, _dt(A_hat)))
    _lib.call("tsvdm_slice_svd", _ptr(A_hat), _dt(A_hat), m, p, n, _ptr(W), _ptr(s2), _ptr(status),
              int(block), int(max_sweeps), float(tol), int(bool(host_poll)), wp, wn, _stream())
    return W, s2, status


def tsvdm_slice_svd_precond(A_hat, block=0, max_sweeps=0, tol=0.0, host_poll=True, ws=None):
    """Rotation-form slice SVDs preconditioned by the Gram form (A_hat is only
    read).  Returns (X, W, s2, status): X holds the orthogonalised vectors
    that tsvdm_slice_svd would leave in A_hat, W and s2 as there."""
    if not is_colmajor(A_hat):
        raise ValueError("A_hat must be column-major")
    m, p, n = A_hat.shape
    r = min(m, p)
    X = colmajor_empty(m, p, n, A_hat.dtype, A_hat.device)
    W = torch.empty((n, r, r), dtype=A_hat.dtype, device=A_hat.device)
    s2 = torch.empty((n, r), dtype=torch.float64, device=A_hat.device)
    status = torch.zeros(1, dtype=torch.int32, device=A_hat.device)
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_slice_svd_precond_workspace_size", m, p, n, _dt(A_hat)))
    _lib.call("tsvdm_slice_svd_precond", _ptr(A_hat), _dt(A_hat), m, p, n, _ptr(X), _ptr(W), _ptr(s2),
              _ptr(status), int(block), int(max_sweeps), float(tol), int(bool(host_poll)), wp, wn, _stream())
    return X, W, s2, status


def tsvdm_slice_svd_gram(A_hat, block=0, max_sweeps=0, tol=0.0, host_poll=True, ws=None, jacobi="auto"):
    """Slice SVDs of an FP32 tensor by way of the FP64 Gram matrix (A_hat is
    only read).  Returns (B, s2, shift, status): B (n, r, r) FP32 holds the
    orthogonalised columns of each slice's Cholesky factor, s2 the squared
    singular values, shift the per-slice Cholesky shift.  jacobi: "auto",
    "rounds" or "lds", where the Jacobi on the factor runs."""
    if not is_colmajor(A_hat) or A_hat.dtype != torch.float32:
        raise ValueError("A_hat must be a column-major FP32 tensor")
    if jacobi not in _lib.GRAM_JACOBI:
        raise ValueError(f"jacobi must be one of {list(_lib.GRAM_JACOBI)}")
    m, p, n = A_hat.shape
    r = min(m, p)
    B = torch.empty((n, r, r), dtype=torch.float32, device=A_hat.device)
    s2 = torch.empty((n, r), dtype=torch.float64, device=A_hat.device)
    shift = torch.empty(n, dtype=torch.float64, device=A_hat.device)
    status = torch.zeros(1, dtype=torch.int32, device=A_hat.device)
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_slice_svd_gram_workspace_size", m, p, n))
    _lib.call("tsvdm_slice_svd_gram", _ptr(A_hat), m, p, n, _ptr(B), _ptr(s2), _ptr(shift), _ptr(status),
              int(block), int(max_sweeps), float(tol), _lib.GRAM_JACOBI[jacobi], int(bool(host_poll)), wp, wn,
              _stream())
    return B, s2, shift, status


def tsvdm_pack_gram(A_hat, B, s2, shift, rho, offsets, capacity, ws=None):
    """Packed factors from the output of tsvdm_slice_svd_gram (FP32)."""
    m, p, n = A_hat.shape
    cap = int(capacity)
    dev = A_hat.device
    U_pk = torch.empty(max(m * cap, 1), dtype=torch.float32, device=dev)
    G_pk = torch.empty(max(p * cap, 1), dtype=torch.float32, device=dev)
    S_pk = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_pack_workspace_size", m, p, n))
    _lib.call("tsvdm_pack_gram", _ptr(A_hat), _ptr(B), _ptr(s2), _ptr(shift), m, p, n, _ptr(rho),
              _ptr(offsets), cap, _ptr(U_pk), _ptr(G_pk), _ptr(S_pk), _ptr(status), wp, wn, _stream())
    return U_pk, G_pk, S_pk, status


def tsvdm_truncate_rank(k, r, n, device="cuda"):
    rho = torch.empty(n, dtype=torch.int32, device=device)
    offsets = torch.empty(n + 1, dtype=torch.int64, device=device)
    _lib.call("tsvdm_truncate_rank", int(k), int(r), int(n), _ptr(rho), _ptr(offsets), _stream())
    return rho, offsets


def tsvdm_slice_svd_outputs(A_hat):
    """Uninitialised W (n, r, r), s2 (n, r) and a status word for A_hat."""
    m, p, n = A_hat.shape
    r = min(m, p)
    W = torch.empty((n, r, r), dtype=A_hat.dtype, device=A_hat.device)
    s2 = torch.empty((n, r), dtype=torch.float64, device=A_hat.device)
    status = torch.zeros(1, dtype=torch.int32, device=A_hat.device)
    return W, s2, status


def tsvdm_slice_svd_subset(A_hat, run, W, s2, status, block=0, max_sweeps=0, tol=0.0,
                           host_poll=True, ws=None):
    """Jacobi on the slices with run[i] != 0 (device int32[n]); the others keep
    their A_hat, W and s2 entries."""
    if not is_colmajor(A_hat):
        raise ValueError("A_hat must be column-major (it is overwritten in place)")
    m, p, n = A_hat.shape
    r = min(m, p)
    if tuple(W.shape) != (n, r, r) or tuple(s2.shape) != (n, r) or run.numel() != n:
        raise ValueError("W, s2 or run do not match A_hat")
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_slice_svd_workspace_size", m, p, n, _dt(A_hat)))
    _lib.call("tsvdm_slice_svd_subset", _ptr(A_hat), _dt(A_hat), m, p, n, _ptr(W), _ptr(s2),
              _ptr(status), _ptr(run), int(block), int(max_sweeps), float(tol),
              int(bool(host_poll)), wp, wn, _stream())
    return status


def tsvdm_slice_energy(A_hat):
    """E[i] = ||A_hat[:, :, i]||_F^2 in FP64."""
    A_hat = as_colmajor(A_hat)
    m, p, n = A_hat.shape
    E = torch.empty(n, dtype=torch.float64, device=A_hat.device)
    _lib.call("tsvdm_slice_energy", _ptr(A_hat), _dt(A_hat), m, p, n, _ptr(E), _stream())
    return E


def tsvdm_certify_lump(E, computed, s2):
    n, r = s2.shape
    _lib.call("tsvdm_certify_lump", _ptr(E), _ptr(computed), _ptr(s2), r, n, _stream())


def tsvdm_certify_check(E, stats, computed, run_next, force, certified):
    n = E.numel()
    _lib.call("tsvdm_certify_check", _ptr(E), _ptr(stats), _ptr(computed), _ptr(run_next), n,
              int(bool(force)), _ptr(certified), _stream())


def tsvdm_truncate_tol(s2, eps, ws=None):
    """s2: (n, r) FP64 device tensor (slice-major).  Returns rho, offsets,
    stats = [tau, discarded, total, J]."""
    n, r = s2.shape
    rho = torch.empty(n, dtype=torch.int32, device=s2.device)
    offsets = torch.empty(n + 1, dtype=torch.int64, device=s2.device)
    stats = torch.empty(4, dtype=torch.float64, device=s2.device)
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_truncate_tol_workspace_size", r, n))
    _lib.call("tsvdm_truncate_tol", _ptr(s2.contiguous()), r, n, float(eps), _ptr(rho), _ptr(offsets),
              _ptr(stats), wp, wn, _stream())
    return rho, offsets, stats


def tsvdm_pack(A_hat, W, s2, rho, offsets, capacity, ws=None):
    m, p, n = A_hat.shape
    dt = A_hat.dtype
    cap = int(capacity)
    U_pk = torch.empty(max(m * cap, 1), dtype=dt, device=A_hat.device)
    G_pk = torch.empty(max(p * cap, 1), dtype=dt, device=A_hat.device)
    S_pk = torch.empty(max(cap, 1), dtype=dt, device=A_hat.device)
    status = torch.zeros(1, dtype=torch.int32, device=A_hat.device)
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_pack_workspace_size", m, p, n))
    _lib.call("tsvdm_pack", _ptr(A_hat), _ptr(W), _ptr(s2), _dt(A_hat), m, p, n, _ptr(rho),
              _ptr(offsets), cap, _ptr(U_pk), _ptr(G_pk), _ptr(S_pk), _ptr(status), wp, wn,
              _stream())
    return U_pk, G_pk, S_pk, status


def tsvdm_reconstruct(U_pk, G_pk, rho, offsets, capacity, Mdev, shape, scale=1.0,
                      out_dtype=None, compute=None, out=None, ws=None, tile=0):
    m, p, n = shape
    dt = U_pk.dtype
    odt = out_dtype or dt
    comp = compute or ("f64" if dt == torch.float64 else "f32")
    A_rec = out if out is not None else colmajor_empty(m, p, n, odt, U_pk.device)
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_reconstruct_workspace_size", m, p, n, _DT[dt]))
    _lib.call("tsvdm_reconstruct", _ptr(U_pk), _ptr(G_pk), _DT[dt], m, p, n, _ptr(rho),
              _ptr(offsets), int(capacity), _ptr(Mdev), float(scale), _ptr(A_rec), _dt(A_rec),
              _COMPUTE[comp], int(tile), wp, wn, _stream())
    return A_rec


def tsvdm_error(A, B, ws=None):
    """Device FP64 [sum (A-B)^2, sum A^2]."""
    out = torch.empty(2, dtype=torch.float64, device=A.device)
    cnt = A.numel()
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_error_workspace_size", cnt))
    _lib.call("tsvdm_error", _ptr(A), _dt(A), _ptr(B), _dt(B), cnt, _ptr(out), wp, wn, _stream())
    return out


def tsvdm_backward(A, Mdev, k, g=1.0, want_dA=True, want_dM=True, ws=None):
    A = as_colmajor(A)
    m, p, n = A.shape
    dA = colmajor_empty(m, p, n, A.dtype, A.device) if want_dA else None
    dM = torch.empty((n, n), dtype=torch.float64, device=A.device) if want_dM else None
    loss = torch.empty(1, dtype=torch.float64, device=A.device)
    status = torch.zeros(1, dtype=torch.int32, device=A.device)
    w = _ws(ws)
    wp, wn = w.args(_lib.workspace_size("tsvdm_backward_workspace_size", m, p, n, _dt(A)))
    _lib.call("tsvdm_backward", _ptr(A), _dt(A), m, p, n, _ptr(Mdev), int(k), float(g), _ptr(dA),
              _ptr(dM), _ptr(loss), _ptr(status), wp, wn, _stream())
    # dM is column-major n x n: the torch (n, n) buffer holds its transpose
    return loss, dA, (dM.t() if dM is not None else None), status
