"""FP64 oracle: star-M t-SVD, t-SVDM-I, t-SVDM-II, reconstruction, adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

Conventions
-----------
Tensors are NumPy arrays of shape (m, p, n); frontal slice i is A[:, :, i]
(Section 2.1).  All arithmetic is FP64: inputs of any float type are
converted with ``np.asarray(A, dtype=np.float64)`` first.  M is an n x n
matrix that is a nonzero multiple of an orthogonal matrix (Algorithm 2's
requirement; Section 3 restricts the implementation to orthonormal M).

Parity status
-------------
pinned   : mode3, mode_product, to_transform_domain, from_transform_domain,
           to_transform_domain_d, from_transform_domain_d, tsvdm_d, slice_svd,
           full_tsvdm, mproduct, ranks_fixed, ranks_tolerance,
           truncated_factors, reconstruct, tsvdm_i, tsvdm_ii,
           compression_ratio, rel_error, trunc_loss, trunc_loss_grad,
           cayley, cayley_grad
           (each is checked by the CPU tests against closed forms,
           invariants, brute force or values printed in the paper).
parity unpinned : none.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "check_transform",
    "mode3",
    "to_transform_domain",
    "from_transform_domain",
    "slice_svd",
    "full_tsvdm",
    "mproduct",
    "ranks_fixed",
    "ranks_tolerance",
    "truncated_factors",
    "reconstruct",
    "tsvdm_i",
    "tsvdm_ii",
    "compression_ratio",
    "rel_error",
    "trunc_loss",
    "trunc_loss_grad",
    "cayley",
    "cayley_grad",
    "mode_product",
    "to_transform_domain_d",
    "from_transform_domain_d",
    "tsvdm_d",
]


def _f64(A):
    return np.asarray(A, dtype=np.float64)


# ---------------------------------------------------------------------------
# transform
# ---------------------------------------------------------------------------

def check_transform(M, tol: float = 1e-10) -> float:
    """Return c^2 if M = c * Q with Q orthogonal, else raise ValueError.

    Algorithm 2 requires M to be a nonzero multiple of an orthogonal matrix;
    then M^T M = c^2 I and M^{-1} = M^T / c^2 (Section 2.1).
    """
    M = _f64(M)
    if M.ndim != 2 or M.shape[0] != M.shape[1]:
        raise ValueError("M must be square")
    G = M.T @ M
    c2 = float(np.mean(np.diag(G)))
    if not np.isfinite(c2) or c2 <= 0.0:
        raise ValueError("M must be a nonzero multiple of an orthogonal matrix")
    if np.max(np.abs(G / c2 - np.eye(M.shape[0]))) > tol:
        raise ValueError("M is not a multiple of an orthogonal matrix")
    return c2


def mode3(A, M):
    """Mode-3 product A x_3 M (Section 2.1: (A x_k M)_(k) = M A_(k)).

    Slice i of the result is sum_l M[i, l] * A[:, :, l]; M may be J x n, the
    result then has J frontal slices.
    """
    A = _f64(A)
    M = _f64(M)
    if A.shape[2] != M.shape[1]:
        raise ValueError("mode-3 size mismatch")
    # column-major like the tensors (slice i contiguous); the layout does
    # not change any operation or its order
    out = np.zeros(A.shape[:2] + (M.shape[0],), order="F")
    for i in range(M.shape[0]):
        for l in range(M.shape[1]):
            if M[i, l] != 0.0:
                out[:, :, i] += M[i, l] * A[:, :, l]
    return out


def to_transform_domain(A, M):
    """A-hat = A x_3 M (first step of Algorithm 1)."""
    return mode3(A, M)


def from_transform_domain(C_hat, M):
    """C = C-hat x_3 M^{-1}, with M^{-1} = M^T / c^2 for M = c * Q
    (third step of the star-M product, Section 2.1)."""
    c2 = check_transform(M)
    return mode3(C_hat, _f64(M).T / c2)


def mproduct(A, B, M):
    """star-M product C = A *_M B (Section 2.1): transform both, multiply
    matching frontal slices, transform back."""
    Ah = to_transform_domain(A, M)
    Bh = to_transform_domain(B, M)
    if Ah.shape[1] != Bh.shape[0]:
        raise ValueError("inner slice sizes differ")
    Ch = np.empty((Ah.shape[0], Bh.shape[1], Ah.shape[2]))
    for i in range(Ah.shape[2]):
        Ch[:, :, i] = Ah[:, :, i] @ Bh[:, :, i]
    return from_transform_domain(Ch, M)


# ---------------------------------------------------------------------------
# slice-wise SVD (Algorithm 1)
# ---------------------------------------------------------------------------

def slice_svd(A_hat):
    """Thin SVD of every frontal slice (the loop of Algorithm 1).

    Returns U (m x r x n), S (r x n) descending per slice, V (p x r x n) with
    r = min(m, p) (Section 3.2).  LAPACK through numpy is the library step.
    """
    A_hat = _f64(A_hat)
    m, p, n = A_hat.shape
    r = min(m, p)
    U = np.empty((m, r, n))
    S = np.empty((r, n))
    V = np.empty((p, r, n))
    for i in range(n):
        u, s, vt = np.linalg.svd(A_hat[:, :, i], full_matrices=False)
        U[:, :, i] = u
        S[:, i] = s
        V[:, :, i] = vt.T
    return U, S, V


def full_tsvdm(A, M):
    """Algorithm 1: full t-SVDM.  Returns the transform-domain factors
    (U_hat, S_hat as r x n, V_hat) and the spatial-domain tensors U, S, V with
    A = U *_M S *_M V^T, where S is the f-diagonal r x r x n tensor."""
    A_hat = to_transform_domain(A, M)
    U_hat, S_hat, V_hat = slice_svd(A_hat)
    r, n = S_hat.shape
    S_diag_hat = np.zeros((r, r, n))
    for i in range(n):
        S_diag_hat[:, :, i] = np.diag(S_hat[:, i])
    return {
        "U_hat": U_hat, "S_hat": S_hat, "V_hat": V_hat,
        "U": from_transform_domain(U_hat, M),
        "S": from_transform_domain(S_diag_hat, M),
        "V": from_transform_domain(V_hat, M),
    }


# ---------------------------------------------------------------------------
# rank selection
# ---------------------------------------------------------------------------

def ranks_fixed(k: int, r: int, n: int):
    """t-SVDM-I: the same rank k on every slice (Section 3.3), clamped to
    r = min(m, p) because a slice has only r singular values."""
    if k < 1:
        raise ValueError("k must be >= 1")
    return np.full(n, min(int(k), int(r)), dtype=np.int64)


_SCALE_BITS = 1074  # every finite non-negative double is a multiple of 2^-1074


def _exact_int(x: float) -> int:
    num, den = float(x).as_integer_ratio()
    return num * ((1 << _SCALE_BITS) // den)


def _rounded(acc: int) -> float:
    # Python int / int is correctly rounded to the nearest double
    return acc / (1 << _SCALE_BITS)


def ranks_tolerance(S, eps: float, squared: bool = False):
    """t-SVDM-II rank selection (Algorithm 2).

    v = every squared singular value of every slice, sorted ascending;
    w = its cumulative sum; J = the largest index with w_J / ||S||_F^2 < eps^2;
    tau = v_J; rho_i = number of squared singular values of slice i that are
    greater than tau.

    Readings where the paper is silent:
      * tau is compared with squared values (v holds squares);
      * every value equal to tau is discarded (the literal rule);
      * ||S||_F^2 is the total of the same array v;
      * sums are exact: each w_J and the total are the correctly rounded
        exact sums, then the test is the double division w_J / W < eps*eps;
      * no such J: nothing is discarded (tau = -inf);
      * W = 0 (zero tensor): every rank is 0.
    `squared=True` means S already holds the squared values (r x n).
    Returns (rho, info) with info = {"tau", "J", "discarded", "total"}.
    """
    S = _f64(S)
    if not (0.0 < eps < 1.0):
        raise ValueError("eps must lie in (0, 1)")
    r, n = S.shape
    sq = S if squared else S * S
    v = np.sort(sq.reshape(-1), kind="stable")
    ints = [_exact_int(x) for x in v]
    total_int = sum(ints)
    W = _rounded(total_int)
    if W == 0.0:
        return np.zeros(n, dtype=np.int64), {
            "tau": 0.0, "J": 0, "discarded": 0.0, "total": 0.0}
    eps2 = eps * eps
    J = 0
    acc = 0
    for j, x in enumerate(ints):
        acc += x
        if _rounded(acc) / W < eps2:
            J = j + 1
        else:
            break  # w is non-decreasing, so no later index can qualify
    if J == 0:
        tau = -np.inf
    else:
        tau = float(v[J - 1])
    rho = np.array([int(np.count_nonzero(sq[:, i] > tau)) for i in range(n)],
                   dtype=np.int64)
    discarded = _rounded(sum(x for x, val in zip(ints, v) if val <= tau))
    return rho, {"tau": tau, "J": J, "discarded": discarded, "total": W}


# ---------------------------------------------------------------------------
# factors, reconstruction, reporting
# ---------------------------------------------------------------------------

def truncated_factors(U, S, V, rho):
    """Keep the leading rho_i triplets of slice i (Algorithm 2, final loop):
    U_i = U[:, :rho_i, i], s_i = S[:rho_i, i], G_i = diag(s_i) V[:, :rho_i, i]^T.
    Returned as a list of (U_i, s_i, G_i)."""
    out = []
    for i, k in enumerate(np.asarray(rho, dtype=np.int64)):
        k = int(k)
        Ui = U[:, :k, i].copy()
        si = S[:k, i].copy()
        Gi = si[:, None] * V[:, :k, i].T
        out.append((Ui, si, Gi))
    return out


def reconstruct(factors, M, shape):
    """C-hat_i = U_i G_i in the transform domain, then C = C-hat x_3 M^{-1}."""
    m, p, n = shape
    C_hat = np.zeros((m, p, n), order="F")   # slice i contiguous; layout only
    for i, (Ui, _si, Gi) in enumerate(factors):
        if Ui.shape[1] > 0:
            C_hat[:, :, i] = Ui @ Gi
    return from_transform_domain(C_hat, M)


def compression_ratio(m: int, p: int, n: int, rho) -> float:
    """Stored values of the input over stored values of the factors.

    The paper prints ratios but not the formula.  Reading: slice i keeps an
    m x rho_i left factor, rho_i singular values and a rho_i x p right factor,
    i.e. rho_i * (m + p + 1) values, and M is not counted; this reproduces
    the three t-SVDM-I ratios printed in Section 4."""
    kept = int(np.sum(np.asarray(rho, dtype=np.int64))) * (m + p + 1)
    return float("inf") if kept == 0 else (m * p * n) / kept


def rel_error(A, B) -> float:
    """||A - B||_F / ||A||_F in FP64 (0 when both are zero)."""
    A = _f64(A)
    B = _f64(B)
    den = np.linalg.norm(A.ravel())
    num = np.linalg.norm((A - B).ravel())
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return float(num / den)


def _pipeline(A, M, rho_fn):
    A = _f64(A)
    m, p, n = A.shape
    A_hat = to_transform_domain(A, M)
    U, S, V = slice_svd(A_hat)
    rho, info = rho_fn(S)
    fac = truncated_factors(U, S, V, rho)
    A_rec = reconstruct(fac, M, (m, p, n))
    return {
        "A_hat": A_hat, "U": U, "S": S, "V": V, "rho": rho,
        "factors": fac, "A_rec": A_rec, "info": info,
        "rel_error": rel_error(A, A_rec),
        "compression": compression_ratio(m, p, n, rho),
    }


def tsvdm_i(A, M, k: int):
    """t-SVDM-I: transform, slice SVDs, uniform rank k, reconstruct."""
    A = _f64(A)
    r = min(A.shape[0], A.shape[1])

    def rf(S):
        rho = ranks_fixed(k, r, A.shape[2])
        sq = S * S
        tail = sum(float(np.sum(sq[rho[i]:, i])) for i in range(sq.shape[1]))
        return rho, {"discarded": tail, "total": float(np.sum(sq))}

    return _pipeline(A, M, rf)


def tsvdm_ii(A, M, eps: float):
    """t-SVDM-II (Algorithm 2): transform, slice SVDs, global tolerance."""
    return _pipeline(A, M, lambda S: ranks_tolerance(S, eps))


# ---------------------------------------------------------------------------
# adjoint of the truncation loss (not in the paper; derived here)
# ---------------------------------------------------------------------------

def trunc_loss(A, M, k: int) -> float:
    """L(A, M) = sum_i sum_{j > k} sigma_ij^2, the squared singular values
    dropped by a rank-k truncation of every slice of A x_3 M.  For
    orthogonal M this equals ||A - A_k||_F^2 (Section 2.3).  Computed as the
    tail sum, never as a difference of totals."""
    A_hat = to_transform_domain(A, M)
    _U, S, _V = slice_svd(A_hat)
    return float(np.sum(S[k:, :] ** 2))


def trunc_loss_grad(A, M, k: int):
    """Gradient of trunc_loss with respect to A and M.

    With R-hat_i the rank-k tail of slice i of A-hat (A-hat_i minus its best
    rank-k approximation; differentiable when sigma_k > sigma_{k+1}):
      dL/dA-hat = 2 R-hat,   dL/dA = 2 R-hat x_3 M^T,
      dL/dM[i, l] = 2 <R-hat_i, A_l>   (G_M = 2 R-hat_(3) A_(3)^T).
    """
    A = _f64(A)
    M = _f64(M)
    A_hat = to_transform_domain(A, M)
    U, S, V = slice_svd(A_hat)
    m, p, n = A.shape
    R_hat = np.zeros((m, p, n))
    for i in range(n):
        R_hat[:, :, i] = (U[:, k:, i] * S[k:, i][None, :]) @ V[:, k:, i].T
    dA = 2.0 * mode3(R_hat, M.T)
    GM = np.empty((n, n))
    for i in range(n):
        for l in range(n):
            GM[i, l] = 2.0 * float(np.sum(R_hat[:, :, i] * A[:, :, l]))
    loss = float(np.sum(S[k:, :] ** 2))
    return loss, dA, GM


def cayley(K):
    """Cayley map M = (I - K)^{-1} (I + K); orthogonal for skew K."""
    K = _f64(K)
    I = np.eye(K.shape[0])
    return np.linalg.solve(I - K, I + K)


def cayley_grad(K, GM):
    """Chain rule through the Cayley map for a skew parameter.

    dM = (I - K)^{-1} dK (I + M), so with G_M = dL/dM,
    Y = (I + K)^{-1} G_M (I + M)^T and, for the free entries K_ab (a < b,
    K_ba = -K_ab), dL/dK_ab = Y_ab - Y_ba.  Returned as the skew matrix D
    with D[a, b] = Y_ab - Y_ba, so dL = sum_{a<b} D[a, b] dK[a, b]."""
    K = _f64(K)
    GM = _f64(GM)
    I = np.eye(K.shape[0])
    M = cayley(K)
    Y = np.linalg.solve(I + K, GM @ (I + M).T)
    return Y - Y.T


# ---------------------------------------------------------------------------
# tensors of order d > 3 (Section 2.1, footnote; Section 3.1)
# ---------------------------------------------------------------------------

def mode_product(A, M, k: int):
    """Mode-k product A x_k M of a tensor of any order (Section 2.1:
    (A x_k M)_(k) = M A_(k)); k is 1-based and M is J x n_k.  Written as the
    definition: the k-th index i of the result gathers sum_l M[i, l] times
    the sub-tensor of A whose k-th index is l."""
    A = _f64(A)
    M = _f64(M)
    ax = k - 1
    if not (0 <= ax < A.ndim) or A.shape[ax] != M.shape[1]:
        raise ValueError("mode-k size mismatch")
    shape = list(A.shape)
    shape[ax] = M.shape[0]
    out = np.zeros(shape)
    for i in range(M.shape[0]):
        oi = [slice(None)] * A.ndim
        oi[ax] = i
        for l in range(M.shape[1]):
            if M[i, l] != 0.0:
                ai = [slice(None)] * A.ndim
                ai[ax] = l
                out[tuple(oi)] += M[i, l] * A[tuple(ai)]
    return out


def to_transform_domain_d(A, Ms):
    """A-hat = A x_3 M_3 x_4 M_4 ... x_d M_d: each mode k >= 3 gets its own
    transform (Section 2.1, footnote on order-d tensors; Section 3.1)."""
    A = _f64(A)
    if len(Ms) != A.ndim - 2:
        raise ValueError("one transform per mode k >= 3")
    for k, M in enumerate(Ms, start=3):
        A = mode_product(A, M, k)
    return A


def from_transform_domain_d(C_hat, Ms):
    """C = C-hat x_3 M_3^{-1} ... x_d M_d^{-1}, M_k^{-1} = M_k^T / c_k^2."""
    C = _f64(C_hat)
    for k, M in enumerate(Ms, start=3):
        c2 = check_transform(M)
        C = mode_product(C, _f64(M).T / c2, k)
    return C


def tsvdm_d(A, Ms, mode: str = "II", k: int | None = None, eps: float | None = None):
    """t-SVDM-I (mode "I", rank k) or t-SVDM-II (mode "II", tolerance eps) of
    an order-d tensor n_1 x n_2 x n_3 x ... x n_d.  A frontal slice fixes every
    index but the first two (Section 2.1, footnote), so after the transforms
    the N = n_3 ... n_d slices (column-major order: mode 3 varies fastest) go
    through the slice SVDs, the rank selection and the back-transforms
    exactly as for three modes."""
    A = _f64(A)
    dims = A.shape
    if len(dims) < 3:
        raise ValueError("order >= 3")
    n1, n2 = dims[0], dims[1]
    A_hat = to_transform_domain_d(A, Ms)
    A3 = A_hat.reshape(n1, n2, -1, order="F")
    U, S, V = slice_svd(A3)
    r, N = S.shape
    if mode == "I":
        rho = ranks_fixed(k, r, N)
        sq = S * S
        info = {"discarded": sum(float(np.sum(sq[rho[i]:, i])) for i in range(N)),
                "total": float(np.sum(sq))}
    elif mode == "II":
        rho, info = ranks_tolerance(S, eps)
    else:
        raise ValueError("mode must be 'I' or 'II'")
    fac = truncated_factors(U, S, V, rho)
    C_hat = np.zeros((n1, n2, N))
    for i, (Ui, _si, Gi) in enumerate(fac):
        if Ui.shape[1] > 0:
            C_hat[:, :, i] = Ui @ Gi
    A_rec = from_transform_domain_d(C_hat.reshape(dims, order="F"), Ms)
    return {"A_hat": A_hat, "S": S, "rho": rho, "factors": fac, "info": info,
            "A_rec": A_rec, "rel_error": rel_error(A, A_rec)}
