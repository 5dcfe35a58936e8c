"""Pins for the FP64 oracle: closed forms, invariants, brute force and the
values the paper prints.  CPU only.

Each test is chosen so that a plausible slip in the oracle (a transposed M,
a wrong sign, a dropped singular value, '<=' for '<', an off-by-one in the
threshold index, a wrong storage count) makes it fail.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# transform (Section 2.1)
# ---------------------------------------------------------------------------

def test_mode3_identity_is_exact():
    A = rng(1).standard_normal((5, 4, 6))
    assert np.array_equal(O.mode3(A, np.eye(6)), A)


def test_mode3_orientation_with_cyclic_permutation():
    # P[i, (i+1) % n] = 1  =>  slice i of A x_3 P is slice i+1 of A.
    # The transpose of P would give slice i-1 instead, so this pins which
    # index of M runs over output slices.
    n = 5
    P = np.zeros((n, n))
    for i in range(n):
        P[i, (i + 1) % n] = 1.0
    A = rng(2).standard_normal((3, 4, n))
    Ah = O.mode3(A, P)
    for i in range(n):
        assert np.array_equal(Ah[:, :, i], A[:, :, (i + 1) % n])


def test_mode3_constant_tubes_under_dct():
    # every tube constant => all energy in frequency 0, with value sqrt(n) B
    n = 12
    B = rng(3).standard_normal((4, 7))
    A = np.repeat(B[:, :, None], n, axis=2)
    Ah = O.mode3(A, synth.dct2_matrix(n))
    assert np.allclose(Ah[:, :, 0], np.sqrt(n) * B, rtol=0, atol=1e-13)
    assert np.max(np.abs(Ah[:, :, 1:])) < 1e-13


def test_mode3_single_cosine_tube_under_dct():
    # tube j -> cos(pi k (2j+1) / (2n)) is DCT basis row k (scaled), so only
    # frequency k survives, with value sqrt(n/2) B for k >= 1
    n, k = 16, 5
    B = rng(4).standard_normal((3, 2))
    tube = np.cos(np.pi * k * (2 * np.arange(n) + 1) / (2 * n))
    A = B[:, :, None] * tube[None, None, :]
    Ah = O.mode3(A, synth.dct2_matrix(n))
    assert np.allclose(Ah[:, :, k], math.sqrt(n / 2) * B, rtol=0, atol=1e-13)
    others = [i for i in range(n) if i != k]
    assert np.max(np.abs(Ah[:, :, others])) < 1e-13


def test_dct_generator_matches_scipy_and_is_orthonormal():
    for n in (1, 2, 7, 16, 33):
        M = synth.dct2_matrix(n)
        ref = scipy.fft.dct(np.eye(n), type=2, norm="ortho", axis=0)
        assert np.allclose(M, ref, rtol=0, atol=1e-14)
        assert np.allclose(M.T @ M, np.eye(n), atol=1e-13)


def test_transform_round_trip_and_norm():
    A = rng(5).standard_normal((6, 5, 7))
    Q = synth.haar_orthogonal(7, rng(6))
    for c in (1.0, 3.0, 0.25):
        M = c * Q
        Ah = O.to_transform_domain(A, M)
        assert math.isclose(np.linalg.norm(Ah), c * np.linalg.norm(A), rel_tol=1e-13)
        back = O.from_transform_domain(Ah, M)
        assert np.allclose(back, A, rtol=0, atol=1e-13)


def test_check_transform_rejects_non_orthogonal():
    with pytest.raises(ValueError):
        O.check_transform(np.array([[1.0, 0.5], [0.0, 1.0]]))
    with pytest.raises(ValueError):
        O.check_transform(np.zeros((3, 3)))
    assert math.isclose(O.check_transform(2.0 * np.eye(4)), 4.0)


# ---------------------------------------------------------------------------
# slice SVD (Algorithm 1)
# ---------------------------------------------------------------------------

def _pure_python_jacobi_sigma(Mat):
    """Singular values by one-sided Jacobi, pure Python floats, written
    independently of numpy's LAPACK path."""
    rows = len(Mat)
    cols = len(Mat[0])
    if rows < cols:  # work on the transpose so there are min(rows, cols) vectors
        Mat = [[Mat[i][j] for i in range(rows)] for j in range(cols)]
        rows, cols = cols, rows
    X = [[Mat[i][j] for i in range(rows)] for j in range(cols)]  # column vectors
    for _sweep in range(60):
        off = 0.0
        for a in range(cols):
            for b in range(a + 1, cols):
                alpha = sum(x * x for x in X[a])
                beta = sum(x * x for x in X[b])
                gamma = sum(x * y for x, y in zip(X[a], X[b]))
                if alpha == 0.0 or beta == 0.0:
                    continue
                off = max(off, abs(gamma) / math.sqrt(alpha * beta))
                if gamma == 0.0:
                    continue
                zeta = (beta - alpha) / (2.0 * gamma)
                t = math.copysign(1.0, zeta) / (abs(zeta) + math.sqrt(1.0 + zeta * zeta))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = c * t
                xa, xb = X[a], X[b]
                X[a] = [c * u - s * v for u, v in zip(xa, xb)]
                X[b] = [s * u + c * v for u, v in zip(xa, xb)]
        if off < 1e-15:
            break
    return sorted((math.sqrt(sum(x * x for x in col)) for col in X), reverse=True)


@pytest.mark.parametrize("shape", [(5, 3, 2), (3, 5, 2), (4, 4, 3)])
def test_slice_svd_matches_pure_python_jacobi(shape):
    A = rng(7).standard_normal(shape)
    _U, S, _V = O.slice_svd(A)
    for i in range(shape[2]):
        ref = _pure_python_jacobi_sigma(A[:, :, i].tolist())
        assert np.allclose(S[:, i], ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("shape", [(9, 5, 3), (5, 9, 3)])
def test_slice_svd_invariants(shape):
    A = rng(8).standard_normal(shape)
    U, S, V = O.slice_svd(A)
    r = min(shape[:2])
    for i in range(shape[2]):
        assert np.allclose(U[:, :, i].T @ U[:, :, i], np.eye(r), atol=1e-13)
        assert np.allclose(V[:, :, i].T @ V[:, :, i], np.eye(r), atol=1e-13)
        rec = (U[:, :, i] * S[:, i][None, :]) @ V[:, :, i].T
        assert np.allclose(rec, A[:, :, i], atol=1e-13)
        assert np.all(np.diff(S[:, i]) <= 0) and np.all(S[:, i] >= 0)


def test_identity_transform_is_per_slice_matrix_truncation():
    # M = I: t-SVDM-I error^2 equals the sum of the dropped eigenvalues of
    # each slice's Gram matrix (matrix Eckart-Young via a different routine)
    A = rng(9).standard_normal((8, 6, 4))
    k = 2
    res = O.tsvdm_i(A, np.eye(4), k)
    expect = 0.0
    for i in range(4):
        ev = np.sort(np.linalg.eigvalsh(A[:, :, i].T @ A[:, :, i]))[::-1]
        expect += float(np.sum(ev[k:]))
    err2 = float(np.sum((A - res["A_rec"]) ** 2))
    assert math.isclose(err2, expect, rel_tol=1e-11)


# ---------------------------------------------------------------------------
# star-M algebra and optimality (Sections 2.1 and 2.3)
# ---------------------------------------------------------------------------

def _slice_transpose(T):
    return np.transpose(T, (1, 0, 2)).copy()


def test_full_tsvdm_factorisation_and_orthogonality():
    A = rng(10).standard_normal((6, 4, 5))
    M = synth.haar_orthogonal(5, rng(11))
    F = O.full_tsvdm(A, M)
    U, S, V = F["U"], F["S"], F["V"]
    # A = U *M S *M V^T  (Algorithm 1's guarantee)
    rec = O.mproduct(O.mproduct(U, S, M), _slice_transpose(V), M)
    assert np.allclose(rec, A, atol=1e-12)
    # U^T *M U = I: the identity tensor has identity slices in the M domain
    r = 4
    I_hat = np.repeat(np.eye(r)[:, :, None], 5, axis=2)
    I_t = O.from_transform_domain(I_hat, M)
    assert np.allclose(O.mproduct(_slice_transpose(U), U, M), I_t, atol=1e-12)
    assert np.allclose(O.mproduct(_slice_transpose(V), V, M), I_t, atol=1e-12)


@pytest.mark.parametrize("mode", ["I", "II"])
def test_eckart_young_energy_identity(mode):
    A = synth.planted_lowrank(12, 9, 8, 3, 5.0, rng(12))
    M = synth.haar_orthogonal(8, rng(13))
    res = O.tsvdm_i(A, M, 3) if mode == "I" else O.tsvdm_ii(A, M, 0.3)
    err2 = float(np.sum((np.asarray(A) - res["A_rec"]) ** 2))
    tail = sum(float(np.sum(res["S"][res["rho"][i]:, i] ** 2)) for i in range(8))
    assert math.isclose(err2, tail, rel_tol=1e-11)
    assert math.isclose(res["info"]["discarded"], tail, rel_tol=1e-12)


def test_truncation_is_optimal_against_perturbed_factors():
    A = synth.planted_lowrank(10, 8, 6, 2, 4.0, rng(14))
    M = synth.dct2_matrix(6)
    res = O.tsvdm_i(A, M, 2)
    best = float(np.sum((np.asarray(A) - res["A_rec"]) ** 2))
    Ah = O.to_transform_domain(A, M)
    g = rng(15)
    for _ in range(25):
        Ch = np.empty_like(Ah)
        for i in range(6):
            Ui = res["factors"][i][0] + 0.05 * g.standard_normal((10, 2))
            Qi, _ = np.linalg.qr(Ui)
            Ch[:, :, i] = Qi @ (Qi.T @ Ah[:, :, i])  # best G for this U
        alt = O.from_transform_domain(Ch, M)
        assert float(np.sum((np.asarray(A) - alt) ** 2)) >= best * (1 - 1e-12)


def test_full_rank_reconstructs_input():
    A = rng(16).standard_normal((7, 5, 6))
    M = synth.haar_orthogonal(6, rng(17))
    res = O.tsvdm_i(A, M, 99)  # k > r clamps to r
    assert np.all(res["rho"] == 5)
    assert O.rel_error(A, res["A_rec"]) < 1e-13


def test_scaled_transform_gives_same_result():
    A = synth.planted_lowrank(9, 7, 5, 2, 3.0, rng(18))
    Q = synth.haar_orthogonal(5, rng(19))
    r1 = O.tsvdm_ii(A, Q, 0.2)
    r2 = O.tsvdm_ii(A, 2.5 * Q, 0.2)
    assert np.array_equal(r1["rho"], r2["rho"])
    assert np.allclose(r1["A_rec"], r2["A_rec"], atol=1e-12)


# ---------------------------------------------------------------------------
# t-SVDM-II rank selection (Algorithm 2)
# ---------------------------------------------------------------------------

def _brute_force_ranks(S, eps):
    """Among all rank vectors (slice i keeps its rho_i largest values) whose
    dropped energy is < eps^2 * total, pick the one that drops the most
    values, then the least energy.  Exact rational arithmetic."""
    r, n = S.shape
    sq = [[Fraction(float(S[j, i])) ** 2 for j in range(r)] for i in range(n)]
    total = sum(sum(col) for col in sq)
    budget = Fraction(eps) ** 2 * total
    best = None
    for rho in itertools.product(range(r + 1), repeat=n):
        dropped = sum(sum(sq[i][rho[i]:]) for i in range(n))
        if not dropped < budget:
            continue
        key = (sum(rho), dropped)
        if best is None or key < best[0]:
            best = (key, rho)
    return np.array(best[1])


def test_ranks_tolerance_matches_brute_force():
    g = rng(20)
    checked = 0
    for trial in range(40):
        n, r = 3, 3
        # dyadic values so every square and every sum is exact
        vals = g.choice(np.arange(1, 200), size=r * n, replace=False) / 8.0
        S = -np.sort(-vals.reshape(n, r), axis=1).T.copy()
        eps = float(g.uniform(0.05, 0.95))
        rho, info = O.ranks_tolerance(S, eps)
        assert np.array_equal(rho, _brute_force_ranks(S, eps)), (S, eps)
        # the guarantee: relative error < eps (for orthogonal M)
        dropped = sum(float(np.sum(S[rho[i]:, i] ** 2)) for i in range(n))
        assert dropped < eps * eps * float(np.sum(S ** 2))
        checked += 1
    assert checked == 40


def test_ranks_tolerance_ties_are_all_discarded():
    # squares sorted: 0, 1, 1, 1, 1, 100 (W = 104); with eps^2 = 0.025 the
    # prefix sums 0, 1, 2 qualify and 3 does not, so J = 3 and tau = 1; the
    # literal rule then drops every value equal to tau (all four ones).
    S = np.array([[10.0, 1.0], [1.0, 1.0], [0.0, 1.0]])  # r=3, n=2; a zero too
    rho, info = O.ranks_tolerance(S, math.sqrt(0.025))
    assert info["tau"] == 1.0
    assert list(rho) == [1, 0]
    assert info["discarded"] == 4.0


def test_ranks_tolerance_special_cases():
    with pytest.raises(ValueError):
        O.ranks_tolerance(np.ones((2, 2)), 0.0)
    with pytest.raises(ValueError):
        O.ranks_tolerance(np.ones((2, 2)), 1.0)
    rho, info = O.ranks_tolerance(np.zeros((3, 4)), 0.5)
    assert list(rho) == [0, 0, 0, 0] and info["total"] == 0.0
    # equal values and a small tolerance: nothing can be dropped
    rho, info = O.ranks_tolerance(np.ones((3, 2)), 0.1)
    assert list(rho) == [3, 3] and info["J"] == 0
    # exact zeros are always dropped when anything is nonzero
    S = np.array([[5.0, 4.0], [0.0, 0.0]])
    rho, _ = O.ranks_tolerance(S, 0.01)
    assert list(rho) == [1, 1]


def test_ranks_fixed_clamps():
    assert list(O.ranks_fixed(8, 5, 3)) == [5, 5, 5]
    assert list(O.ranks_fixed(2, 5, 2)) == [2, 2]
    with pytest.raises(ValueError):
        O.ranks_fixed(0, 5, 2)


def test_tsvdm_ii_meets_tolerance_on_workload_recipe():
    w = synth.workload("climate", small=True)
    res = O.tsvdm_ii(w.A, w.M, 0.05)
    assert res["rel_error"] < 0.05
    # the error is the predicted one: sqrt(discarded / total)
    pred = math.sqrt(res["info"]["discarded"] / res["info"]["total"])
    assert math.isclose(res["rel_error"], pred, rel_tol=1e-9)


# ---------------------------------------------------------------------------
# compression accounting (Section 4, printed ratios)
# ---------------------------------------------------------------------------

def test_compression_ratio_reproduces_printed_values():
    with open(os.path.join(GOLDEN, "compression_ratios.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        m, p, k = c["slice_rows"], c["slice_cols"], c["k"]
        n = 10  # uniform rank: the ratio does not depend on n
        ratio = O.compression_ratio(m, p, n, [k] * n)
        assert round(ratio, c["digits"]) == c["printed"], (c, ratio)
    # the alternative readings do not reproduce the first printed value
    assert round(73 * 144 / (73 + 144), 1) != 48.2
    assert O.compression_ratio(2, 2, 1, [0]) == float("inf")


# ---------------------------------------------------------------------------
# adjoint of the truncation loss (derived, not in the paper)
# ---------------------------------------------------------------------------

def _skew(n, g):
    W = g.standard_normal((n, n))
    return 0.3 * (W - W.T)


def test_cayley_is_orthogonal():
    K = _skew(6, rng(21))
    M = O.cayley(K)
    assert np.allclose(M.T @ M, np.eye(6), atol=1e-13)
    assert np.allclose(O.cayley(np.zeros((3, 3))), np.eye(3))


def test_trunc_loss_equals_truncation_error_for_orthogonal_M():
    A = rng(22).standard_normal((7, 5, 6))
    M = O.cayley(_skew(6, rng(23)))
    L = O.trunc_loss(A, M, 2)
    err2 = float(np.sum((A - O.tsvdm_i(A, M, 2)["A_rec"]) ** 2))
    assert math.isclose(L, err2, rel_tol=1e-11)


def test_adjoint_matches_central_differences():
    g = rng(24)
    A = g.standard_normal((7, 5, 6))
    K = _skew(6, g)
    k, h = 2, 1e-6
    M = O.cayley(K)
    L, dA, GM = O.trunc_loss_grad(A, M, k)
    dK = O.cayley_grad(K, GM)
    # closed form for orthogonal M: dA = 2 (A - A_k)
    A_k = O.tsvdm_i(A, M, k)["A_rec"]
    assert np.allclose(dA, 2 * (A - A_k), atol=1e-11)
    for _ in range(6):
        E = g.standard_normal(A.shape)
        fd = (O.trunc_loss(A + h * E, M, k) - O.trunc_loss(A - h * E, M, k)) / (2 * h)
        assert math.isclose(fd, float(np.sum(dA * E)), rel_tol=1e-6, abs_tol=1e-7)
        D = _skew(6, g)  # skew direction
        fdk = (O.trunc_loss(A, O.cayley(K + h * D), k)
               - O.trunc_loss(A, O.cayley(K - h * D), k)) / (2 * h)
        iu = np.triu_indices(6, 1)
        an = float(np.sum(dK[iu] * D[iu]))
        assert math.isclose(fdk, an, rel_tol=1e-6, abs_tol=1e-7)
        # gradient wrt M itself (unconstrained direction)
        Em = g.standard_normal((6, 6))
        fdm = (O.trunc_loss(A, M + h * Em, k) - O.trunc_loss(A, M - h * Em, k)) / (2 * h)
        assert math.isclose(fdm, float(np.sum(GM * Em)), rel_tol=1e-6, abs_tol=1e-7)
