"""Pins of the order-d oracle (Section 2.1 footnote; Section 3.1): the mode-k
product against numpy's tensordot, the Kronecker identity that turns two
transformed modes into one 3-way transform (so the order-d method equals the
pinned 3-way method on the reshaped tensor), the Eckart-Young energy
identity, full rank, identity transforms (per-slice matrix SVDs) and
scaled-orthogonal transforms."""
import numpy as np
import pytest

import oracle as O
import synth


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_mode_product_matches_tensordot(k):
    A = _rand((4, 3, 5, 2, 3), 1)
    M = _rand((6, A.shape[k - 1]), 2)   # J != n_k on purpose
    ref = np.moveaxis(np.tensordot(M, A, axes=(1, k - 1)), 0, k - 1)
    got = O.mode_product(A, M, k)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_mode_product_rejects_mismatch():
    with pytest.raises(ValueError):
        O.mode_product(np.zeros((2, 3, 4)), np.zeros((4, 5)), 3)


def _kron_case(seed):
    g = np.random.default_rng(seed)
    A = g.standard_normal((9, 7, 4, 3)) + 5.0 * np.einsum(
        "a,b,c,d->abcd", g.standard_normal(9), g.standard_normal(7), g.standard_normal(4),
        g.standard_normal(3))
    M3 = synth.haar_orthogonal(4, g)
    M4 = synth.dct2_matrix(3)
    return A, M3, M4


def test_two_transformed_modes_equal_one_kronecker_transform():
    """Column-major order makes mode 3 the fast index of the merged mode, so
    A x_3 M3 x_4 M4 reshaped to 3 modes is A_3 x_3 (M4 kron M3)."""
    A, M3, M4 = _kron_case(3)
    n1, n2 = A.shape[:2]
    lhs = O.to_transform_domain_d(A, [M3, M4]).reshape(n1, n2, -1, order="F")
    rhs = O.mode3(A.reshape(n1, n2, -1, order="F"), np.kron(M4, M3))
    assert np.max(np.abs(lhs - rhs)) <= 1e-13 * np.max(np.abs(rhs))


@pytest.mark.parametrize("mode,arg", [("II", 0.05), ("II", 0.3), ("I", 2)])
def test_order4_method_equals_3way_method_on_reshaped_tensor(mode, arg):
    A, M3, M4 = _kron_case(4)
    n1, n2 = A.shape[:2]
    A3 = A.reshape(n1, n2, -1, order="F")
    Mk = np.kron(M4, M3)
    if mode == "II":
        d = O.tsvdm_d(A, [M3, M4], mode="II", eps=arg)
        t = O.tsvdm_ii(A3, Mk, arg)
    else:
        d = O.tsvdm_d(A, [M3, M4], mode="I", k=arg)
        t = O.tsvdm_i(A3, Mk, arg)
    assert np.array_equal(d["rho"], t["rho"])
    rec = d["A_rec"].reshape(n1, n2, -1, order="F")
    assert np.max(np.abs(rec - t["A_rec"])) <= 1e-12 * np.max(np.abs(A))
    assert abs(d["rel_error"] - t["rel_error"]) <= 1e-12


def test_order5_energy_identity_and_tolerance():
    g = np.random.default_rng(5)
    A = g.standard_normal((6, 8, 3, 2, 4))
    Ms = [synth.haar_orthogonal(n, g) for n in (3, 2, 4)]
    eps = 0.4
    res = O.tsvdm_d(A, Ms, mode="II", eps=eps)
    err2 = np.sum((A - res["A_rec"]) ** 2)
    assert abs(err2 - res["info"]["discarded"]) <= 1e-12 * np.sum(A * A)
    assert res["rel_error"] < eps
    # nothing dropped at a tiny tolerance: A comes back
    full = O.tsvdm_d(A, Ms, mode="I", k=6)
    assert O.rel_error(A, full["A_rec"]) <= 1e-13


def test_identity_transforms_are_per_slice_matrix_truncations():
    A = _rand((7, 5, 2, 3), 6)
    Ms = [np.eye(2), np.eye(3)]
    k = 2
    res = O.tsvdm_d(A, Ms, mode="I", k=k)
    for i3 in range(2):
        for i4 in range(3):
            X = A[:, :, i3, i4]
            u, s, vt = np.linalg.svd(X, full_matrices=False)
            Xk = (u[:, :k] * s[:k]) @ vt[:k]
            assert np.max(np.abs(res["A_rec"][:, :, i3, i4] - Xk)) <= 1e-13 * np.max(np.abs(X))


def test_scaled_transforms_give_the_same_result():
    A, M3, M4 = _kron_case(7)
    a = O.tsvdm_d(A, [M3, M4], mode="II", eps=0.1)
    b = O.tsvdm_d(A, [2.0 * M3, 0.5 * M4], mode="II", eps=0.1)
    assert np.array_equal(a["rho"], b["rho"])
    assert np.max(np.abs(a["A_rec"] - b["A_rec"])) <= 1e-12 * np.max(np.abs(A))


def test_unit_modes_reduce_to_lower_order():
    A = _rand((6, 5, 4), 8)
    M = synth.haar_orthogonal(4, np.random.default_rng(9))
    a = O.tsvdm_d(A[:, :, :, None], [M, np.eye(1)], mode="II", eps=0.2)
    b = O.tsvdm_ii(A, M, 0.2)
    assert np.array_equal(a["rho"], b["rho"])
    assert np.max(np.abs(a["A_rec"][:, :, :, 0] - b["A_rec"])) <= 1e-13 * np.max(np.abs(A))
