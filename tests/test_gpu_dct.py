"""GPU parity of the fast DCT-II transform (tsvdm_transform_dct; Section
2.2, choice of M: the DCT applies in O(n log n); Section 5, operator
transforms for the TTM stage) against the oracle's dense mode product with
the orthonormal DCT-II: every power of two n from 2 to 1024, forward and
inverse, FP64 (<= 1e-13) and FP32 (<= 3e-6) arithmetic, mixed input/output
precisions, middle modes of order-5 tensors, a block count beyond one
launch's grid, ragged row counts, the round trip, agreement with the dense
MFMA transform, sampled tubes of the 512x1024x256 climate tensor, and the
t-SVDM pipeline with transform="dct" against the dense pipeline and the
oracle."""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def to_dev_nd(A, dtype):
    from paper_2605_16058_amd import ops
    out = ops.colmajor_empty_nd(A.shape, dtype, "cuda")
    out.copy_(torch.from_numpy(np.asfortranarray(A)).to(dtype))
    return out


def to_np(T):
    return T.detach().double().cpu().numpy()


def rel(a, b):
    d = np.linalg.norm(np.asarray(b, np.float64).ravel())
    return float(np.linalg.norm((np.asarray(a, np.float64) - b).ravel()) / (d if d > 0 else 1.0))


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("compute,dt,bound", [("f64", torch.float64, 1e-13), ("f32", torch.float32, 3e-6)])
def test_dct_matches_oracle(n, compute, dt, bound):
    from paper_2605_16058_amd import ops
    g = np.random.default_rng(n)
    m, p = (37, 5) if n >= 512 else (37, 29)   # m p not a multiple of the tubes per workgroup
    A = g.standard_normal((m, p, n))
    if dt == torch.float32:
        A = A.astype(np.float32).astype(np.float64)
    C = synth.dct2_matrix(n)
    X = to_dev_nd(A, dt)
    Y = ops.tsvdm_transform_dct(X, 3, inverse=False, compute=compute, out_dtype=dt)
    assert rel(to_np(Y), O.mode_product(A, C, 3)) <= bound
    Z = ops.tsvdm_transform_dct(X, 3, inverse=True, compute=compute, out_dtype=dt)
    assert rel(to_np(Z), O.mode_product(A, C.T, 3)) <= bound


@pytest.mark.parametrize("xdt,ydt,compute,bound", [
    (torch.float32, torch.float64, "f64", 1e-13),
    (torch.float64, torch.float32, "f64", 1e-7),
    (torch.float32, torch.float64, "f32", 3e-6),
    (torch.float64, torch.float64, "f32", 3e-6)])
def test_dct_mixed_precisions(xdt, ydt, compute, bound):
    from paper_2605_16058_amd import ops
    g = np.random.default_rng(11)
    A = g.standard_normal((19, 23, 64))
    if xdt == torch.float32:
        A = A.astype(np.float32).astype(np.float64)
    X = to_dev_nd(A, xdt)
    Y = ops.tsvdm_transform_dct(X, 3, compute=compute, out_dtype=ydt)
    assert Y.dtype == ydt
    assert rel(to_np(Y), O.mode_product(A, synth.dct2_matrix(64), 3)) <= bound


def test_dct_every_mode_of_order5():
    from paper_2605_16058_amd import ops
    g = np.random.default_rng(5)
    dims = (9, 7, 8, 4, 16)
    A = g.standard_normal(dims)
    X = to_dev_nd(A, torch.float64)
    for k in (3, 4, 5):
        C = synth.dct2_matrix(dims[k - 1])
        Y = ops.tsvdm_transform_dct(X, k, compute="f64")
        assert rel(to_np(Y), O.mode_product(A, C, k)) <= 1e-13
        Z = ops.tsvdm_transform_dct(X, k, inverse=True, compute="f64")
        assert rel(to_np(Z), O.mode_product(A, C.T, k)) <= 1e-13


def test_dct_blocks_beyond_one_grid():
    # mode 3 of a 3 x 2 x 4 x 70000 tensor: 70,000 blocks (more than one
    # launch's grid height)
    from paper_2605_16058_amd import ops
    g = np.random.default_rng(6)
    A = g.standard_normal((3, 2, 4, 70000))
    X = to_dev_nd(A, torch.float64)
    Y = ops.tsvdm_transform_dct(X, 3, compute="f64")
    assert rel(to_np(Y), O.mode_product(A, synth.dct2_matrix(4), 3)) <= 1e-13


@pytest.mark.parametrize("compute,dt,bound", [("f64", torch.float64, 1e-14), ("f32", torch.float32, 2e-6)])
def test_dct_round_trip(compute, dt, bound):
    from paper_2605_16058_amd import ops
    g = np.random.default_rng(8)
    A = g.standard_normal((33, 31, 256))
    X = to_dev_nd(A, dt)
    Y = ops.tsvdm_transform_dct(X, 3, compute=compute, out_dtype=dt)
    Z = ops.tsvdm_transform_dct(Y, 3, inverse=True, compute=compute, out_dtype=dt)
    assert rel(to_np(Z), to_np(X)) <= bound


def test_dct_equals_dense_transform():
    from paper_2605_16058_amd import ops
    g = np.random.default_rng(9)
    A = g.standard_normal((64, 48, 128))
    X = to_dev_nd(A, torch.float64)
    Md = ops.device_matrix(synth.dct2_matrix(128))
    dense = ops.tsvdm_transform(X, Md, compute="f64", out_dtype=torch.float64)
    fast = ops.tsvdm_transform_dct(X, 3, compute="f64")
    assert rel(to_np(fast), to_np(dense)) <= 1e-13


@pytest.mark.slow
def test_dct_climate_full_size_sampled_tubes():
    # the 512x1024x256 climate tensor in FP32, FP32 arithmetic, checked on
    # 2,000 sampled tubes against the oracle's dense product
    from paper_2605_16058_amd import ops
    w = synth.workload("climate")
    A = w.A
    X = to_dev_nd(A, torch.float32)
    Y = ops.tsvdm_transform_dct(X, 3, compute="f32", out_dtype=torch.float32)
    g = np.random.default_rng(12)
    ia = g.integers(0, A.shape[0], 2000)
    ib = g.integers(0, A.shape[1], 2000)
    C = synth.dct2_matrix(A.shape[2])
    tubes = A.astype(np.float32).astype(np.float64)[ia, ib, :]       # 2000 x n
    ref = tubes @ C.T
    got = Y[torch.from_numpy(ia).cuda(), torch.from_numpy(ib).cuda(), :].double().cpu().numpy()
    assert rel(got, ref) <= 3e-6
    Z = ops.tsvdm_transform_dct(Y, 3, inverse=True, compute="f32", out_dtype=torch.float32)
    back = Z[torch.from_numpy(ia).cuda(), torch.from_numpy(ib).cuda(), :].double().cpu().numpy()
    assert rel(back, tubes) <= 3e-6


@pytest.mark.parametrize("precision,bound", [("f64", 1e-12), ("f32", 3e-5)])
def test_pipeline_dct_matches_dense_and_oracle(precision, bound):
    from paper_2605_16058_amd.pipeline import TSVDM
    w = synth.workload("planted")
    A, M = w.A, w.M
    n = A.shape[2]
    dt = torch.float64 if precision == "f64" else torch.float32
    X = to_dev_nd(A if dt == torch.float64 else A.astype(np.float32).astype(np.float64), dt)
    for mode, kw in (("I", {"k": 8}), ("II", {"eps": 0.3})):
        fast = TSVDM(A.shape, M, mode=mode, precision=precision, transform="dct", **kw)(X)
        dense = TSVDM(A.shape, M, mode=mode, precision=precision, **kw)(X)
        assert torch.equal(fast.rho.cpu(), dense.rho.cpu())
        assert rel(to_np(fast.A_rec), to_np(dense.A_rec)) <= bound
        if precision == "f64":
            ref = O.tsvdm_i(A, M, 8) if mode == "I" else O.tsvdm_ii(A, M, 0.3)
            assert list(fast.rho.cpu().numpy()) == list(ref["rho"])
            assert rel(to_np(fast.A_rec), ref["A_rec"]) <= 1e-10
    with pytest.raises(ValueError):
        TSVDM(A.shape, synth.haar_orthogonal(n, np.random.default_rng(1)), transform="dct", eps=0.1)
