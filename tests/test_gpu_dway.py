"""GPU parity of the order-d path (Section 2.1, footnote; Section 3.1):
tsvdm_transform_mode against the oracle's mode-k product on every mode of
order-4/5 tensors (middle modes with many blocks and the last mode), the
block loop beyond one launch's grid, bit-identity with the 3-way calls, and
TSVDMd against the oracle's tsvdm_d (FP64: ranks bit-exact when the
threshold margin allows, reconstruction <= 1e-10; FP32: <= 3e-5)."""
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


def rel(a, b):
    d = np.linalg.norm(np.asarray(b, np.float64).ravel())
    return float(np.linalg.norm((np.asarray(a, np.float64) - b).ravel()) / (d if d > 0 else 1.0))


@pytest.mark.parametrize("dims", [(7, 5, 3, 4, 6), (33, 17, 9, 5), (1, 3, 2, 70)])
@pytest.mark.parametrize("compute,dt,bound", [("f64", torch.float64, 1e-13), ("f32", torch.float32, 3e-6)])
def test_transform_mode_matches_oracle(dims, compute, dt, bound):
    from paper_2605_16058_amd import ops
    g = np.random.default_rng(sum(dims))
    A = g.standard_normal(dims)
    X = to_dev_nd(A, dt)
    for k in range(3, len(dims) + 1):
        M = synth.haar_orthogonal(dims[k - 1], g)
        Md = ops.device_matrix(M)
        Y = ops.tsvdm_transform_mode(X, k, Md, compute=compute, out_dtype=dt)
        ref = O.mode_product(A, M, k)
        assert rel(Y.double().cpu().numpy(), ref) <= bound, k
        # transpose with a scale, every tile shape gives the same bits
        Z = [ops.tsvdm_transform_mode(X, k, Md, transpose=True, scale=0.5, compute=compute,
                                      out_dtype=dt, tile=t) for t in (0, 1, 2, 3)]
        torch.cuda.synchronize()
        refT = O.mode_product(A, 0.5 * M.T, k)
        assert rel(Z[0].double().cpu().numpy(), refT) <= bound, k
        for t in range(1, 4):
            assert torch.equal(Z[0], Z[t])


def test_transform_mode_many_blocks():
    """P = 70000 blocks: more than one launch's grid height."""
    from paper_2605_16058_amd import ops
    g = np.random.default_rng(1)
    A = g.standard_normal((2, 3, 5, 70000))
    M = synth.dct2_matrix(5)
    Y = ops.tsvdm_transform_mode(to_dev_nd(A, torch.float64), 3, ops.device_matrix(M), compute="f64")
    torch.cuda.synchronize()
    assert rel(Y.cpu().numpy(), O.mode_product(A, M, 3)) <= 1e-13


def test_mode3_of_3way_is_tsvdm_transform():
    from paper_2605_16058_amd import ops
    g = np.random.default_rng(2)
    A = g.standard_normal((40, 30, 12))
    X = to_dev_nd(A, torch.float32)
    Md = ops.device_matrix(synth.haar_orthogonal(12, g))
    a = ops.tsvdm_transform_mode(X, 3, Md, compute="f32", out_dtype=torch.float32)
    b = ops.tsvdm_transform(X, Md, compute="f32", out_dtype=torch.float32)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_tsvdmd_order3_equals_tsvdm():
    from paper_2605_16058_amd.pipeline import TSVDMd, tsvdm
    w = synth.workload("climate", small=True)
    A = to_dev_nd(w.A, torch.float32)
    a = TSVDMd(w.A.shape, [w.M], mode="II", eps=1e-2, precision="f32")(A)
    b = tsvdm(A, w.M, mode="II", eps=1e-2, precision="f32")
    torch.cuda.synchronize()
    assert torch.equal(a.rho, b.rho) and torch.equal(a.A_rec, b.A_rec)


# The FP32 reconstruction bound (pipeline.RECON_BOUND): against the oracle's
# truncation at the same tolerance, relative to ||A||, plus the energy of the
# squared singular values between the two ranks where a rank differs; with the
# guard the FP32 path selects with eps - FP32_REL and its error stays below eps
FP32_REL = 3e-5


def _flipped(S, rho_a, rho_b):
    """Energy of the oracle's squared singular values (S: r x N) ranked
    between rho_a[i] and rho_b[i]: the squared distance of the two truncations."""
    tot = 0.0
    for i in range(S.shape[1]):
        a, b = sorted((int(rho_a[i]), int(rho_b[i])))
        tot += float(np.sum(S[a:b, i] ** 2))
    return tot


def _margin(S, tau):
    v = np.sort((S ** 2).ravel())
    if not np.isfinite(tau) or not np.any(v > tau):
        return 1.0
    lo = v[v <= tau].max()
    return (v[v > tau].min() - lo) / max(lo, 1e-300)


@pytest.mark.parametrize("dims,mode,arg", [((20, 14, 6, 5), "II", 0.05), ((12, 18, 3, 4, 5), "II", 0.2),
                                           ((16, 16, 7, 3), "I", 5)])
def test_tsvdmd_matches_oracle(dims, mode, arg):
    from paper_2605_16058_amd.pipeline import TSVDMd
    g = np.random.default_rng(len(dims) * 100 + dims[0])
    A = g.standard_normal(dims) + 4.0 * np.einsum(
        "a,b,c->abc", g.standard_normal(dims[0]), g.standard_normal(dims[1]),
        g.standard_normal(int(np.prod(dims[2:])))).reshape(dims, order="F")
    Ms = [synth.haar_orthogonal(n, g) if i % 2 == 0 else synth.dct2_matrix(n)
          for i, n in enumerate(dims[2:])]
    kw = {"eps": arg} if mode == "II" else {"k": arg}
    ref = O.tsvdm_d(A, Ms, mode=mode, **kw)
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        res = TSVDMd(dims, Ms, mode=mode, precision=prec, **kw)(to_dev_nd(A, dt))
        torch.cuda.synchronize()
        assert int(res.svd_status.item()) == 0 and int(res.pack_status.item()) == 0
        rho = res.rho.cpu().numpy()
        same = np.array_equal(rho, ref["rho"])
        if prec == "f64":
            if mode == "I" or _margin(ref["S"], ref["info"]["tau"]) > 1e-10:
                assert same
            nA = np.linalg.norm(A)
            d = rel(res.A_rec.cpu().numpy(), ref["A_rec"]) * np.linalg.norm(ref["A_rec"]) / nA
            assert d <= 1e-10 + np.sqrt(_flipped(ref["S"], rho, ref["rho"])) / nA
            # ranks from the GPU's own squares through the oracle's selection
            if mode == "II":
                rho_o, _ = O.ranks_tolerance(res.s2.cpu().numpy().T, arg, squared=True)
                assert np.array_equal(rho, rho_o)
        else:
            r32 = ref if mode == "I" else O.tsvdm_d(A, Ms, mode=mode, eps=res.eps_sel)
            nA = np.linalg.norm(A)
            d = rel(res.A_rec.double().cpu().numpy(), r32["A_rec"]) * np.linalg.norm(r32["A_rec"]) / nA
            flip = np.sqrt(_flipped(r32["S"], rho, r32["rho"])) / nA
            assert d <= FP32_REL + flip, (d, flip)
        if mode == "II":
            assert res.rel_error() < arg


def test_climate6_small_matches_oracle():
    """The order-6 climate recipe at test size, FP64 and FP32, against tsvdm_d."""
    from paper_2605_16058_amd.pipeline import TSVDMd
    w = synth.workload("climate6", small=True)
    A64 = w.A.astype(np.float64)
    ref = O.tsvdm_d(A64, w.M, mode="II", eps=w.eps)
    for prec, bound in (("f64", 1e-10), ("f32", 3e-5)):
        res = TSVDMd(w.A.shape, w.M, mode="II", eps=w.eps, precision=prec)(to_dev_nd(w.A, torch.float32))
        torch.cuda.synchronize()
        rho = res.rho.cpu().numpy()
        rho_o, _ = O.ranks_tolerance(res.s2.cpu().numpy().T, res.eps_sel, squared=True)
        assert np.array_equal(rho, rho_o)
        r_o = ref if prec == "f64" else O.tsvdm_d(A64, w.M, mode="II", eps=res.eps_sel)
        if prec == "f64":
            assert np.array_equal(rho, r_o["rho"]) or _margin(r_o["S"], r_o["info"]["tau"]) <= 1e-10
        nA = np.linalg.norm(A64)
        d = rel(res.A_rec.double().cpu().numpy(), r_o["A_rec"]) * np.linalg.norm(r_o["A_rec"]) / nA
        flip = np.sqrt(_flipped(r_o["S"], rho, r_o["rho"])) / nA
        print(f"{prec}: |A_rec - oracle| / |A| = {d:.3e}, flipped {flip:.3e}")
        assert d <= bound + flip, (prec, d, flip)
        assert res.rel_error() < w.eps
