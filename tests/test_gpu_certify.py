"""GPU parity of the certified t-SVDM-II selection (Algorithm 2; Section
4.1): slice energies against the oracle's, the subset Jacobi leaving the
other slices untouched and reproducing the full call bit for bit on its
own, and TSVDM(certify=True) against the oracle's full t-SVDM-II (FP64:
bit-exact ranks when the threshold margin allows, reconstruction <= 1e-10;
FP32: the same ranks as the uncertified FP32 pipeline) both when the first
round certifies and when it has to add slices or fall back to all of them."""
import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def to_dev(A, dtype):
    from paper_2605_16058_amd import ops
    out = ops.colmajor_empty(*A.shape, dtype, "cuda")
    out.copy_(torch.from_numpy(np.asfortranarray(A)).to(dtype))
    return out


def to_np(T):
    return T.detach().double().cpu().numpy()


def rel(a, b):
    d = np.linalg.norm(np.asarray(b, np.float64).ravel())
    return float(np.linalg.norm((np.asarray(a, np.float64) - b).ravel()) / (d if d > 0 else 1.0))


def smooth_tensor(m, p, n, noise, seed):
    """Low-rank in space, a few low temporal frequencies, plus noise: under
    the DCT-II most slices hold only noise."""
    g = np.random.default_rng(seed)
    t = np.arange(n)
    A = np.zeros((m, p, n))
    for l in range(6):
        a, b = g.standard_normal(m), g.standard_normal(p)
        f = g.integers(0, 3)
        A += np.einsum("i,j,t->ijt", a, b, np.cos(np.pi * f * (2 * t + 1) / (2 * n) + g.uniform(0, 1)) / (1 + l))
    return A + noise * g.standard_normal((m, p, n))


def _margin(sq, tau):
    v = np.sort(sq.ravel())
    if not np.isfinite(tau) or not np.any(v > tau):
        return 1.0
    lo = v[v <= tau].max()
    return (v[v > tau].min() - lo) / max(lo, 1e-300)


@pytest.mark.parametrize("dt,bound", [(torch.float64, 1e-14), (torch.float32, 1e-12)])
def test_slice_energy(dt, bound):
    from paper_2605_16058_amd import ops
    g = np.random.default_rng(1)
    A = g.standard_normal((33, 17, 9))
    if dt == torch.float32:
        A = A.astype(np.float32).astype(np.float64)
    E = to_np(ops.tsvdm_slice_energy(to_dev(A, dt)))
    ref = np.einsum("abi,abi->i", A, A)
    assert np.max(np.abs(E - ref) / ref) <= bound


@pytest.mark.parametrize("shape", [(40, 24, 7), (24, 40, 7)])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_subset_svd_touches_only_its_slices(shape, dt):
    from paper_2605_16058_amd import ops
    m, p, n = shape
    r = min(m, p)
    g = np.random.default_rng(2)
    A = g.standard_normal(shape)
    run = torch.tensor([1, 0, 1, 1, 0, 0, 1], dtype=torch.int32, device="cuda")
    X = to_dev(A, dt)
    W, s2, st = ops.tsvdm_slice_svd_outputs(X)
    W.fill_(7.0)
    s2.fill_(-3.0)
    ops.tsvdm_slice_svd_subset(X, run, W, s2, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    Xf = to_dev(A, dt)
    Wf, s2f, stf = ops.tsvdm_slice_svd(Xf)
    for i in range(n):
        if run[i]:
            assert torch.equal(X[:, :, i], Xf[:, :, i])
            assert torch.equal(W[i], Wf[i]) and torch.equal(s2[i], s2f[i])
        else:
            assert torch.equal(X[:, :, i], to_dev(A, dt)[:, :, i])
            assert bool((W[i] == 7.0).all()) and bool((s2[i] == -3.0).all())


@pytest.mark.parametrize("noise,eps,expect_first", [(1e-4, 1e-2, True), (3e-2, 1e-2, False)])
def test_certified_tsvdm_matches_oracle(noise, eps, expect_first):
    from paper_2605_16058_amd.pipeline import TSVDM
    m, p, n = 48, 40, 32
    A = smooth_tensor(m, p, n, noise, 5)
    M = synth.dct2_matrix(n)
    X = to_dev(A, torch.float64)
    res = TSVDM(A.shape, M, mode="II", eps=eps, precision="f64", certify=True)(X)
    torch.cuda.synchronize()
    assert int(res.svd_status.item()) == 0
    ref = O.tsvdm_ii(A, M, eps)
    computed = res.computed.cpu().numpy()
    if expect_first:
        assert res.passes == 1 and computed.sum() < n
    if _margin(ref["S"] ** 2, ref["info"]["tau"]) > 1e-10:
        assert list(res.rho.cpu().numpy()) == list(ref["rho"])
    assert rel(to_np(res.A_rec), ref["A_rec"]) <= 1e-10
    assert np.all(res.rho.cpu().numpy()[computed == 0] == 0)


def test_certified_forced_full_round():
    # max_passes = 1: an uncertified first round computes every remaining slice
    from paper_2605_16058_amd.pipeline import TSVDM
    A = smooth_tensor(32, 36, 16, 3e-2, 6)
    M = synth.dct2_matrix(16)
    X = to_dev(A, torch.float64)
    res = TSVDM(A.shape, M, mode="II", eps=1e-2, precision="f64", certify=True, theta=1.0,
                max_passes=1)(X)
    ref = O.tsvdm_ii(A, M, 1e-2)
    if res.passes > 1:
        assert int(res.computed.sum().item()) == 16
    if _margin(ref["S"] ** 2, ref["info"]["tau"]) > 1e-10:
        assert list(res.rho.cpu().numpy()) == list(ref["rho"])
    assert rel(to_np(res.A_rec), ref["A_rec"]) <= 1e-10


def test_certified_fp32_equals_uncertified():
    from paper_2605_16058_amd.pipeline import TSVDM
    m, p, n = 64, 96, 64
    A = smooth_tensor(m, p, n, 1e-4, 7).astype(np.float32).astype(np.float64)
    M = synth.dct2_matrix(n)
    X = to_dev(A, torch.float32)
    a = TSVDM(A.shape, M, mode="II", eps=1e-2, precision="f32", certify=True)(X)
    b = TSVDM(A.shape, M, mode="II", eps=1e-2, precision="f32", svd="jacobi")(X)
    assert int(a.computed.sum().item()) < n
    assert torch.equal(a.rho.cpu(), b.rho.cpu())
    assert rel(to_np(a.A_rec), to_np(b.A_rec)) <= 1e-6
