"""GPU parity of the batch path (many ragged tensors through one plan).

The batch kernels are the single-tensor kernels driven by task tables, so
with the same Jacobi block width a batch must reproduce the single-tensor
results bit for bit (ranks, reconstruction); the error sums use another
reduction split and agree to rounding.  Against the FP64 oracle the FP64
batch meets the same bounds as the single-tensor path; hipGraph replays must
equal the eager run exactly.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth
from paper_2605_16058_amd._lib import GRAM_LDS_MAX_R, GRAM_MAX_R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def to_dev(A, dtype):
    out = torch.empty((A.shape[2], A.shape[1], A.shape[0]), dtype=dtype, device="cuda").permute(2, 1, 0)
    out.copy_(torch.from_numpy(np.asfortranarray(A)).to(dtype))
    return out

def plan_gram_jacobi(shapes):
    """Where a FP32 batch plan runs the Gram form's Jacobi: in LDS when every
    tensor has min(m, p) <= GRAM_LDS_MAX_R, else in the block rounds."""
    return "lds" if all(min(s[0], s[1]) <= GRAM_LDS_MAX_R for s in shapes) else "rounds"



def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (d if d > 0 else 1.0))


@pytest.fixture(scope="module")
def ragged():
    return synth.workload("ragged", small=True)


@pytest.mark.parametrize("precision,dtype", [("f64", torch.float64), ("f32", torch.float32)])
def test_batch_equals_single_tensor_calls(ragged, precision, dtype):
    from paper_2605_16058_amd.pipeline import BatchTSVDM, tsvdm
    w = ragged
    Ts = [to_dev(A, torch.float32) for A in w.A]
    b = BatchTSVDM(Ts, w.M, w.mode, ks=w.k, epss=w.eps, precision=precision, block=16)
    st = b.run(host_poll=True)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    gj = plan_gram_jacobi([A.shape for A in Ts])
    for t, A in enumerate(Ts):
        # the plan's choice of slice SVD: the Gram form for FP32 slices with
        # min(m, p) <= GRAM_MAX_R, the rotation form otherwise
        svd = "gram" if precision == "f32" and min(A.shape[0], A.shape[1]) <= GRAM_MAX_R else "jacobi"
        res = tsvdm(A, w.M[t], mode=w.mode[t], k=w.k[t], eps=w.eps[t], precision=precision, block=16,
                    svd=svd, guard="bound", gram_jacobi=gj)
        torch.cuda.synchronize()
        assert torch.equal(res.rho, b.rho[t]), t
        assert torch.equal(res.offsets, b.offsets[t]), t
        assert torch.equal(res.A_rec, b.A_rec[t]), t
        e1, e2 = res.err.cpu().numpy(), b.err[t].cpu().numpy()
        assert np.allclose(e1, e2, rtol=1e-12, atol=1e-300), t


@pytest.mark.parametrize("precision,dtype", [("f64", torch.float64), ("f32", torch.float32)])
def test_batch_host_poll_matches_fixed_steps(ragged, precision, dtype):
    # the host reads the count of unconverged slices one poll behind the
    # queued steps; the result must equal running every step without reading
    from paper_2605_16058_amd.pipeline import BatchTSVDM
    w = ragged
    n = 24
    Ts = [to_dev(A, torch.float32) for A in w.A[:n]]
    b = BatchTSVDM(Ts, w.M[:n], w.mode[:n], ks=w.k[:n], epss=w.eps[:n], precision=precision)
    st = b.run(host_poll=True)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ref = [a.clone() for a in b.A_rec]
    ref_rho = [r.clone() for r in b.rho]
    for a in b.A_rec:
        a.zero_()
    st = b.run(host_poll=False)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    for t in range(n):
        assert torch.equal(b.rho[t], ref_rho[t]), t
        assert torch.equal(b.A_rec[t], ref[t]), t


def test_batch_fp64_matches_oracle(ragged):
    from paper_2605_16058_amd.pipeline import BatchTSVDM
    w = ragged
    Ts = [to_dev(A, torch.float32) for A in w.A]
    b = BatchTSVDM(Ts, w.M, w.mode, ks=w.k, epss=w.eps, precision="f64", keep_factors=True)
    st = b.run()
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    errs = b.rel_errors()
    for t, A in enumerate(w.A):
        A64 = A.astype(np.float64)
        ref = O.tsvdm_i(A64, w.M[t], w.k[t]) if w.mode[t] == "I" else O.tsvdm_ii(A64, w.M[t], w.eps[t])
        rho = b.rho[t].cpu().numpy()
        if w.mode[t] == "I":
            assert np.array_equal(rho, ref["rho"])
        sq = np.sort((ref["S"] ** 2).ravel())
        tau = ref["info"].get("tau", None)
        margin_ok = True
        if w.mode[t] == "II" and tau is not None and np.isfinite(tau):
            lo = sq[sq <= tau].max()
            hi = sq[sq > tau].min() if np.any(sq > tau) else np.inf
            margin_ok = (hi - lo) / max(lo, 1e-300) > 1e-10
        if margin_ok:
            assert np.array_equal(rho, ref["rho"]), t
            assert rel(b.A_rec[t].cpu().numpy(), ref["A_rec"]) <= 1e-10, t
            # |err - err_oracle| <= |A_rec - A_rec_oracle| / |A| by the triangle
            # inequality; below ~1e-13 both errors are FP64 rounding of A_rec
            assert abs(errs[t] - ref["rel_error"]) <= 1e-9 * ref["rel_error"] + 1e-13, t
        # packed singular values are the oracle's leading ones
        off = b.offsets[t].cpu().numpy()
        S = b.S_pk[t].cpu().numpy()
        for i in range(A.shape[2]):
            k = int(rho[i])
            assert np.allclose(S[off[i]: off[i] + k], ref["S"][:k, i], rtol=0,
                               atol=1e-12 * max(ref["S"][0, i], 1e-300))


def test_batch_graph_replays_equal_eager(ragged):
    from paper_2605_16058_amd.pipeline import BatchTSVDM
    w = ragged
    Ts = [to_dev(A, torch.float32) for A in w.A[:8]]
    b = BatchTSVDM(Ts, w.M[:8], w.mode[:8], ks=w.k[:8], epss=w.eps[:8], precision="f32")
    b.run(host_poll=True)
    torch.cuda.synchronize()
    ref = [a.clone() for a in b.A_rec]
    ref_rho = [r.clone() for r in b.rho]
    junk = torch.randn(1 << 20, device="cuda")
    side = torch.cuda.Stream()  # graphs are captured on a non-default stream
    for rep in range(3):
        for a in b.A_rec:
            a.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            st = b.run(use_graph=True)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        for t in range(len(Ts)):
            assert torch.equal(b.A_rec[t], ref[t]), (rep, t)
            assert torch.equal(b.rho[t], ref_rho[t]), (rep, t)
        # eager work between replays
        junk.mul_(1.0001).add_(0.5)
        b.run(host_poll=True)
        torch.cuda.synchronize()
        for t in range(len(Ts)):
            assert torch.equal(b.A_rec[t], ref[t]), (rep, t)


@pytest.mark.parametrize("block", [16, 32])
def test_batch_mixed_routes_equal_single_calls(block):
    """FP32 batches whose tensors take every slice-SVD route (the Gram form
    up to GRAM_MAX_R with the Jacobi in the block rounds, or in LDS when the
    whole batch is small; the rotation form above GRAM_MAX_R) equal the
    single-tensor calls of the same form bit for bit, and their FP32 errors
    stay below eps.  Block 32 (pairs of 64 vectors) runs the batched round
    instance with checked loads at four workgroups per compute unit."""
    from paper_2605_16058_amd.pipeline import BatchTSVDM, tsvdm
    g = np.random.default_rng(77)
    shapes = [(40, 60, 5), (210, 230, 3), (150, 90, 4), (230, 200, 2), (129, 300, 2), (128, 128, 2),
              (96, 180, 3), (GRAM_MAX_R + 6, GRAM_MAX_R + 12, 1)]
    As, Ms, modes, ks, epss = [], [], [], [], []
    for t, (m, p, n) in enumerate(shapes):
        A = g.standard_normal((m, p, n)) + 3.0 * np.einsum("a,b,c->abc", g.standard_normal(m),
                                                           g.standard_normal(p), g.standard_normal(n))
        As.append(A.astype(np.float32))
        Ms.append(synth.haar_orthogonal(n, g))
        modes.append("I" if t % 2 == 0 else "II")
        ks.append(7 if t % 2 == 0 else None)
        epss.append(None if t % 2 == 0 else 0.3)
    Ts = [to_dev(A, torch.float32) for A in As]
    small = [t for t, (m, p, n) in enumerate(shapes) if min(m, p) <= GRAM_LDS_MAX_R]
    for sel in (list(range(len(shapes))), small):
        gj = plan_gram_jacobi([shapes[t] for t in sel])
        print(f"batch of {len(sel)} tensors, Gram-form Jacobi: {gj}", flush=True)
        b = BatchTSVDM([Ts[t] for t in sel], [Ms[t] for t in sel], [modes[t] for t in sel],
                       ks=[ks[t] for t in sel], epss=[epss[t] for t in sel], precision="f32", block=block)
        st = b.run(host_poll=True)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        errs = b.rel_errors()
        for i, t in enumerate(sel):
            A = Ts[t]
            svd = "gram" if min(A.shape[0], A.shape[1]) <= GRAM_MAX_R else "jacobi"
            print(f"tensor {t} {tuple(A.shape)}: {svd} form, rel error {errs[i]:.6e}", flush=True)
            res = tsvdm(A, Ms[t], mode=modes[t], k=ks[t], eps=epss[t], precision="f32", block=block, svd=svd,
                        guard="bound", gram_jacobi=gj)
            torch.cuda.synchronize()
            assert torch.equal(res.rho, b.rho[i]), t
            assert torch.equal(res.A_rec, b.A_rec[i]), t
            if modes[t] == "II":
                assert errs[i] < epss[t]