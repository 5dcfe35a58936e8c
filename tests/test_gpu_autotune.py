"""GPU checks of the tuned knobs: every transform tile shape gives the same
bits, a batch with mixed per-item block widths and tile shapes reproduces the
single-tensor calls with the same choices bit for bit, and the autotuner's
choices are valid and reusable from its cache."""
import numpy as np
import pytest

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



@pytest.mark.parametrize("shape", [(70, 50, 20), (33, 17, 5), (130, 3, 64), (300, 7, 33), (40, 30, 140)])
@pytest.mark.parametrize("compute,dt", [("f64", torch.float64), ("f32", torch.float32),
                                        ("bf16x3", torch.float32), ("bf16", torch.float32)])
def test_transform_tiles_bit_identical(shape, compute, dt):
    from paper_2605_16058_amd import ops
    g = np.random.default_rng(7 + shape[2])
    A = to_dev(g.standard_normal(shape), dt)
    Md = ops.device_matrix(synth.haar_orthogonal(shape[2], g))
    outs = [ops.tsvdm_transform(A, Md, compute=compute, out_dtype=dt, tile=t) for t in range(9)]
    torch.cuda.synchronize()
    for t in range(1, 9):
        assert torch.equal(outs[0], outs[t]), t


def test_batch_mixed_blocks_and_tiles_equal_single_calls():
    from paper_2605_16058_amd.pipeline import BatchTSVDM, tsvdm
    w = synth.workload("ragged", small=True)
    Ts = [to_dev(A, torch.float32) for A in w.A]
    cnt = len(Ts)
    blocks = [16 if t % 3 else 32 for t in range(cnt)]
    tiles = [1 + t % 8 for t in range(cnt)]
    b = BatchTSVDM(Ts, w.M, w.mode, ks=w.k, epss=w.eps, precision="f32", blocks=blocks, tiles=tiles)
    st = b.run(host_poll=True)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    gj = plan_gram_jacobi([A.shape for A in Ts])
    for t, A in enumerate(Ts):
        svd = "gram" if min(A.shape[0], A.shape[1]) <= GRAM_MAX_R else "jacobi"
        res = tsvdm(A, w.M[t], mode=w.mode[t], k=w.k[t], eps=w.eps[t], precision="f32",
                    block=blocks[t], tile=tiles[t], svd=svd, guard="bound", gram_jacobi=gj)
        torch.cuda.synchronize()
        assert torch.equal(res.rho, b.rho[t]), t
        assert torch.equal(res.A_rec, b.A_rec[t]), t


def test_tune_batch_choices_are_valid_and_cached(tmp_path):
    from paper_2605_16058_amd import autotune
    from paper_2605_16058_amd.pipeline import BatchTSVDM
    w = synth.workload("ragged", small=True)
    Ts = [to_dev(A, torch.float32) for A in w.A]
    path = str(tmp_path / "tune.json")
    blocks, tiles, report = autotune.tune_batch(Ts, w.M, w.mode, ks=w.k, epss=w.eps,
                                                precision="f32", cache=path, sample=12, reps=1)
    assert len(blocks) == len(Ts) and len(tiles) == len(Ts)
    assert set(blocks) <= {16, 32} and set(tiles) <= set(range(9))
    assert report
    # a second call is served from the cache: no timing, same answer
    b2, t2, rep2 = autotune.tune_batch(Ts, w.M, w.mode, ks=w.k, epss=w.eps, precision="f32",
                                       cache=path, sample=12, reps=1)
    assert rep2 == {}
    sampled = set(autotune._sample(list(range(len(Ts))), 12))
    for i in sampled:
        assert b2[i] == blocks[i] and t2[i] == tiles[i]
    bt = BatchTSVDM(Ts, w.M, w.mode, ks=w.k, epss=w.eps, precision="f32", blocks=blocks, tiles=tiles)
    assert int(bt.run().item()) == 0


def test_tune_tsvdm_single_tensor(tmp_path):
    from paper_2605_16058_amd import autotune
    from paper_2605_16058_amd.pipeline import tsvdm
    w = synth.workload("climate", small=True)
    A = to_dev(w.A, torch.float32)
    ch = autotune.tune_tsvdm(A, w.M, mode="II", eps=1e-2, precision="f32",
                             cache=str(tmp_path / "t.json"), reps=1)
    assert ch.block in (16, 32) and ch.tile in range(1, 9)
    res = tsvdm(A, w.M, mode="II", eps=1e-2, precision="f32", block=ch.block, tile=ch.tile)
    assert int(res.svd_status.item()) == 0
