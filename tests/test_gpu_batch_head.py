"""Planned batches whose levels 1 and 2 run as one head launch over every
image (DWT2_PLAN_HEAD).

The head runs the same per-quad arithmetic as one launch per level (and as the
fused tail), so every output must equal the single-image transform bit for
bit, whatever the batch, the grid or the storage type; against the oracle the
FP32 bound is 1e-5 of max|x|.
"""
import numpy as np
import pytest

import oracle
import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_08266_amd as dwt  # noqa: E402
from paper_1705_08266_amd import batch as dwb  # noqa: E402


def _images(n, lo=32, hi=1024, multiple=32, seed=21, dtype=torch.float32):
    sizes = synthetic.batch_sizes(n, lo, hi, multiple, seed=seed)
    return [torch.from_numpy(synthetic.uniform_image(h, w, seed=seed + i)).to("cuda").to(dtype)
            for i, (w, h) in enumerate(sizes)]


@pytest.mark.parametrize("wavelet", ["cdf97", "cdf53"])
@pytest.mark.parametrize("scheme", ["nonseparable", "separable"])
def test_head_batch_forward_equals_single_and_oracle(wavelet, scheme):
    imgs = _images(16)
    print(f"case head batch forward {wavelet} {scheme}", flush=True)
    plan = dwb.BatchPlan.forward(imgs, 3, wavelet, scheme, fuse_head=True)
    total, per = plan.launches()
    assert per[0] == 1 and per[1] == 0 and total == 1 + per[2]
    plan.run()
    torch.cuda.synchronize()
    for x, c in zip(imgs, plan.outputs):
        assert torch.equal(dwt.forward(x, wavelet, 3, scheme), c)
    for x, c in list(zip(imgs, plan.outputs))[:4]:
        ref = oracle.forward(x.cpu().numpy().astype(np.float64), wavelet, 3)
        assert np.abs(c.cpu().numpy() - ref).max() <= 1e-5 * 255


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("levels", [2, 3])
def test_head_batch_inverse_and_round_trip(persistent, levels):
    imgs = _images(24, hi=2048, seed=31)
    print(f"case head batch L={levels} persistent={persistent}", flush=True)
    fwd = dwb.BatchPlan.forward(imgs, levels, fuse_head=True, persistent=persistent)
    fwd.run()
    inv = dwb.BatchPlan.inverse_of(fwd.outputs, levels, fuse_head=True, persistent=persistent)
    inv.run()
    torch.cuda.synchronize()
    for x, c, r in zip(imgs, fwd.outputs, inv.outputs):
        assert torch.equal(dwt.forward(x, "cdf97", levels), c)
        assert torch.equal(dwt.inverse(c, "cdf97", levels), r)
        assert (r - x).abs().max().item() <= 1e-5 * 255


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
@pytest.mark.parametrize("scheme", ["nonseparable", "separable"])
def test_head_batch_16_bit_equals_single(dtype, scheme):
    imgs = _images(10, lo=64, seed=41, dtype=dtype)
    print(f"case head batch {dtype} {scheme}", flush=True)
    fwd = dwb.BatchPlan.forward(imgs, 3, scheme=scheme, fuse_head=True)
    fwd.run()
    inv = dwb.BatchPlan.inverse_of(fwd.outputs, 3, scheme=scheme, fuse_head=True)
    inv.run()
    torch.cuda.synchronize()
    for x, c, r in zip(imgs, fwd.outputs, inv.outputs):
        assert torch.equal(dwt.forward(x, "cdf97", 3, scheme), c)
        assert torch.equal(dwt.inverse(c, "cdf97", 3, scheme), r)


def test_head_batch_graph_replays_match_eager():
    imgs = _images(12, seed=51)
    print("case head batch graph replay", flush=True)
    plan = dwb.BatchPlan.forward(imgs, 3, fuse_head=True)
    plan.run()
    torch.cuda.synchronize()
    eager = [o.clone() for o in plan.outputs]
    plan.capture()
    for _ in range(3):
        for o in plan.outputs:            # eager work between replays
            o.zero_()
        plan.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, plan.outputs):
            assert torch.equal(a, b)


@pytest.mark.parametrize("inverse", [False, True])
def test_head_batch_tiny_and_ragged_images(inverse):
    sizes = [(4, 4), (8, 4), (4, 8), (12, 8), (36, 20), (260, 132), (116, 44), (232, 72)]
    imgs = [torch.from_numpy(synthetic.uniform_image(h, w, seed=61 + i)).to("cuda")
            for i, (w, h) in enumerate(sizes)]
    print(f"case head batch tiny/ragged inverse={inverse}", flush=True)
    srcs = [dwt.forward(x, "cdf97", 2) for x in imgs] if inverse else imgs
    plan = (dwb.BatchPlan.inverse_of(srcs, 2, fuse_head=True) if inverse
            else dwb.BatchPlan.forward(srcs, 2, fuse_head=True))
    plan.run()
    torch.cuda.synchronize()
    for s, o in zip(srcs, plan.outputs):
        single = dwt.inverse(s, "cdf97", 2) if inverse else dwt.forward(s, "cdf97", 2)
        assert torch.equal(single, o), tuple(s.shape)
