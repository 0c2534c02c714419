"""The head level batches (dwt2_forward_head_batch / dwt2_inverse_head_batch):
two consecutive levels of many images per launch, the band between them in
LDS. Each pair must give exactly the outputs of the two level jobs run one
after the other with the level batches, in every storage type, for pairs at
the finest levels and deeper in the pyramid, down to 4 x 4 inputs; and the
serving loop must give the same results with and without fused heads."""
import pytest

import synthetic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1705_08266_amd as dwt  # noqa: E402
from paper_1705_08266_amd import _lib, load  # noqa: E402
from paper_1705_08266_amd import serving as sv  # noqa: E402

SIZES = [(4, 4), (8, 4), (4, 8), (8, 8), (64, 32), (520, 264), (1024, 768), (232, 72),
         (2048, 1024), (96, 1600)]


def _requests(levels, inverse, tdt, seed):
    """(src, out, ws0, ws1, jobs) per size: jobs in execution order."""
    reqs = []
    for i, (w, h) in enumerate(SIZES):
        if w % (1 << levels) or h % (1 << levels):
            continue
        x = torch.from_numpy(synthetic.uniform_image(h, w, seed=seed + i)).to("cuda").to(tdt)
        src = dwt.forward(x, "cdf97", levels) if inverse else x
        out = torch.zeros_like(src)
        ws0 = torch.zeros((w // 2) * (h // 2), dtype=torch.float32, device="cuda")
        ws1 = torch.zeros(max(1, (w // 4) * (h // 4)), dtype=torch.float32, device="cuda")
        reqs.append((src, out, ws0, ws1, sv.level_jobs(src, out, ws0, ws1, levels, inverse)))
    return reqs


def _run_levels(reqs, ks, inverse):
    lib = load()
    fn = lib.dwt2_inverse_level_batch if inverse else lib.dwt2_forward_level_batch
    for k in ks:
        jobs = [r[4][k] for r in reqs]
        arr = (_lib.LevelJob * len(jobs))(*jobs)
        _lib.check(fn(arr, len(jobs), 0, 0, None, None), "level batch")


def _run_head(reqs, pair_levels, levels, inverse, scheme=0):
    lib = load()
    fn = lib.dwt2_inverse_head_batch if inverse else lib.dwt2_forward_head_batch
    jobs = []
    for r in reqs:
        index = {(levels - k if inverse else k + 1): k for k in range(levels)}
        jobs += [r[4][index[pair_levels[0]]], r[4][index[pair_levels[1]]]]
    arr = (_lib.LevelJob * len(jobs))(*jobs)
    _lib.check(fn(arr, len(jobs) // 2, 0, scheme, None), "head batch")


@pytest.mark.parametrize("tdt", [torch.float32, torch.float16, torch.bfloat16])
@pytest.mark.parametrize("inverse", [False, True])
def test_head_pair_equals_two_level_jobs(tdt, inverse):
    print(f"case head batch levels 1-2 {tdt} inverse={inverse}", flush=True)
    a = _requests(2, inverse, tdt, seed=100)
    b = _requests(2, inverse, tdt, seed=100)
    _run_levels(a, [0, 1], inverse)
    _run_head(b, (1, 2), 2, inverse)
    torch.cuda.synchronize()
    for ra, rb in zip(a, b):
        assert torch.equal(ra[1], rb[1]), tuple(ra[0].shape)


@pytest.mark.parametrize("inverse", [False, True])
def test_head_pair_deeper_in_the_pyramid(inverse):
    """Levels 3 and 4 of a 4-level transform as one head, the rest per level."""
    print(f"case head batch levels 3-4 inverse={inverse}", flush=True)
    L = 4
    a = _requests(L, inverse, torch.float16, seed=200)
    b = _requests(L, inverse, torch.float16, seed=200)
    _run_levels(a, range(L), inverse)
    if inverse:           # execution order 4, 3, 2, 1: the pair first
        _run_head(b, (3, 4), L, inverse)
        _run_levels(b, [2, 3], inverse)
    else:
        _run_levels(b, [0, 1], inverse)
        _run_head(b, (3, 4), L, inverse)
    torch.cuda.synchronize()
    for ra, rb in zip(a, b):
        assert torch.equal(ra[1], rb[1]), tuple(ra[0].shape)


def test_serving_gives_the_same_results_with_and_without_fused_heads():
    trace = synthetic.request_stream(30, 5000.0, lo=64, hi=1024, seed=33)
    reqs, inputs = [], {}
    for r in trace:
        x = torch.from_numpy(synthetic.uniform_image(r.side, r.side, seed=r.seed)).to("cuda")
        x = x.to(torch.float16)
        inputs[r.rid] = dwt.forward(x, "cdf97", r.levels) if r.inverse else x
        reqs.append(sv.Request(r.rid, r.arrival_s, r.side, r.side, r.levels, r.inverse))
    torch.cuda.synchronize()
    print("case serving fused vs per-level", flush=True)
    fused = sv.Server(fuse_heads=True)
    plain = sv.Server(fuse_heads=False)
    rf = {r.rid: r.output for r in fused.run(reqs, inputs, keep_outputs=True, realtime=False)}
    rp = {r.rid: r.output for r in plain.run(reqs, inputs, keep_outputs=True, realtime=False)}
    torch.cuda.synchronize()
    assert fused.iterations < plain.iterations
    for rid in rp:
        assert torch.equal(rf[rid], rp[rid]), rid
