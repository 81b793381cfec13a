"""GPU parity of batched execution (many uneven requests in one persistent,
graph-replayed launch): every request equals the oracle's single-request
result, byte for byte, with its own histogram and sums."""
import numpy as np
import pytest
import torch

import oracle
import paper_1510_06585_amd as sk
import synth
from gpu_helpers import assert_image_equal, cuda

pytestmark = pytest.mark.gpu

PIPE_NSBM = [("noise", {"seed": synth.NOISE_SEED}), ("solarise", {}), ("blur5", {}), ("mirror", {})]


def make_reqs(sides, seed0, reduce="hist_sum"):
    reqs, imgs = [], []
    for r, (H, W) in enumerate(sides):
        img = synth.image(seed0 + r, H, W)
        x = cuda(img)
        a = [x, torch.empty_like(x)]
        if reduce == "hist_sum":
            a += [torch.full((4, 256), 5, dtype=torch.int32, device="cuda"),
                  torch.full((4,), 5, dtype=torch.int64, device="cuda")]
        reqs.append(a)
        imgs.append(img)
    return reqs, imgs


def plan_for(stages, reduce="hist_sum", options=None):
    proto = [sk.proto([8, 8, 4], sk.U8)] * 2
    if reduce == "hist_sum":
        proto += [sk.proto([4, 256], sk.U32), sk.proto([4], sk.U64)]
    return sk.Plan(sk.image_chain(stages, reduce), proto, options)


def test_small_uneven_batch_against_oracle():
    rng = np.random.default_rng(21)
    sides = [(int(rng.integers(1, 300)), int(rng.integers(1, 700))) for _ in range(40)] + [(0, 5), (3, 0)]
    reqs, imgs = make_reqs(sides, 1000)
    bound = sk.bind_batch(reqs)
    # one, two and four wavefronts per work-group take groups of consecutive tiles
    for opt in (None, {"tile_h": 16}, {"tile_h": 5, "wg": 64}, {"tile_h": 7, "wg": 128}):
        p = plan_for(PIPE_NSBM, options=opt)
        for rep in range(2):   # capture, then replay of the same request set (pre-marshalled)
            for a in reqs:
                a[1].fill_(7)
            p.batch_run(reqs if rep == 0 else bound)
            torch.cuda.synchronize()
            for (H, W), img, a in zip(sides, imgs, reqs):
                ref, rh, rs = oracle.run_image_pipeline(img, PIPE_NSBM, "hist_sum")
                assert_image_equal(a[1].cpu().numpy(), ref, f"{H}x{W} {opt} rep{rep}")
                assert (a[2].cpu().numpy().view(np.uint32) == rh).all()
                assert (a[3].cpu().numpy().view(np.uint64) == rs).all()


def test_pointwise_batch_without_reduce():
    st = [("noise", {"seed": 4}), ("mirror", {}), ("solarise", {})]
    sides = [(5, 9), (300, 257), (1, 1), (64, 1000)]
    reqs, imgs = make_reqs(sides, 50, reduce=None)
    p = plan_for(st, reduce=None)
    p.batch_run(reqs)
    torch.cuda.synchronize()
    for img, a in zip(imgs, reqs):
        assert_image_equal(a[1].cpu().numpy(), oracle.run_image_pipeline(img, st), "pointwise batch")


@pytest.mark.parametrize("options", [None, {"tile_h": 64}], ids=["bench_default_plan", "tile64"])
def test_256_uneven_requests_every_one_against_oracle(options):
    """The batched workload the benchmark times (256 square requests, sides
    log-uniform in [256, 4096], noise > solarise > blur > mirror + histogram,
    the plan's default tiles and work-groups), replayed from its captured
    graph: every request's image, histogram and sums equal the oracle's."""
    sides = synth.batch_sides(synth.SEED_BATCH, 256)
    reqs, imgs = make_reqs([(s, s) for s in sides], 4000)
    p = plan_for(PIPE_NSBM, options=options)
    bound = sk.bind_batch(reqs)
    p.batch_run(bound)                    # capture
    torch.cuda.synchronize()
    for a in reqs:                        # clobber every output, then replay the graph
        a[1].fill_(3)
        a[2].fill_(3)
        a[3].fill_(3)
    p.batch_run(bound)
    torch.cuda.synchronize()
    print(p.describe()["batch_grid"], "work-groups", options)
    for r in range(256):
        a = reqs[r]
        ref, rh, rs = oracle.run_image_pipeline(imgs[r], PIPE_NSBM, "hist_sum")
        assert_image_equal(a[1].cpu().numpy(), ref, f"request {r} side {sides[r]} {options}")
        assert (a[2].cpu().numpy().view(np.uint32) == rh).all(), f"request {r} hist"
        assert (a[3].cpu().numpy().view(np.uint64) == rs).all(), f"request {r} sum"


def test_batch_needs_a_fused_plan():
    p = plan_for(PIPE_NSBM, options={"fusion": sk.FUSE_OFF})
    reqs, _ = make_reqs([(4, 4)], 1)
    with pytest.raises(sk.SkelError) as e:
        p.batch_run(reqs)
    assert e.value.status == sk.EUNSUPPORTED


def test_batch_tuner_choice_matches_oracle(tmp_path):
    """skel_tune_batch on an uneven batch: the exhaustive search times all 30
    points (10 tile heights x 3 work-group sizes) and logs each after one
    provenance line; the Algorithm-1 walk times a subset of them; the batched
    run with either choice equals the oracle for every request."""
    rng = np.random.default_rng(23)
    sides = [(int(s), int(s)) for s in np.round(64 * 16 ** rng.random(24))]
    sides[3] = (37, 1001)
    reqs, imgs = make_reqs(sides, 7000)
    root = sk.image_chain(PIPE_NSBM, "hist_sum")
    db = str(tmp_path / "batch.db")
    best, us, timed = sk.tune_batch(root, reqs, db, reps=5)
    assert timed == 30 and us > 0
    lines = open(db).read().splitlines()
    assert lines[0].startswith("# skel tuning session: tuner=batch-exhaustive")
    rows = [l for l in lines if not l.startswith("#")]
    assert len(rows) == 30 and all(r.startswith("batch24|px") for r in rows)
    assert min(float(r.split(",")[-2]) for r in rows) == pytest.approx(us, rel=1e-3)
    best_p, us_p, timed_p = sk.tune_batch(root, reqs, db, reps=5, pruned=True, precision_us=1.0)
    assert 1 <= timed_p < 30
    for opt in (best, best_p):
        assert opt["fusion"] == sk.FUSE_ON and opt["wg"] in (64, 128, 256)
        p = plan_for(PIPE_NSBM, options={"tile_h": opt["tile_h"], "wg": opt["wg"]})
        for a in reqs:
            a[1].fill_(3)
            a[2].fill_(3)
        p.batch_run(reqs)
        torch.cuda.synchronize()
        for (H, W), img, a in zip(sides, imgs, reqs):
            ref, rh, rs = oracle.run_image_pipeline(img, PIPE_NSBM, "hist_sum")
            assert_image_equal(a[1].cpu().numpy(), ref, f"{H}x{W} tuned {opt}")
            assert (a[2].cpu().numpy().view(np.uint32) == rh).all()
            assert (a[3].cpu().numpy().view(np.uint64) == rs).all()
        p.destroy()


def test_batch_at_the_request_limit():
    """65535 requests (the tile -> request table holds 16-bit request
    indices), tiny images of 1..3 x 1..5 pixels carved from one buffer, in
    one persistent launch: every request's image, histogram and sums equal the
    oracle's; one more request is rejected."""
    n = 65535
    rng = np.random.default_rng(29)
    Hs = rng.integers(1, 4, n)
    Ws = rng.integers(1, 6, n)
    px = Hs * Ws
    off = np.concatenate([[0], np.cumsum(px)])
    flat_in = rng.integers(0, 256, (int(off[-1]), 4), dtype=np.uint8)
    x = cuda(flat_in)
    y = torch.empty_like(x)
    hist = torch.full((n, 4, 256), 5, dtype=torch.int32, device="cuda")
    sums = torch.full((n, 4), 5, dtype=torch.int64, device="cuda")
    reqs = []
    for r in range(n):
        a, b = int(off[r]), int(off[r + 1])
        reqs.append([x[a:b].view(int(Hs[r]), int(Ws[r]), 4), y[a:b].view(int(Hs[r]), int(Ws[r]), 4), hist[r],
                     sums[r]])
    p = plan_for(PIPE_NSBM)
    p.batch_run(reqs)
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    hh = hist.cpu().numpy().view(np.uint32)
    ss = sums.cpu().numpy().view(np.uint64)
    for r in range(0, n, 1):
        a, b = int(off[r]), int(off[r + 1])
        img = flat_in[a:b].reshape(int(Hs[r]), int(Ws[r]), 4)
        ref, rh, rs = oracle.run_image_pipeline(img, PIPE_NSBM, "hist_sum")
        assert (out[a:b].reshape(ref.shape) == ref).all(), r
        assert (hh[r] == rh).all() and (ss[r] == rs).all(), r
    with pytest.raises(sk.SkelError) as e:
        p.batch_run(reqs + [reqs[0]])
    assert e.value.status == sk.EUNSUPPORTED
    p.destroy()
