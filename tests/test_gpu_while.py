"""GPU parity of the while Loop with a device-evaluated stop condition
(skel_loop_while) against the oracle's loop: bit-exact image, histogram, sums
and iteration count, for stops after the first iteration, after an odd and
an even count (the result's ping-pong parity), at the limit, with host checks
every 1, 3 and 8 iterations, fused and unfused bodies."""
import numpy as np
import pytest
import torch

import oracle
import paper_1510_06585_amd as sk
import synth
from gpu_helpers import assert_image_equal, cuda

pytestmark = pytest.mark.gpu

BODIES = {
    "blur": [("blur5", {})],
    "nsbm": [("noise", {"seed": synth.NOISE_SEED}), ("solarise", {}), ("blur5", {}), ("mirror", {})],
    "noise_mirror": [("noise", {"seed": 5}), ("mirror", {})],
}


def _sums(img, stages, reduce, n):
    out, seq = img, []
    for _ in range(n):
        out, _, s = oracle.run_image_pipeline(out, stages, reduce)
        seq.append(s)
    return seq


def _run(img, stages, reduce, channel, cmp, thr, limit, every=0, options=None):
    body = sk.image_chain(stages, reduce)
    root = sk.LoopWhile(body, limit, channel, cmp, thr, every)
    H, W = img.shape[:2]
    args = [cuda(img), torch.empty((H, W, 4), dtype=torch.uint8, device="cuda")]
    if reduce == "hist_sum":
        args.append(torch.full((4, 256), 7, dtype=torch.int32, device="cuda"))
    args.append(torch.full((4,), 7, dtype=torch.int64, device="cuda"))
    args.append(torch.full((1,), 99, dtype=torch.int32, device="cuda"))
    p = sk.Plan(root, args, options)
    p.run(args)
    torch.cuda.synchronize()
    out = args[1].cpu().numpy()
    hist = args[2].cpu().numpy().view(np.uint32) if reduce == "hist_sum" else None
    s = args[-2].cpu().numpy().view(np.uint64)
    n = int(args[-1].cpu().numpy().view(np.uint32)[0])
    return p, args, out, hist, s, n


def _check(img, stages, reduce, channel, cmp, thr, limit, every=0, options=None):
    ref, rh, rs, rn = oracle.run_image_while(img, stages, reduce, channel, cmp, thr, limit)
    p, _, out, h, s, n = _run(img, stages, reduce, channel, cmp, thr, limit, every, options)
    p.destroy()
    assert n == rn, (n, rn)
    assert_image_equal(out, ref, f"while count {n}")
    assert (s == rs).all()
    if rh is not None:
        assert (h == rh).all()
    return n


@pytest.mark.parametrize("body", sorted(BODIES))
@pytest.mark.parametrize("shape", [(300, 517), (1, 1), (64, 700)], ids=["300x517", "1x1", "64x700"])
def test_while_stops_where_the_oracle_stops(body, shape):
    H, W = shape
    img = synth.image(H * 3 + W, H, W)
    stages = BODIES[body]
    seq = _sums(img, stages, "hist_sum", 6)
    counts = set()
    # continue while sum[1] != seq[k][1] in effect: pick thresholds between the
    # sums of consecutive iterations, in the direction the sequence moves
    for k in range(5):
        a, b = int(seq[k][1]), int(seq[k + 1][1])
        if a == b:
            continue
        cmp, thr = (">", b) if b < a else ("<", b)
        counts.add(_check(img, stages, "hist_sum", 1, cmp, thr, 6, every=3))
    counts.add(_check(img, stages, "hist_sum", 0, ">=", 0, 5, every=1))      # always true: runs to the limit
    counts.add(_check(img, stages, "hist_sum", 0, "<", 0, 5))                # never true: one iteration
    assert 1 in counts and 5 in counts


@pytest.mark.parametrize("options", [{}, {"fusion": sk.FUSE_OFF}, {"variant": 1}, {"tile_h": 5, "wg": 64}],
                         ids=["fused", "plain", "interpreter", "small-tiles"])
def test_while_configurations_and_parities(options):
    img = synth.image(31, 257, 333)
    stages = BODIES["nsbm"]
    for limit in (1, 2, 3, 4, 9):
        _check(img, stages, "hist_sum", 2, ">=", 0, limit, every=2, options=options)
    _check(img, stages, "sum", 3, ">=", 0, 4, options=options)


@pytest.mark.parametrize("every", [1, 2, 5])
def test_while_plan_reruns_and_checks_every_iteration(every):
    # the stop falls inside a later block of `every` iterations, with the block
    # after it already enqueued when the host reads the flag
    img = synth.image(40, 128, 260)
    stages = BODIES["blur"]
    seq = _sums(img, stages, "hist_sum", 12)
    thr = int(seq[6][0])
    p, args, out, h, s, n = _run(img, stages, "hist_sum", 0, ">", thr, 12, every=every)
    ref, rh, rs, rn = oracle.run_image_while(img, stages, "hist_sum", 0, ">", thr, 12)
    assert n == rn and (out == ref).all() and (s == rs).all()
    img2 = synth.image(41, 128, 260)          # a second run on the same plan with new data
    args[0].copy_(cuda(img2))
    p.run(args)
    torch.cuda.synchronize()
    ref2, _, rs2, rn2 = oracle.run_image_while(img2, stages, "hist_sum", 0, ">", thr, 12)
    assert int(args[-1].cpu().numpy().view(np.uint32)[0]) == rn2
    assert (args[1].cpu().numpy() == ref2).all() and (args[3].cpu().numpy().view(np.uint64) == rs2).all()
    d = p.describe()
    assert d["while"]["max"] == 12 and d["while"]["channel"] == 0
    p.destroy()


def test_while_rejections():
    body = sk.image_chain(BODIES["blur"], "hist_sum")
    with pytest.raises(sk.SkelError) as e:
        sk.LoopWhile(sk.image_chain(BODIES["blur"]), 3, 0, ">", 0)        # body is not a MapReduce
    assert e.value.status == sk.EINVAL
    with pytest.raises(sk.SkelError):
        sk.LoopWhile(body, 0, 0, ">", 0)                                    # limit below 1
    with pytest.raises(sk.SkelError):
        sk.LoopWhile(body, 3, 4, ">", 0)                                    # channel out of range
    vec = sk.image_chain([("saxpy", {"a": 1.0})], "sum")
    n = 64
    x = torch.zeros(n, device="cuda")
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.LoopWhile(vec, 3, 0, ">", 0), [x, x.clone(), x.clone(), torch.zeros(1, device="cuda"),
                                                   torch.zeros(1, dtype=torch.int32, device="cuda")])
    assert e.value.status == sk.ETYPE
    img = cuda(synth.image(1, 8, 8))
    h = torch.zeros(4, 256, dtype=torch.int32, device="cuda")
    s = torch.zeros(4, dtype=torch.int64, device="cuda")
    c = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = sk.Plan(sk.LoopWhile(body, 3, 0, ">", 0), [img, torch.empty_like(img), h, s, c])
    with pytest.raises(sk.SkelError) as e:
        p.run([img, img, h, s, c])                                          # in place is rejected
    assert e.value.status == sk.EINVAL
    p.destroy()


def test_bench_size_8192_nsbm_body():
    """The bench workload's body and size (noise>solarise>blur>mirror MapReduce on 8192^2, limit 10),
    with a threshold that stops the loop after the third iteration, checked in
    full against the oracle's loop."""
    img = synth.image(synth.SEED_PIPE_FUSED, 8192, 8192)
    st = BODIES["nsbm"]
    s = [int(x[0]) for x in _sums(img, st, "hist_sum", 3)]
    if s[2] < min(s[0], s[1]):
        cmp, thr = ">=", s[2] + 1
    elif s[2] > max(s[0], s[1]):
        cmp, thr = "<=", s[2] - 1
    else:                                   # not separable at 3: run to a limit of 3
        cmp, thr = ">=", 0
    n = _check(img, st, "hist_sum", 0, cmp, thr, 10 if thr else 3)
    assert n == 3
