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


def _run_full(img, stages, reduce, channel, cmp, thr, limit, every=0, kind="value", carried=(), init_hist=None,
              init_sum=None, options=None):
    """Runs a while plan with the given initial reduce-output contents and
    returns the plan, its arguments and (out, hist, sum, count)."""
    H, W = img.shape[:2]
    mask = 0
    sum_arg = 3 if reduce == "hist_sum" else 2
    if "hist" in carried:
        mask |= 1 << 2
    if "sum" in carried:
        mask |= 1 << sum_arg
    body = sk.image_chain(stages, reduce)
    root = sk.LoopWhile(body, limit, channel, cmp, thr, every, carried_mask=mask, kind=kind)
    args = [cuda(img), torch.empty((H, W, 4), dtype=torch.uint8, device="cuda")]
    if reduce == "hist_sum":
        args.append(cuda(np.asarray(init_hist, np.uint32).view(np.int32)))
    args.append(cuda(np.asarray(init_sum, np.uint64).view(np.int64)))
    args.append(torch.full((1,), 99, dtype=torch.int32, device="cuda"))
    p = sk.Plan(root, args, options)
    p.run(args)
    torch.cuda.synchronize()
    out = args[1].cpu().numpy()
    hist = args[2].cpu().numpy().view(np.uint32) if reduce == "hist_sum" else None
    s = args[-2].cpu().numpy().view(np.uint64)
    n = int(args[-1].cpu().numpy().view(np.uint32)[0])
    return p, args, (out, hist, s, n)


def _check_full(img, stages, reduce, channel, cmp, thr, limit, every=0, kind="value", carried=(), seed=0,
                options=None):
    rng = np.random.default_rng(seed)
    # initial reduce-output contents: large values, so that a carried u32
    # count wraps and a non-carried output is visibly overwritten
    ih = rng.integers(0, 2 ** 32, (4, 256), dtype=np.uint64).astype(np.uint32)
    isum = rng.integers(0, 2 ** 63, 4, dtype=np.uint64)
    ref, rh, rs, rn = oracle.run_image_while(img, stages, reduce, channel, cmp, thr, limit, kind=kind,
                                             carried=carried, init_hist=ih, init_sum=isum)
    p, _, (out, h, s, n) = _run_full(img, stages, reduce, channel, cmp, thr, limit, every, kind, carried, ih, isum,
                                     options)
    d = p.describe()
    p.destroy()
    assert n == rn, (n, rn)
    assert_image_equal(out, ref, f"while count {n}")
    assert (s == rs).all(), (s, rs)
    if rh is not None:
        assert (h == rh).all()
    return n, d


def _stop_threshold(seq, k, channel):
    """A value condition on seq[i][channel] that holds for i < k and fails at k
    (None when the sums do not separate there)."""
    v = [int(x[channel]) for x in seq]
    if v[k] < min(v[:k]):
        return ">", v[k]
    if v[k] > max(v[:k]):
        return "<", v[k]
    return None


@pytest.mark.parametrize("carried", [("hist", "sum"), ("hist",), ("sum",), ()],
                         ids=["hist+sum", "hist", "sum", "none"])
@pytest.mark.parametrize("every", [0, 2, -1], ids=["blocks8", "blocks2", "async"])
def test_while_carried_outputs_merge_by_addition(carried, every):
    """Carried reduce outputs are the caller's initial contents plus the sum
    of every iteration's result (uint32 counts wrap); the others hold the last
    iteration's; the condition reads the iteration's own sums."""
    img = synth.image(77, 300, 517)
    stages = BODIES["nsbm"]
    seq = _sums(img, stages, "hist_sum", 6)
    stops = set()
    for k in (1, 2, 4):
        c = _stop_threshold(seq, k, 2)
        if c is None:
            continue
        n, d = _check_full(img, stages, "hist_sum", 2, c[0], c[1], 6, every, "value", carried, seed=k)
        stops.add(n)
        assert d["loop_carried"] == ((4 if "hist" in carried else 0) | (8 if "sum" in carried else 0))
    n, _ = _check_full(img, stages, "hist_sum", 0, ">=", 0, 5, every, "value", carried, seed=9)    # to the limit
    assert n == 5 and len(stops) >= 2


@pytest.mark.parametrize("every", [0, -1], ids=["blocks8", "async"])
def test_while_sum_only_body_carried(every):
    img = synth.image(78, 129, 250)
    stages = BODIES["noise_mirror"]
    for carried in (("sum",), ()):
        _check_full(img, stages, "sum", 1, ">=", 0, 3, every, "value", carried, seed=3)


@pytest.mark.parametrize("body", ["blur", "nsbm"])
def test_while_convergence_condition(body):
    """kind "delta": continue while |s_i - s_(i-1)| cmp T; the first iteration
    has no predecessor and always continues.  Thresholds between consecutive
    changes of the sum stop the loop where the oracle's loop stops."""
    img = synth.image(79, 200, 311)
    stages = BODIES[body]
    seq = [int(x[1]) for x in _sums(img, stages, "hist_sum", 8)]
    deltas = [abs(seq[i] - seq[i - 1]) for i in range(1, 8)]
    counts = set()
    for i in range(1, 5):
        # stop at iteration i + 1: deltas[0..i-2] satisfy the condition, deltas[i-1] does not
        prior = deltas[:i - 1]
        d = deltas[i - 1]
        if d == 0:
            continue
        if not prior or d > max(prior):
            cmp, thr = "<=", d - 1
        elif d < min(prior):
            cmp, thr = ">=", d + 1
        else:
            continue
        n, desc = _check_full(img, stages, "hist_sum", 1, cmp, thr, 8, 3, "delta", ("sum",), seed=i)
        counts.add(n)
        assert desc["while"]["kind"] == "delta"
    # never satisfied: the first iteration continues, the second stops
    n, _ = _check_full(img, stages, "hist_sum", 1, "<", 0, 8, 0, "delta")
    assert n == 2
    # limit 1: one iteration whatever the condition
    n, _ = _check_full(img, stages, "hist_sum", 1, "<", 0, 1, -1, "delta", ("hist", "sum"))
    assert n == 1
    assert len(counts) >= 2, counts


def test_while_async_run_does_not_wait_and_reruns():
    """check_every < 0: the run returns after enqueuing every guarded
    iteration; results match the oracle once the stream is synchronised, and
    a second run of the same plan on the same buffers starts over."""
    img = synth.image(80, 256, 300)
    stages = BODIES["blur"]
    seq = _sums(img, stages, "hist_sum", 10)
    c = _stop_threshold(seq, 3, 0)
    assert c is not None
    ih = np.zeros((4, 256), np.uint32)
    isum = np.zeros(4, np.uint64)
    p, args, (out, h, s, n) = _run_full(img, stages, "hist_sum", 0, c[0], c[1], 10, -1, "value", ("sum",), ih, isum)
    ref, rh, rs, rn = oracle.run_image_while(img, stages, "hist_sum", 0, c[0], c[1], 10, carried=("sum",))
    assert n == rn == 4 and (out == ref).all() and (h == rh).all() and (s == rs).all()
    p.run(args)                     # carried sums accumulate on top of the first run's
    torch.cuda.synchronize()
    ref2, rh2, rs2, rn2 = oracle.run_image_while(img, stages, "hist_sum", 0, c[0], c[1], 10, carried=("sum",),
                                                 init_sum=rs)
    assert int(args[-1].cpu().numpy().view(np.uint32)[0]) == rn2
    assert (args[1].cpu().numpy() == ref2).all()
    assert (args[3].cpu().numpy().view(np.uint64) == rs2).all()
    p.destroy()
