"""GPU parity of fp32 vector chains (saxpy = one fused multiply-add per stage,
reversal) against the oracle: bit-exact vectors; sums within 1e-5 * sum|v|."""
import numpy as np
import pytest
import torch

import oracle
import paper_1510_06585_amd as sk
import synth
from gpu_helpers import cuda

pytestmark = pytest.mark.gpu


def run_chain(stages, v, sides, reduce=None, options=None):
    root = sk.image_chain(stages, reduce)
    x = cuda(v)
    ws = [cuda(w) for w in sides]
    out = torch.empty_like(x)
    args = [x] + ws + [out]
    if reduce:
        args.append(torch.full((1,), 123.0, dtype=torch.float32, device="cuda"))
    p = sk.Plan(root, args, options)
    p.run(args)
    torch.cuda.synchronize()
    res = out.cpu().numpy(), (float(args[-1].cpu()[0]) if reduce else None)
    p.destroy()
    return res


def check(stages, n, seed, options, reduce="sum"):
    rng = np.random.default_rng(seed)
    v = synth.vector(seed, n)
    sides = [synth.vector(seed + 1 + k, n) for k, (nm, _) in enumerate(stages) if nm == "saxpy"]
    ref = oracle.run_f32_chain(v, stages, sides, reduce)
    out, s = run_chain(stages, v, sides, reduce, options)
    ref_v = ref[0] if reduce else ref
    assert out.tobytes() == ref_v.tobytes(), (stages, n, options)
    if reduce:
        S, A = ref[1]
        assert abs(s - S) <= 1e-5 * A + 1e-30, (s, S, A)
    del rng


ST = [("saxpy", {"a": 1.5}), ("mirror", {}), ("saxpy", {"a": -2.25}), ("saxpy", {"a": 0.0})]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 64, 1000, 4097, 65536 + 3, 1 << 20])
@pytest.mark.parametrize("options", [{}, {"fusion": sk.FUSE_OFF}, {"wg": 64, "ept": 3}, {"wg": 1024, "ept": 1},
                                     {"fusion": sk.FUSE_MASK, "split_mask": 0b1010}],
                         ids=["fused", "plain", "wg64ept3", "wg1024", "mask"])
def test_saxpy_chain_bit_exact(n, options):
    check(ST, n, 100 + n, options)


def test_saxpy_single_stage_map_and_reversal_only():
    check([("saxpy", {"a": synth.saxpy_coeff(np.random.default_rng(3))})], 10001, 5, {}, reduce=None)
    check([("mirror", {})], 10001, 6, {}, reduce=None)
    check([("mirror", {}), ("mirror", {})], 10001, 7, {}, reduce="sum")


def test_saxpy_chain_2p26():
    rng = np.random.default_rng(synth.SEED_SELECT)
    st = [("saxpy", {"a": synth.saxpy_coeff(rng)}), ("mirror", {}), ("saxpy", {"a": synth.saxpy_coeff(rng)})]
    check(st, 1 << 26, 8, {})


def test_sum_of_empty_vector_is_zero():
    out, s = run_chain([("saxpy", {"a": 2.0})], np.zeros(0, np.float32), [np.zeros(0, np.float32)], "sum")
    assert s == 0.0 and out.size == 0


def test_sum_cancellation_and_all_ones():
    n = (1 << 22) + 5
    v = np.ones(n, np.float32)
    out, s = run_chain([("mirror", {})], v, [], "sum")
    assert s == float(n)
    v = synth.vector(9, n)
    v[n // 2:] = -v[: n - n // 2][: n - n // 2]
    ref = oracle.run_f32_chain(v, [("mirror", {})], [], "sum")
    out, s = run_chain([("mirror", {})], v, [], "sum")
    S, A = ref[1]
    assert abs(s - S) <= 1e-5 * A


def test_sum_without_cancellation_at_the_bench_size():
    """5 x 10^7 values uniform in [0, 1) (no cancellation, so the plain
    relative error is well conditioned): |S - S_ref| / |S_ref| <= 1e-5, after
    a two-stage saxpy chain and after a reversal alone."""
    n = 50_000_000
    v = synth.vector(21, n, 0.0, 1.0)
    out, s = run_chain([("mirror", {})], v, [], "sum")
    S, A = oracle.run_f32_chain(v, [("mirror", {})], [], "sum")[1]
    assert S == A and abs(s - S) / abs(S) <= 1e-5, (s, S)
    w1, w2 = synth.vector(22, n, 0.0, 1.0), synth.vector(23, n, 0.0, 1.0)
    st = [("saxpy", {"a": 0.5}), ("saxpy", {"a": 1.25})]
    ref = oracle.run_f32_chain(v, st, [w1, w2], "sum")
    out, s = run_chain(st, v, [w1, w2], "sum")
    assert out.tobytes() == ref[0].tobytes()
    S = ref[1][0]
    assert S > 0 and abs(s - S) / abs(S) <= 1e-5, (s, S)


def test_random_vector_compositions():
    rng = np.random.default_rng(synth.SEED_SELECT + 1)
    done = 0
    while done < 20:
        comp = synth.composition(rng, log2_lo=4, log2_hi=18)
        if comp["domain"] != "f32":
            continue
        check(comp["stages"], comp["n"], comp["seed"] % 100000, {}, comp["reduce"])
        check(comp["stages"], comp["n"], comp["seed"] % 100000, {"fusion": sk.FUSE_OFF}, comp["reduce"])
        done += 1


def test_inplace_and_aliasing():
    n = 1000
    v = synth.vector(1, n)
    w = synth.vector(2, n)
    x = cuda(v)
    args = [x, cuda(w), x]
    p = sk.Plan(sk.Map("saxpy", a=3.0), args)
    p.run(args)
    torch.cuda.synchronize()
    assert x.cpu().numpy().tobytes() == oracle.saxpy(v, w, 3.0).tobytes()
    y = cuda(v)
    args = [y, cuda(w), y]
    p = sk.Plan(sk.Pipeline(sk.Map("saxpy", a=3.0), sk.Map("mirror")), args)
    with pytest.raises(sk.SkelError) as e:
        p.run(args)
    assert e.value.status == sk.EINVAL


def test_saxpy_near_the_2gib_limit():
    """(2^31 - 64) / 4 - 3 fp32 elements: byte offsets near the top of the
    2^31-byte vector limit, ragged against the 4-element vectors."""
    n = ((1 << 31) - 64) // 4 - 3
    check([("saxpy", {"a": 1.5})], n, 17, {}, reduce=None)
