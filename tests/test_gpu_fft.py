"""GPU parity of the batched 65536-point FFT chains (the paper's FFT
benchmark: FFT pipelined with its inversion) against the oracle (numpy, in
complex128 from the same fp32 inputs).

Tolerance: per transform, ||X_gpu - X_ref||_2 / ||X_ref||_2 <= 1e-5 per
stage.  The worst-case bound for a radix-2-class fp32 FFT with twiddles
accurate to u (Higham, Thm 24.2) is log2(N) * (u + gamma_4 (sqrt 2 + u))
~ 16 * 4.6e-7 = 7.4e-6 per stage, u = 2^-24."""
import numpy as np
import pytest
import torch

import oracle
import paper_1510_06585_amd as sk
import synth

pytestmark = pytest.mark.gpu
N = 65536


def _run(x, stages, options=None):
    inp = torch.from_numpy(x).cuda()
    out = torch.empty_like(inp)
    p = sk.Plan(sk.image_chain([(s, {}) for s in stages]), [inp, out], options)
    p.run([inp, out])
    torch.cuda.synchronize()
    y = out.cpu().numpy()
    d = p.describe()
    p.destroy()
    return y[..., 0].astype(np.float64) + 1j * y[..., 1], d


def _check(x, stages, options=None):
    got, d = _run(x, stages, options)
    ref = oracle.fft_chain(x, stages)
    err = np.linalg.norm(got - ref, axis=-1) / np.linalg.norm(ref, axis=-1)
    assert err.max() <= 1e-5 * len(stages), (stages, options, err.max())
    return d, err.max()


@pytest.mark.parametrize("stages", [["fft"], ["ifft"], ["fft", "ifft"], ["fft", "fft", "ifft"],
                                    ["ifft", "fft", "fft", "ifft"]], ids=lambda s: "-".join(s))
def test_fft_chains_match_oracle(stages):
    x = synth.complex_batch(synth.SEED_FFT + len(stages), 5)
    d, _ = _check(x, stages)
    assert len(d["kernels"]) == len(stages) + 1          # fused: L + 1 passes
    d2, _ = _check(x, stages, {"fusion": sk.FUSE_OFF})
    assert len(d2["kernels"]) == 2 * len(stages)         # one kernel per half-stage
    if len(stages) >= 2:
        d3, _ = _check(x, stages, {"fusion": sk.FUSE_MASK, "split_mask": 1})
        assert len(d3["kernels"]) == len(stages) + 2


def test_fft_round_trip_and_closed_forms():
    # delta -> ones, exponential -> spike, fft then ifft -> input
    B = 3
    x = np.zeros((B, N, 2), np.float32)
    x[0, 0, 0] = 1.0
    n = np.arange(N)
    e = np.exp(2j * np.pi * 1234 * n / N)
    x[1, :, 0], x[1, :, 1] = e.real, e.imag
    x[2] = synth.complex_batch(9, 1)[0]
    got, _ = _run(x, ["fft"])
    assert np.abs(got[0] - 1.0).max() < 1e-6
    assert abs(got[1, 1234] - N) < 1e-1 and np.abs(np.delete(got[1], 1234)).max() < 1e-1
    back, _ = _run(x, ["fft", "ifft"])
    z = x[..., 0].astype(np.float64) + 1j * x[..., 1]
    assert (np.linalg.norm(back - z, axis=-1) / np.linalg.norm(z, axis=-1)).max() < 2e-5


def test_fft_batch_of_64_and_rejections():
    x = synth.complex_batch(synth.SEED_FFT, 64)
    _check(x, ["fft", "ifft"])
    t = torch.from_numpy(x).cuda()
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.image_chain([("fft", {})]), [t, t]).run([t, t])     # in place
    assert e.value.status == sk.EINVAL
    bad = torch.zeros(2, 1024, 2, device="cuda")
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.image_chain([("fft", {})]), [bad, bad.clone()])      # not 65536 points
    assert e.value.status == sk.ESHAPE
    with pytest.raises(sk.SkelError) as e:
        sk.image_chain([("fft", {}), ("mirror", {})])
        sk.Plan(sk.image_chain([("fft", {}), ("mirror", {})]), [t, torch.empty_like(t)])
    assert e.value.status == sk.ETYPE


def test_bench_size_512_transforms_every_one():
    # the bench workload (512 transforms, FFT then IFFT, fused and unfused):
    # every transform against the oracle, at the two-stage tolerance
    x = synth.complex_batch(synth.SEED_FFT, 512)
    ref = np.concatenate([oracle.fft_chain(x[i:i + 128], ["fft", "ifft"]) for i in range(0, 512, 128)])
    for opt in (None, {"fusion": sk.FUSE_OFF}):
        got, d = _run(x, ["fft", "ifft"], opt)
        err = np.linalg.norm(got - ref, axis=-1) / np.linalg.norm(ref, axis=-1)
        assert err.shape == (512,) and err.max() <= 2e-5, (opt, err.max())
        assert len(d["kernels"]) == (3 if opt is None else 4)
        del got


def test_empty_batch_runs_nothing():
    x = torch.zeros(0, N, 2, device="cuda")
    y = torch.zeros(0, N, 2, device="cuda")
    p = sk.Plan(sk.image_chain([("fft", {}), ("ifft", {})]), [x, y])
    p.run([x, y])
    torch.cuda.synchronize()
    assert y.shape == (0, N, 2)
    p.destroy()
