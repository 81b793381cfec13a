"""Pins of the oracle's FFT chain (numpy's FFT as the step) against closed forms
and a direct DFT written from the definition, so a wrong sign, scaling or
axis fails here."""
import numpy as np
import pytest

import oracle


def _pack(z):
    return np.stack([z.real, z.imag], axis=-1).astype(np.float32)


def test_fft_of_delta_and_constant():
    N = 65536
    x = np.zeros((2, N), np.complex128)
    x[0, 0] = 1.0
    x[1, :] = 1.0
    X = oracle.fft_chain(_pack(x), ["fft"])
    assert np.abs(X[0] - 1.0).max() < 1e-12
    assert abs(X[1, 0] - N) < 1e-9 and np.abs(X[1, 1:]).max() < 1e-9


def test_fft_of_complex_exponential_is_a_spike():
    N = 65536
    n = np.arange(N)
    for k0 in (1, 257, 40000):
        x = np.exp(2j * np.pi * k0 * n / N)      # forward transform: spike of height N at k0
        X = oracle.fft_chain(_pack(x), ["fft"])
        assert abs(X[k0] - N) < 1e-2 and np.abs(np.delete(X, k0)).max() < 1e-2
        Y = oracle.fft_chain(_pack(x), ["ifft"])  # inverse: spike of height 1 at N - k0
        assert abs(Y[(N - k0) % N] - 1.0) < 1e-6


@pytest.mark.parametrize("N", [8, 64])
def test_small_transforms_against_direct_dft(N):
    rng = np.random.default_rng(N)
    x = rng.uniform(-1, 1, (3, N)) + 1j * rng.uniform(-1, 1, (3, N))
    x = x.astype(np.complex64).astype(np.complex128)
    n = np.arange(N)
    F = np.exp(-2j * np.pi * np.outer(n, n) / N)          # X[k] = sum_n x[n] e^{-2 pi i nk/N}
    got = oracle.fft_chain(_pack(x), ["fft"])
    assert np.allclose(got, x @ F.T, atol=1e-9)
    inv = oracle.fft_chain(_pack(x), ["ifft"])
    assert np.allclose(inv, x @ F.conj().T / N, atol=1e-9)


def test_round_trip_and_parseval():
    x = np.random.default_rng(1).uniform(-1, 1, (2, 65536, 2)).astype(np.float32)
    z = x[..., 0].astype(np.float64) + 1j * x[..., 1]
    X = oracle.fft_chain(x, ["fft"])
    assert np.allclose((np.abs(X) ** 2).sum(-1), 65536 * (np.abs(z) ** 2).sum(-1), rtol=1e-12)
    back = oracle.fft_chain(x, ["fft", "ifft"])
    assert np.abs(back - z).max() < 1e-12


def test_full_length_bins_against_direct_sums():
    # at the real transform length, a few output bins of the forward and
    # inverse stages written out as the defining sums (fp64, O(N) per bin)
    N = 65536
    rng = np.random.default_rng(1234)
    x = (rng.uniform(-1, 1, N) + 1j * rng.uniform(-1, 1, N)).astype(np.complex64).astype(np.complex128)
    X = oracle.fft_chain(_pack(x[None]), ["fft"])[0]
    Y = oracle.fft_chain(_pack(x[None]), ["ifft"])[0]
    n = np.arange(N)
    for k in (0, 1, 255, 256, 4097, 32768, 65535):
        fwd = np.sum(x * np.exp(-2j * np.pi * ((n * k) % N) / N))
        inv = np.sum(x * np.exp(2j * np.pi * ((n * k) % N) / N)) / N
        assert abs(X[k] - fwd) <= 1e-9 * max(1.0, abs(fwd)), (k, X[k], fwd)
        assert abs(Y[k] - inv) <= 1e-12 * max(1.0, abs(inv)) + 1e-13, (k, Y[k], inv)
