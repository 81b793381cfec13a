"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random numbers and shapes; it holds none of the
skeleton arithmetic.  Shapes and value distributions follow the workloads the
paper benchmarks (Sec. 4: image filter pipeline on square RGBA images of
1024^2..8192^2 pixels, N-body direct sum with 8192..65536 bodies, single
precision saxpy) plus the added stages (blur, histogram, batching, cost model).
"""
from __future__ import annotations

import math

import numpy as np

# Seeds of the named workloads.
SEED_PIPE_PLAIN = 1        # 1024 x 1024 plain filter pipeline
SEED_PIPE_FUSED = 2        # 8192 x 8192 fused pipeline + MapReduce
SEED_NBODY = 3             # 65536-body Loop
SEED_BATCH = 4             # 256 uneven batched requests
SEED_SELECT = 5            # learned config selector compositions
SEED_FFT = 6               # batched 65536-point FFT pipeline
SEED_SEGMENT = 7           # gray volumes for Segmentation
NOISE_SEED = 0x1510


def image(seed: int, H: int, W: int) -> np.ndarray:
    """RGBA uint8 image, H x W x 4, every byte uniform in [0, 255]."""
    return np.random.default_rng(seed).integers(0, 256, (H, W, 4), dtype=np.uint8)


def image_rows(seed: int, H: int, W: int, y0: int, y1: int) -> np.ndarray:
    """Rows [y0, y1) of ``image(seed, H, W)`` without drawing the whole image
    (the generator draws row-major, so the rows are a contiguous slice of the
    stream: skip y0*W*4 bytes, then draw)."""
    rng = np.random.default_rng(seed)
    if y0 > 0:
        # Draw and discard in bounded chunks to keep memory small.
        left = y0 * W * 4
        while left > 0:
            k = min(left, 1 << 26)
            rng.integers(0, 256, k, dtype=np.uint8)
            left -= k
    return rng.integers(0, 256, ((y1 - y0), W, 4), dtype=np.uint8)


def complex_batch(seed: int, B: int, N: int = 65536) -> np.ndarray:
    """B complex fp32 signals of N points as float32 [B, N, 2] (re, im), every
    component uniform in [-1, 1)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (B, N, 2)).astype(np.float32)


def gray_volume(seed: int, D: int, H: int, W: int) -> np.ndarray:
    """A gray uint8 volume [D, H, W], every voxel uniform in 0..255."""
    return np.random.default_rng(seed).integers(0, 256, (D, H, W), dtype=np.uint8)


def nbody(seed: int, N: int):
    """(pos [N, 4] float32 = x, y, z, m; vel [N, 4] float32 = 0).

    Positions uniform in [-1, 1]^3 and masses uniform in [0.5, 1.5], drawn in
    float64 and rounded to float32; both sides read the same float32 buffers."""
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(-1.0, 1.0, (N, 3))
    m = rng.uniform(0.5, 1.5, N)
    pos = np.empty((N, 4), np.float32)
    pos[:, :3] = xyz.astype(np.float32)
    pos[:, 3] = m.astype(np.float32)
    return pos, np.zeros((N, 4), np.float32)


def vector(seed: int, n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """float32 vector, uniform in [lo, hi)."""
    return np.random.default_rng(seed).uniform(lo, hi, n).astype(np.float32)


def saxpy_coeff(rng: np.random.Generator) -> float:
    """A saxpy constant a ~ U[-4, 4], rounded to float32."""
    return float(np.float32(rng.uniform(-4.0, 4.0)))


def batch_sides(seed: int, nreq: int = 256):
    """Square sides of the batched requests: round(256 * 16**u), u ~ U[0, 1),
    i.e. log-uniform in [256, 4096]; sides are not rounded to multiples of 4."""
    u = np.random.default_rng(seed).uniform(0.0, 1.0, nreq)
    return [int(round(256.0 * 16.0 ** x)) for x in u]


IMAGE_OPS = ("noise", "solarise", "mirror", "blur5")
VECTOR_OPS = ("saxpy", "mirror")


def composition(rng: np.random.Generator, min_stages: int = 2, max_stages: int = 6,
                log2_lo: int = 16, log2_hi: int = 26):
    """A random skeleton composition for the config-selector workload.

    Returns a dict: ``domain`` ("u8" or "f32"), ``stages`` (list of (name, params)),
    ``reduce`` (None, "sum" or, for images, "hist_sum"), ``n`` (elements, log-uniform
    in [2^log2_lo, 2^log2_hi]) and, for images, ``H``/``W`` with W = ceil(sqrt(n)),
    H = ceil(n / W)."""
    k = int(rng.integers(min_stages, max_stages + 1))
    domain = "u8" if rng.uniform() < 0.5 else "f32"
    n = int(round(2.0 ** rng.uniform(log2_lo, log2_hi)))
    stages = []
    ops = IMAGE_OPS if domain == "u8" else VECTOR_OPS
    # The last stage may be the reduce side (a MapReduce), counted as a stage.
    with_reduce = rng.uniform() < 0.5
    nmaps = k - 1 if with_reduce else k
    nmaps = max(nmaps, 1)
    for _ in range(nmaps):
        name = ops[int(rng.integers(0, len(ops)))]
        if name == "noise":
            stages.append((name, {"seed": int(rng.integers(0, 2**32))}))
        elif name == "saxpy":
            stages.append((name, {"a": saxpy_coeff(rng)}))
        else:
            stages.append((name, {}))
    reduce = None
    if with_reduce:
        reduce = "sum" if domain == "f32" else ("hist_sum" if rng.uniform() < 0.5 else "sum")
    out = {"domain": domain, "stages": stages, "reduce": reduce, "n": n,
           "seed": int(rng.integers(0, 2**31))}
    if domain == "u8":
        W = int(math.ceil(math.sqrt(n)))
        out["W"], out["H"] = W, int(math.ceil(n / W))
    return out


def mlp_init(seed: int, n_in: int = 24, n_h1: int = 64, n_h2: int = 64) -> np.ndarray:
    """He-uniform initial weights (U[-sqrt(6/fan_in), +sqrt(6/fan_in)]), zero biases,
    flat float64 in the order W1 [h1, in], b1, W2 [h2, h1], b2, W3 [1, h2], b3."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((n_h1, n_in), (n_h2, n_h1), (1, n_h2)):
        lim = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)
