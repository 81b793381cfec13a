"""CPU oracle for the skeleton hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product (the HIP library under
``paper_1510_06585_amd/``) never imports it and shares no code with it.

Every skeleton is executed stage by stage, each stage reading a whole input
and materialising a whole output: the depth-first, one-kernel-at-a-time
single-device execution of a skeleton computational tree (the overview of
the framework in Sec. 2).  The per-stage arithmetic of the image, vector and
N-body stages lives in ``oracle.c`` (plain C loops); the cost-model MLP is in
``oracle/mlp.py`` (numpy, fp64); Segmentation is written out in numpy below
and the FFT stages use numpy's FFT in complex128 as their step.

Stage descriptions used here are plain tuples ``(name, params)`` with names
``"noise"`` (params ``{"seed": int}``), ``"solarise"``, ``"mirror"``,
``"blur5"`` and, for fp32 vectors, ``"saxpy"`` (params ``{"a": float}``, plus
one side vector per saxpy stage) and ``"mirror"`` (reversal).  Segmentation
chains are lists of ``(lo, hi)`` threshold pairs and FFT chains lists of
``"fft"`` / ``"ifft"``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "_oracle.so")
_lib = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64 = ctypes.c_int64


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc into ``_oracle.so`` (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_fmix32.restype = ctypes.c_uint32
        L.orc_fmix32.argtypes = [ctypes.c_uint32]
        L.orc_noise_offset.restype = ctypes.c_int
        L.orc_noise_offset.argtypes = [ctypes.c_uint32, _i64, _i64, ctypes.c_int]
        L.orc_noise.restype = ctypes.c_int
        L.orc_noise.argtypes = [_u8p, _u8p, _i64, _i64, ctypes.c_uint32]
        L.orc_solarise.argtypes = [_u8p, _u8p, _i64]
        L.orc_mirror.argtypes = [_u8p, _u8p, _i64, _i64]
        L.orc_blur5.argtypes = [_u8p, _u8p, _i64, _i64]
        L.orc_hist_sum.argtypes = [_u8p, _i64, _i64, _u32p, _u64p]
        L.orc_saxpy.argtypes = [_f32p, _f32p, ctypes.c_float, _f32p, _i64]
        L.orc_reverse_f32.argtypes = [_f32p, _f32p, _i64]
        L.orc_sum_f32.argtypes = [_f32p, _i64, _f64p, _f64p]
        L.orc_nbody_accel.argtypes = [_f64p, _f64p, _i64, ctypes.c_double, ctypes.c_double]
        L.orc_nbody_run.restype = ctypes.c_int
        L.orc_nbody_run.argtypes = [_f64p, _f64p, _i64, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _p(a: np.ndarray, t):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(t)


def _img(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype != np.uint8 or a.ndim != 3 or a.shape[2] != 4:
        raise ValueError("image must be uint8 H x W x 4")
    return a


# ----------------------------------------------------------------- image stages
def fmix32(h: int) -> int:
    return int(lib().orc_fmix32(h & 0xFFFFFFFF))


def noise_offset(seed: int, x: int, y: int, c: int) -> int:
    return int(lib().orc_noise_offset(seed & 0xFFFFFFFF, x, y, c))


def noise(img: np.ndarray, seed: int) -> np.ndarray:
    img = _img(img)
    H, W, _ = img.shape
    out = np.empty_like(img)
    if lib().orc_noise(_p(img, _u8p), _p(out, _u8p), W, H, seed & 0xFFFFFFFF) != 0:
        raise ValueError("noise needs W, H <= 65536")
    return out


def solarise(img: np.ndarray) -> np.ndarray:
    img = _img(img)
    out = np.empty_like(img)
    lib().orc_solarise(_p(img, _u8p), _p(out, _u8p), img.size)
    return out


def mirror(img: np.ndarray) -> np.ndarray:
    img = _img(img)
    H, W, _ = img.shape
    out = np.empty_like(img)
    lib().orc_mirror(_p(img, _u8p), _p(out, _u8p), W, H)
    return out


def blur5(img: np.ndarray) -> np.ndarray:
    img = _img(img)
    H, W, _ = img.shape
    out = np.empty_like(img)
    lib().orc_blur5(_p(img, _u8p), _p(out, _u8p), W, H)
    return out


def hist_sum(img: np.ndarray):
    """MapReduce reduce side: (hist uint32 [4, 256], sum uint64 [4]) of an RGBA image."""
    img = _img(img)
    H, W, _ = img.shape
    hist = np.zeros((4, 256), np.uint32)
    s = np.zeros(4, np.uint64)
    lib().orc_hist_sum(_p(img, _u8p), W, H, _p(hist, _u32p), _p(s, _u64p))
    return hist, s


_IMAGE_STAGES = {
    "noise": lambda img, prm: noise(img, prm["seed"]),
    "solarise": lambda img, prm: solarise(img),
    "mirror": lambda img, prm: mirror(img),
    "blur5": lambda img, prm: blur5(img),
}


def run_image_pipeline(img: np.ndarray, stages, reduce: str | None = None):
    """Pipeline of Map stages over an RGBA image (Sec. 2.1, Pipeline and Map), each
    stage materialised in turn; ``reduce`` = ``"hist_sum"`` or ``"sum"`` appends the
    MapReduce reduce side over the final image.  Returns ``out`` or ``(out, hist, sum)``
    (``hist`` is None for ``"sum"``)."""
    cur = _img(img)
    for name, prm in stages:
        cur = _IMAGE_STAGES[name](cur, prm or {})
    if reduce is None:
        return cur
    hist, s = hist_sum(cur)
    if reduce == "hist_sum":
        return cur, hist, s
    if reduce == "sum":
        return cur, None, s
    raise ValueError(reduce)


_CMP = {">": lambda v, t: v > t, ">=": lambda v, t: v >= t, "<": lambda v, t: v < t, "<=": lambda v, t: v <= t}


def run_image_while(img: np.ndarray, stages, reduce: str, channel: int, cmp: str, threshold: int,
                    max_iterations: int, kind: str = "value", carried=(), init_hist=None, init_sum=None):
    """While Loop over a MapReduce body (Sec. 2.1, Loop: while loops whose state
    holds the stop condition, the items updated after every iteration, and
    whether that update needs a global synchronisation; Sec. 3.4, partial
    results merged by a merging function).

    Each iteration runs the body (``stages`` then ``reduce``) on the current
    image, giving that iteration's image, histogram h_i and channel sums s_i,
    and counts itself.  The loop repeats while the condition holds and fewer
    than ``max_iterations`` iterations have run (the body runs at least once):

    * ``kind="value"``: ``s_i[channel] cmp threshold``;
    * ``kind="delta"`` (convergence of the reduction):
      ``|s_i[channel] - s_(i-1)[channel]| cmp threshold``; the first iteration
      has no predecessor and always continues.

    The condition reads the iteration's own sums.  The loop state's outputs
    are the last image and the reduce outputs: an output named in ``carried``
    (``"hist"``, ``"sum"``) is carried across iterations and merged by addition,
    starting from ``init_hist`` / ``init_sum`` (zeros if None); any other
    reduce output is the last iteration's.  Returns ``(out, hist, sum, count)``
    (``hist`` is None for ``reduce="sum"``)."""
    if kind not in ("value", "delta"):
        raise ValueError(kind)
    cur = _img(img)
    count = 0
    acc_h = np.zeros((4, 256), np.uint64) if init_hist is None else np.asarray(init_hist).astype(np.uint64)
    acc_s = np.zeros(4, np.uint64) if init_sum is None else np.asarray(init_sum).astype(np.uint64)
    prev = None
    while True:
        cur, hist, s = run_image_pipeline(cur, stages, reduce)
        count += 1
        if hist is not None:
            acc_h = acc_h + hist.astype(np.uint64)
        acc_s = acc_s + s
        v = int(s[channel])
        if kind == "value":
            go = _CMP[cmp](v, int(threshold))
        else:
            go = True if prev is None else _CMP[cmp](abs(v - prev), int(threshold))
        prev = v
        if count >= max_iterations or not go:
            break
    out_h = None
    if hist is not None:
        # uint32 outputs wrap modulo 2^32 like the device counters
        out_h = (acc_h % (1 << 32)).astype(np.uint32) if "hist" in carried else hist
    out_s = acc_s if "sum" in carried else s
    return cur, out_h, out_s, count


# ---------------------------------------------------------- Segmentation stages
SEGMENT_LO, SEGMENT_HI = 85, 170


def segment(vol: np.ndarray, lo: int = SEGMENT_LO, hi: int = SEGMENT_HI) -> np.ndarray:
    """Segmentation (Sec. 4): every voxel of a gray uint8 volume becomes black
    (0), gray (128) or white (255).  The paper does not give the thresholds;
    the reading here: black below ``lo``, white from ``hi`` up, gray between
    (defaults split 0..255 into three equal ranges of 85 values)."""
    v = np.asarray(vol)
    if v.dtype != np.uint8:
        raise ValueError("volume must be uint8")
    if not 0 <= lo <= hi <= 256:
        raise ValueError("need 0 <= lo <= hi <= 256")
    out = np.full(v.shape, 128, np.uint8)
    out[v < lo] = 0
    out[v >= hi] = 255
    return out


def run_segment_chain(vol: np.ndarray, stages) -> np.ndarray:
    """Pipeline (Sec. 2) of Segmentation stages, each materialised: stages
    are (lo, hi) pairs, (0, 0) for the default thresholds."""
    cur = np.asarray(vol)
    for lo, hi in stages:
        cur = segment(cur, lo, hi) if (lo or hi) else segment(cur)
    return cur


# ------------------------------------------------------------------ FFT stages
def fft_chain(x: np.ndarray, stages):
    """Pipeline of FFT / IFFT stages (Sec. 4 FFT, pipelined with its inversion)
    over the last axis of ``x`` (float32 [..., N, 2] as interleaved re, im),
    each stage materialised in complex128 with numpy's FFT (the library FFT is
    the step; the forward transform uses exp(-2 pi i nk / N), the inverse
    exp(+2 pi i nk / N) / N).  Returns complex128 [..., N]."""
    x = np.asarray(x)
    cur = x[..., 0].astype(np.float64) + 1j * x[..., 1].astype(np.float64)
    for name in stages:
        if name == "fft":
            cur = np.fft.fft(cur, axis=-1)
        elif name == "ifft":
            cur = np.fft.ifft(cur, axis=-1)
        else:
            raise ValueError(name)
    return cur


# ------------------------------------------------------------------ fp32 stages
def _f32(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype != np.float32 or a.ndim != 1:
        raise ValueError("vector must be 1-D float32")
    return a


def saxpy(v: np.ndarray, w: np.ndarray, a: float) -> np.ndarray:
    v, w = _f32(v), _f32(w)
    if v.shape != w.shape:
        raise ValueError("saxpy operands differ in length")
    out = np.empty_like(v)
    lib().orc_saxpy(_p(v, _f32p), _p(w, _f32p), np.float32(a), _p(out, _f32p), v.size)
    return out


def reverse(v: np.ndarray) -> np.ndarray:
    v = _f32(v)
    out = np.empty_like(v)
    lib().orc_reverse_f32(_p(v, _f32p), _p(out, _f32p), v.size)
    return out


def sum_f32(v: np.ndarray):
    """(sum, sum of |v|) of an fp32 vector, accumulated in fp64."""
    v = _f32(v)
    s = ctypes.c_double()
    a = ctypes.c_double()
    lib().orc_sum_f32(_p(v, _f32p), v.size, ctypes.byref(s), ctypes.byref(a))
    return s.value, a.value


def run_f32_chain(v: np.ndarray, stages, sides, reduce: str | None = None):
    """Pipeline of fp32 Map stages; ``sides[k]`` is the side vector of the k-th saxpy
    stage.  ``reduce="sum"`` returns ``(out, (sum, abs_sum))``."""
    cur = _f32(v)
    k = 0
    for name, prm in stages:
        if name == "saxpy":
            cur = saxpy(cur, sides[k], prm["a"])
            k += 1
        elif name == "mirror":
            cur = reverse(cur)
        else:
            raise ValueError(name)
    if reduce is None:
        return cur
    if reduce == "sum":
        return cur, sum_f32(cur)
    raise ValueError(reduce)


# ---------------------------------------------------------------------- N-body
def nbody_accel(pos4: np.ndarray, G: float = 1.0, eps: float = 1e-2) -> np.ndarray:
    """fp64 accelerations (N x 3) of bodies ``pos4`` = N x 4 (x, y, z, m)."""
    p = np.ascontiguousarray(pos4, dtype=np.float64)
    N = p.shape[0]
    acc = np.zeros((N, 3), np.float64)
    lib().orc_nbody_accel(_p(p, _f64p), _p(acc, _f64p), N, G, eps)
    return acc


def nbody_run(pos4, vel, steps: int, G: float = 1.0, eps: float = 1e-2, dt: float = 1e-3):
    """Loop skeleton over (force -> kick-drift) in fp64, started from the given
    (fp32 or fp64) state; returns (pos N x 4, vel N x 3) in fp64."""
    p = np.array(pos4, dtype=np.float64, order="C", copy=True)
    v = np.array(np.asarray(vel)[:, :3], dtype=np.float64, order="C", copy=True)
    N = p.shape[0]
    if lib().orc_nbody_run(_p(p, _f64p), _p(v, _f64p), N, steps, G, eps, dt) != 0:
        raise MemoryError("oracle n-body allocation failed")
    return p, v
