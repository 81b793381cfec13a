"""Pins of the image-stage oracle against facts fixed outside it: published hash
vectors, hand-derived golden cases, closed forms, invariants and library routines."""
import os

import numpy as np
import pytest
import scipy.ndimage

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand(seed, H, W):
    return synth.image(seed, H, W)


# ------------------------------------------------------------------ noise
def test_fmix32_published_vectors(orc):
    # MurmurHash3_x86_32 with an empty key reduces to fmix32(seed); values are the
    # published test vectors (see tests/golden/noise_hash_vectors.txt).
    assert orc.fmix32(0) == 0
    assert orc.fmix32(1) == 0x514E28B7
    assert orc.fmix32(0xFFFFFFFF) == 0x81F16F39
    assert orc.fmix32(0xE6546B60) == 0x2362F9DE


def _noise_cases():
    rows = []
    with open(os.path.join(GOLD, "noise_hash_vectors.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            t = line.split()
            rows.append((int(t[0], 16), int(t[1]), int(t[2]),
                         [int(v) for v in t[3:7]], [int(v) for v in t[7:11]]))
    return rows


@pytest.mark.parametrize("case", _noise_cases())
def test_noise_golden(orc, case):
    seed, x, y, pin, pout = case
    W, H = 9, 6
    img = _rand(11, H, W)
    img[y, x] = pin
    out = orc.noise(img, seed)
    assert list(out[y, x]) == pout


def test_noise_offsets_range_and_coverage(orc):
    img = np.full((64, 96, 4), 128, np.uint8)
    out = orc.noise(img, 0x1510).astype(int) - 128
    assert out.min() == -16 and out.max() == 16
    assert len(np.unique(out)) == 33
    # roughly uniform over the 33 offsets (256 = 7*33 + 25 byte values)
    counts = np.bincount((out + 16).ravel(), minlength=33)
    assert counts.min() > 0.5 * counts.mean()


def test_noise_clamps(orc):
    lo = np.zeros((8, 8, 4), np.uint8)
    hi = np.full((8, 8, 4), 255, np.uint8)
    assert orc.noise(lo, 5).max() <= 16
    assert orc.noise(hi, 5).min() >= 239
    # noise depends on the pixel coordinate: a different seed gives a different field
    a, b = orc.noise(np.full((8, 8, 4), 100, np.uint8), 1), orc.noise(np.full((8, 8, 4), 100, np.uint8), 2)
    assert (a != b).any()


def test_noise_rejects_oversized(orc):
    with pytest.raises(ValueError):
        orc.noise(np.zeros((1, 65537, 4), np.uint8), 0)


# ----------------------------------------------------------------- solarise
def test_solarise_exhaustive(orc):
    v = np.arange(256, dtype=np.uint8).reshape(1, 64, 4)
    s = orc.solarise(v).ravel().astype(int)
    ref = np.minimum(np.arange(256), 255 - np.arange(256))   # equivalent closed form
    assert (s == ref).all()
    assert s.max() == 127
    assert (orc.solarise(orc.solarise(v)) == orc.solarise(v)).all()     # idempotent
    fixed = np.arange(128)
    assert (s[fixed] == fixed).all()                                      # fixed points v <= 127


# ------------------------------------------------------------------- mirror
@pytest.mark.parametrize("H,W", [(1, 1), (3, 5), (17, 33), (8, 1)])
def test_mirror_is_row_reversal(orc, H, W):
    img = _rand(H * 100 + W, H, W)
    m = orc.mirror(img)
    assert (m == img[:, ::-1, :]).all()         # library reversal of whole pixels
    assert (orc.mirror(m) == img).all()          # involution


def test_mirror_commutes_with_pointwise_and_blur_not_noise(orc):
    img = _rand(3, 9, 7)
    assert (orc.mirror(orc.solarise(img)) == orc.solarise(orc.mirror(img))).all()
    assert (orc.mirror(orc.blur5(img)) == orc.blur5(orc.mirror(img))).all()
    assert (orc.mirror(orc.noise(img, 9)) != orc.noise(orc.mirror(img), 9)).any()


# --------------------------------------------------------------------- blur
def _blur_cases():
    cases, cur = [], None
    with open(os.path.join(GOLD, "blur5_impulse.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            t = line.split()
            if t[0] == "case":
                cur = {"W": int(t[1]), "H": int(t[2]), "px": int(t[3]), "py": int(t[4]),
                       "V": int(t[5]), "rows": []}
                cases.append(cur)
            else:
                cur["rows"].append([int(v) for v in t])
    return cases


@pytest.mark.parametrize("case", _blur_cases(), ids=lambda c: "W%dH%d_%d_%d_V%d" % (c["W"], c["H"], c["px"], c["py"], c["V"]))
def test_blur_golden_impulses(orc, case):
    img = np.zeros((case["H"], case["W"], 4), np.uint8)
    img[case["py"], case["px"], 0] = case["V"]
    out = orc.blur5(img)
    assert out[:, :, 0].tolist() == case["rows"]
    assert (out[:, :, 1:] == 0).all()


@pytest.mark.parametrize("H,W", [(1, 1), (2, 3), (13, 17), (31, 9), (64, 70)])
def test_blur_matches_library_correlate(orc, H, W):
    img = _rand(H * 7 + W, H, W)
    out = orc.blur5(img)
    # scipy's correlate with mode='nearest' is clamp-to-edge; exact integer sums
    ref = scipy.ndimage.correlate(img.astype(np.int64), np.ones((5, 5, 1), np.int64), mode="nearest") // 25
    assert (out == ref.astype(np.uint8)).all()


def test_blur_constant_and_bounds(orc):
    for v in (0, 1, 77, 127, 255):
        img = np.full((11, 6, 4), v, np.uint8)
        assert (orc.blur5(img) == v).all()
    img = orc.solarise(_rand(5, 20, 20))
    assert orc.blur5(img).max() <= 127


# ------------------------------------------------------------ hist and sum
@pytest.mark.parametrize("H,W", [(1, 1), (5, 7), (64, 33)])
def test_hist_sum_library(orc, H, W):
    img = _rand(H + W, H, W)
    hist, s = orc.hist_sum(img)
    for c in range(4):
        assert (hist[c] == np.bincount(img[:, :, c].ravel(), minlength=256)).all()
        assert int(s[c]) == int(img[:, :, c].astype(np.int64).sum())
        assert int(hist[c].sum()) == H * W
        assert int(s[c]) == int((np.arange(256) * hist[c].astype(np.int64)).sum())
    h2, s2 = orc.hist_sum(orc.mirror(img))
    assert (h2 == hist).all() and (s2 == s).all()


def test_hist_after_solarise_upper_bins_empty(orc):
    hist, _ = orc.hist_sum(orc.solarise(_rand(8, 40, 40)))
    assert (hist[:, 128:] == 0).all()


# ---------------------------------------------------------------- pipelines
def test_pipeline_order_is_stage_order(orc):
    img = _rand(1, 16, 12)
    st = [("noise", {"seed": 0x1510}), ("solarise", {}), ("blur5", {}), ("mirror", {})]
    out, hist, s = orc.run_image_pipeline(img, st, "hist_sum")
    manual = orc.mirror(orc.blur5(orc.solarise(orc.noise(img, 0x1510))))
    assert (out == manual).all()
    h2, s2 = orc.hist_sum(manual)
    assert (hist == h2).all() and (s == s2).all()
    # reordering noise and mirror changes the result: noise is position dependent
    swapped = orc.run_image_pipeline(img, [("mirror", {}), ("noise", {"seed": 0x1510})])
    assert (swapped != orc.run_image_pipeline(img, [("noise", {"seed": 0x1510}), ("mirror", {})])).any()


def test_image_rows_generator_matches_full_draw():
    a = synth.image(7, 37, 53)
    assert (synth.image_rows(7, 37, 53, 5, 20) == a[5:20]).all()


# ------------------------------------------------------------- while Loop
def test_while_loop_counts_on_constant_image(orc):
    """A 5x5 box blur leaves a constant image unchanged, so the channel sums stay
    W*H*v: a condition that holds runs the body to the limit, one that fails
    stops after the first iteration (the body runs at least once)."""
    img = np.full((6, 9, 4), 40, np.uint8)
    body = [("blur5", {})]
    total = 6 * 9 * 40
    out, h, s, n = orc.run_image_while(img, body, "hist_sum", 2, ">", total - 1, 7)
    assert n == 7 and (out == img).all() and int(s[2]) == total and int(h[2, 40]) == 54
    out, h, s, n = orc.run_image_while(img, body, "hist_sum", 2, "<", total, 7)
    assert n == 1
    _, _, _, n = orc.run_image_while(img, body, "sum", 0, ">=", total, 1)
    assert n == 1


def test_while_loop_matches_library_iteration(orc):
    """The loop against an explicit iteration of scipy's 'nearest' correlation
    with a 5x5 box followed by one floor division (the blur's definition)."""
    from scipy.ndimage import correlate
    img = np.random.default_rng(8).integers(0, 256, (23, 31, 4), dtype=np.uint8)
    seq, cur = [], img.astype(np.int64)
    for _ in range(8):
        cur = np.stack([correlate(cur[..., c], np.ones((5, 5), np.int64), mode="nearest") // 25
                        for c in range(4)], axis=-1)
        seq.append((cur.copy(), cur.reshape(-1, 4).sum(0)))
    T = int(seq[4][1][1])
    stop = next(i for i, (_, s) in enumerate(seq) if int(s[1]) <= T) + 1
    out, h, s, n = orc.run_image_while(img, [("blur5", {})], "hist_sum", 1, ">", T, 8)
    assert n == stop
    assert (out.astype(np.int64) == seq[stop - 1][0]).all() and (s.astype(np.int64) == seq[stop - 1][1]).all()


def _scipy_blur_iterates(img, n):
    """The first n iterates of the 5x5 box blur written with scipy's 'nearest'
    correlation and one floor division, with each iterate's channel sums and
    per-channel histograms (numpy bincount), independent of the oracle."""
    from scipy.ndimage import correlate
    cur = img.astype(np.int64)
    out = []
    for _ in range(n):
        cur = np.stack([correlate(cur[..., c], np.ones((5, 5), np.int64), mode="nearest") // 25
                        for c in range(4)], axis=-1)
        h = np.stack([np.bincount(cur[..., c].ravel(), minlength=256) for c in range(4)])
        out.append((cur.copy(), cur.reshape(-1, 4).sum(0), h))
    return out


def test_while_delta_condition_and_carried_merge_on_constant_image(orc):
    """On a constant image the blur changes nothing: the first iteration has no
    predecessor and continues, the second sees a change of 0 and stops under
    'continue while |change| > 0'.  Carried outputs are the sum of the two
    iterations' results (merge by addition); uncarried ones the last."""
    H, W, v = 6, 9, 40
    img = np.full((H, W, 4), v, np.uint8)
    body = [("blur5", {})]
    out, h, s, n = orc.run_image_while(img, body, "hist_sum", 0, ">", 0, 10, kind="delta")
    assert n == 2 and (out == img).all()
    assert int(s[0]) == H * W * v and int(h[1, v]) == H * W
    out, h, s, n = orc.run_image_while(img, body, "hist_sum", 0, ">", 0, 10, kind="delta",
                                       carried=("hist", "sum"))
    assert n == 2 and all(int(s[c]) == 2 * H * W * v for c in range(4))
    assert int(h[3, v]) == 2 * H * W and int(h.sum()) == 2 * 4 * H * W
    # only the sums carried: the histogram is the last iteration's
    _, h, s, n = orc.run_image_while(img, body, "hist_sum", 0, ">", 0, 10, kind="delta", carried=("sum",))
    assert int(s[2]) == 2 * H * W * v and int(h[2, v]) == H * W
    # a limit of 1 stops after the first iteration whatever the condition
    _, _, s, n = orc.run_image_while(img, body, "sum", 0, ">", 0, 1, kind="delta", carried=("sum",))
    assert n == 1 and int(s[0]) == H * W * v


def test_while_delta_and_carried_match_explicit_iteration(orc):
    """Random image, blur body: the loop stops at the first iteration i >= 2
    whose channel-1 sum changed by at most T since iteration i - 1; carried
    sums and histograms equal the totals over the explicit iterates."""
    img = np.random.default_rng(18).integers(0, 256, (21, 33, 4), dtype=np.uint8)
    seq = _scipy_blur_iterates(img, 12)
    sums = [int(t[1][1]) for t in seq]
    deltas = [abs(sums[i] - sums[i - 1]) for i in range(1, 12)]
    T = sorted(deltas)[len(deltas) // 2]               # stops somewhere inside the 12 iterations
    stop = next(i for i in range(1, 12) if abs(sums[i] - sums[i - 1]) <= T) + 1
    assert 2 <= stop <= 12
    out, h, s, n = orc.run_image_while(img, [("blur5", {})], "hist_sum", 1, ">", T, 12, kind="delta",
                                       carried=("hist", "sum"))
    assert n == stop
    assert (out.astype(np.int64) == seq[stop - 1][0]).all()
    assert (s.astype(np.int64) == sum(t[1] for t in seq[:stop])).all()
    assert (h.astype(np.int64) == sum(t[2] for t in seq[:stop])).all()
    # uncarried: the last iterate's results
    _, h, s, n = orc.run_image_while(img, [("blur5", {})], "hist_sum", 1, ">", T, 12, kind="delta")
    assert n == stop and (s.astype(np.int64) == seq[stop - 1][1]).all() and (h == seq[stop - 1][2]).all()
    # the value condition is unaffected by carrying (it reads the iteration's own sums)
    Tv = sums[3]
    _, _, s, n = orc.run_image_while(img, [("blur5", {})], "sum", 1, ">", Tv, 12, carried=("sum",))
    nv = next(i for i, x in enumerate(sums) if not x > Tv) + 1
    assert n == nv and (s.astype(np.int64) == sum(t[1] for t in seq[:nv])).all()


def test_while_carried_outputs_start_from_the_callers_values(orc):
    """Carried outputs start from the loop state the caller passes in; the
    uint32 histogram counters wrap modulo 2^32 as the device's do."""
    img = np.full((4, 5, 4), 9, np.uint8)
    init_h = np.zeros((4, 256), np.uint32)
    init_h[0, 9] = 2 ** 32 - 7
    init_h[2, 200] = 5
    init_s = np.array([1, 2, 3, 2 ** 63], np.uint64)
    _, h, s, n = orc.run_image_while(img, [("blur5", {})], "hist_sum", 0, ">=", 0, 3,
                                     carried=("hist", "sum"), init_hist=init_h, init_sum=init_s)
    assert n == 3
    assert int(h[0, 9]) == (2 ** 32 - 7 + 3 * 20) % 2 ** 32 and int(h[2, 200]) == 5 and int(h[1, 9]) == 60
    assert [int(x) for x in s] == [1 + 540, 2 + 540, 3 + 540, 2 ** 63 + 540]
