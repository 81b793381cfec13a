"""GPU parity of Segmentation chains (Sec. 4 Segmentation) against the oracle:
bit-exact on every voxel, at the paper's three volume sizes (1 MB, 8 MB,
60 MB), ragged volumes whose byte count is not a multiple of the 16-byte
vector, fused and unfused chains, custom and degenerate thresholds, and in
place."""
import numpy as np
import pytest
import torch

import oracle
import paper_1510_06585_amd as sk
import synth

pytestmark = pytest.mark.gpu


def _run(vol, stages, options=None, inplace=False):
    inp = torch.from_numpy(vol).cuda()
    out = inp if inplace else torch.empty_like(inp)
    p = sk.Plan(sk.image_chain([("segment", {"lo": lo, "hi": hi}) for lo, hi in stages]), [inp, out], options)
    p.run([inp, out])
    torch.cuda.synchronize()
    d = p.describe()
    p.destroy()
    return out.cpu().numpy(), d


def _check(vol, stages, options=None, inplace=False):
    got, d = _run(vol, stages, options, inplace)
    ref = oracle.run_segment_chain(vol, stages)
    bad = np.flatnonzero(got.reshape(-1) != ref.reshape(-1))
    assert bad.size == 0, (stages, options, vol.shape, bad[:8])
    return d


@pytest.mark.parametrize("shape", [(64, 128, 128), (128, 256, 256), (240, 512, 512)], ids=["1MB", "8MB", "60MB"])
def test_paper_volume_sizes(shape):
    vol = synth.gray_volume(synth.SEED_SEGMENT, *shape)
    d = _check(vol, [(0, 0)])
    assert len(d["kernels"]) == 1


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 15), (1, 1, 17), (17, 19, 23), (3, 1000, 1001), (5, 7)])
def test_ragged_volumes(shape):
    vol = np.random.default_rng(sum(shape)).integers(0, 256, shape, dtype=np.uint8)
    _check(vol, [(0, 0)])
    _check(vol, [(31, 77), (0, 0)])


def test_all_256_values_and_degenerate_thresholds():
    vol = np.tile(np.arange(256, dtype=np.uint8), 16 * 17).reshape(17, 16, 256)
    for lo, hi in [(85, 170), (0, 256), (100, 100), (256, 256), (1, 255), (0, 1), (255, 256), (129, 200)]:
        _check(vol, [(lo, hi)])


def test_threshold_grid_on_every_byte_value():
    """Every byte value under each pair of thresholds drawn from the edges
    (0, 1, 2, 127, 128, 129, 254, 255, 256) and under 200 random pairs, one
    stage at a time and chained three at a time (the chain's fold)."""
    vol = np.tile(np.arange(256, dtype=np.uint8), 4).reshape(4, 256)
    edges = [0, 1, 2, 127, 128, 129, 254, 255, 256]
    pairs = [(a, b) for a in edges for b in edges if a <= b]
    rng = np.random.default_rng(77)
    for _ in range(200):
        a, b = sorted(int(t) for t in rng.integers(0, 257, 2))
        pairs.append((a, b))
    for lo, hi in pairs:
        _check(vol, [(lo, hi)])
    for i in range(0, len(pairs) - 2, 3):
        _check(vol, pairs[i:i + 3])


@pytest.mark.parametrize("fusion", ["on", "off", "mask"])
def test_chains_fused_and_unfused(fusion):
    vol = synth.gray_volume(synth.SEED_SEGMENT + 1, 33, 100, 101)
    stages = [(0, 0), (129, 200), (10, 20), (0, 256), (5, 250)]
    opts = {"on": None, "off": {"fusion": sk.FUSE_OFF}, "mask": {"fusion": sk.FUSE_MASK, "split_mask": 0b0101}}[fusion]
    d = _check(vol, stages, opts)
    assert len(d["kernels"]) == {"on": 1, "off": 5, "mask": 3}[fusion]


def test_in_place_and_ept_variants():
    vol = synth.gray_volume(synth.SEED_SEGMENT + 2, 40, 256, 259)
    _check(vol, [(0, 0)], inplace=True)
    for ept in (1, 2, 4, 16):
        for wg in (64, 256, 1024):
            _check(vol, [(60, 180), (0, 0)], {"ept": ept, "wg": wg})


def test_rejections():
    t = torch.zeros(4, 8, 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(sk.SkelError):
        sk.Map("segment", lo=10, hi=5)
    with pytest.raises(sk.SkelError):
        sk.Map("segment", lo=0, hi=257)
    with pytest.raises(sk.SkelError) as e:   # partial overlap
        flat = torch.zeros(4 * 8 * 8 + 16, dtype=torch.uint8, device="cuda")
        a, b = flat[:256].view(4, 8, 8), flat[16:272].view(4, 8, 8)
        sk.Plan(sk.image_chain([("segment", {})]), [a, b]).run([a, b])
    assert e.value.status == sk.EINVAL
    with pytest.raises(sk.SkelError) as e:   # mixed with image stages
        sk.Plan(sk.image_chain([("segment", {}), ("solarise", {})]), [t, t.clone()])
    assert e.value.status == sk.ETYPE
    f = torch.zeros(4, 8, 8, device="cuda")
    with pytest.raises(sk.SkelError):
        sk.Plan(sk.image_chain([("segment", {})]), [f, f.clone()])


def test_tuners_cover_gray_chains(tmp_path):
    vol = synth.gray_volume(synth.SEED_SEGMENT + 3, 16, 128, 130)
    inp = torch.from_numpy(vol).cuda()
    out = torch.empty_like(inp)
    root = sk.image_chain([("segment", {}), ("segment", {"lo": 100, "hi": 200}), ("segment", {"lo": 5, "hi": 9})])
    best, us = sk.tune(root, [inp, out], str(tmp_path / "db.csv"), reps=2)[:2]
    assert us > 0
    lines = (tmp_path / "db.csv").read_text().strip().splitlines()
    assert len(lines) >= 2 * 4              # every split mask of 3 stages at two ept values
    pbest, pus, timed = sk.tune_pruned(root, [inp, out], None, reps=2)
    assert pus > 0 and 1 <= timed <= 8
    p = sk.Plan(root, [inp, out], pbest)
    p.run([inp, out])
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.run_segment_chain(vol, [(0, 0), (100, 200), (5, 9)]))
    p.destroy()


def test_empty_volume_runs_nothing():
    for shape in [(0,), (0, 5, 7), (3, 0, 2)]:
        vol = torch.zeros(shape, dtype=torch.uint8, device="cuda")
        out = torch.zeros(shape, dtype=torch.uint8, device="cuda")
        p = sk.Plan(sk.image_chain([("segment", {}), ("segment", {"lo": 3, "hi": 9})]), [vol, out])
        p.run([vol, out])
        torch.cuda.synchronize()
        assert p.describe()["kernels"][0]["grid"] == 0
        p.destroy()


def test_volume_near_the_2gib_limit():
    """2047 x 1023 x 1023 voxels (2.14 GB, just under the 2^31-voxel limit,
    and not a multiple of 16: the ragged tail at the top of the 32-bit range),
    a two-stage chain checked on every voxel."""
    shape = (2047, 1023, 1023)
    n = shape[0] * shape[1] * shape[2]
    assert n < (1 << 31) and n % 16
    vol = synth.gray_volume(synth.SEED_SEGMENT + 9, *shape)
    _check(vol, [(0, 0), (100, 200)])
