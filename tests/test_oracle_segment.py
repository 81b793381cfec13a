"""Pins of the oracle's Segmentation stage (Sec. 4: gray voxels to black, gray
or white).  The thresholds are a reading (the paper gives none): black below
lo, white from hi up, gray between.  Pinned by class counts over all 256
values, the boundary voxels on either side of each threshold, the degenerate
threshold pairs, idempotence of the default stage and monotonicity."""
import numpy as np
import pytest

import oracle

ALL = np.arange(256, dtype=np.uint8)


@pytest.mark.parametrize("lo,hi", [(85, 170), (0, 0), (1, 255), (100, 100), (0, 256), (37, 201), (256, 256)])
def test_class_counts_over_all_values(lo, hi):
    if (lo, hi) == (0, 0):
        out, (lo, hi) = oracle.run_segment_chain(ALL, [(0, 0)]), (85, 170)   # (0, 0) means the defaults
    else:
        out = oracle.segment(ALL, lo, hi)
    # exactly lo values are black, hi - lo gray, 256 - hi white
    assert (out == 0).sum() == lo
    assert (out == 128).sum() == hi - lo
    assert (out == 255).sum() == 256 - hi
    assert set(np.unique(out)) <= {0, 128, 255}


def test_boundary_voxels():
    v = np.array([0, 84, 85, 169, 170, 255], np.uint8)
    assert oracle.segment(v).tolist() == [0, 0, 128, 128, 255, 255]
    v = np.array([9, 10, 11, 199, 200, 201], np.uint8)
    assert oracle.segment(v, 10, 200).tolist() == [0, 128, 128, 128, 255, 255]


def test_monotone_and_default_stage_idempotent():
    for lo, hi in [(85, 170), (3, 250), (128, 129)]:
        out = oracle.segment(ALL, lo, hi).astype(int)
        assert np.all(np.diff(out) >= 0)
    once = oracle.segment(ALL)
    assert np.array_equal(oracle.segment(once), once)       # 0, 128, 255 are fixed points of the default stage
    # a chain composes stage by stage: 128 is black for lo = 129
    assert np.array_equal(oracle.run_segment_chain(ALL, [(0, 0), (129, 200)]),
                          np.where(ALL < 170, 0, 255).astype(np.uint8))


def test_shape_kept_and_rejections():
    vol = np.random.default_rng(0).integers(0, 256, (3, 5, 7), dtype=np.uint8)
    assert oracle.segment(vol).shape == (3, 5, 7)
    with pytest.raises(ValueError):
        oracle.segment(vol, 10, 5)
    with pytest.raises(ValueError):
        oracle.segment(vol.astype(np.int16))
