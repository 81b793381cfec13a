"""GPU auto-tuner: every measured configuration lands in the database, the
returned configuration is one of them and the fastest, and a plan compiled with
it still matches the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_1510_06585_amd as sk
import synth
from gpu_helpers import assert_image_equal, image_args, image_results

pytestmark = pytest.mark.gpu


def test_tune_image_chain(tmp_path):
    st = [("noise", {"seed": 9}), ("blur5", {}), ("mirror", {})]
    img = synth.image(3, 300, 500)
    args = image_args(img, "hist_sum")
    root = sk.image_chain(st, "hist_sum")
    db = str(tmp_path / "db.csv")
    best, us = sk.tune(root, args, db, reps=3)
    assert sk.config_count(root, args) == len(open(db).readlines())
    rows = [l.strip().split(",") for l in open(db)]
    assert len(rows) >= 8 and us > 0
    times = [float(r[-2]) for r in rows]
    assert min(times) == pytest.approx(us, rel=1e-6)
    p = sk.Plan(root, args, best)
    p.run(args)
    out, h, s = image_results(args, "hist_sum")
    ref, rh, rs = oracle.run_image_pipeline(img, st, "hist_sum")
    assert_image_equal(out, ref, "tuned")
    assert (h == rh).all() and (s == rs).all()


def test_tune_vector_and_nbody(tmp_path):
    n = 1 << 16
    x = torch.from_numpy(synth.vector(1, n)).cuda()
    w = torch.from_numpy(synth.vector(2, n)).cuda()
    out = torch.empty_like(x)
    s = torch.empty(1, device="cuda")
    root = sk.image_chain([("saxpy", {"a": 2.0}), ("mirror", {})], "sum")
    best, us = sk.tune(root, [x, w, out, s], str(tmp_path / "v.csv"), reps=3)
    assert best["wg"] in (64, 256, 1024) and us > 0
    pos, vel = synth.nbody(1, 512)
    args = [torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda(), torch.empty(512, 4, device="cuda")]
    best, us = sk.tune(sk.nbody_loop(2), args, None, reps=2)
    assert 1 <= best["tile_h"] <= 16
