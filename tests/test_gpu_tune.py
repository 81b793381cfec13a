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
    lines = open(db).readlines()
    # one provenance line for the session, then one row per configuration
    assert lines[0].startswith("# skel tuning session: tuner=exhaustive") and "device=gfx950" in lines[0]
    rows = [l.strip().split(",") for l in lines if not l.startswith("#")]
    assert sk.config_count(root, args) == len(rows) == len(lines) - 1
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


def test_tune_pruned_walks_ordered_dimensions(tmp_path):
    """Algorithm 1 search: every timed configuration is a candidate of the
    exhaustive set, the fully fused partition is timed first, the search times
    no more than the exhaustive one, and its choice is the fastest it timed
    and still matches the oracle."""
    st = [("noise", {"seed": 9}), ("solarise", {}), ("blur5", {}), ("mirror", {})]
    img = synth.image(4, 700, 900)
    args = image_args(img, "hist_sum")
    root = sk.image_chain(st, "hist_sum")
    db = str(tmp_path / "pruned.csv")
    best, us, timed = sk.tune_pruned(root, args, db, reps=3)
    assert open(db).readline().startswith("# skel tuning session: tuner=pruned")
    rows = [l.strip().split(",") for l in open(db) if not l.startswith("#")]
    assert timed == len(rows) and 1 <= timed <= sk.config_count(root, args)
    full = str(tmp_path / "full.csv")
    sk.tune(root, args, full, reps=1)
    cands = {tuple(r[1:7]) for r in (l.strip().split(",") for l in open(full) if not l.startswith("#"))}
    assert all(tuple(r[1:7]) in cands for r in rows)
    assert float(rows[0][7 + 10]) == 1.0                  # feature 10 (kernels) of the first timed config
    assert min(float(r[-2]) for r in rows) == pytest.approx(us, rel=1e-6)
    p = sk.Plan(root, args, best)
    p.run(args)
    out, h, s = image_results(args, "hist_sum")
    ref, rh, rs = oracle.run_image_pipeline(img, st, "hist_sum")
    assert_image_equal(out, ref, "pruned")
    assert (h == rh).all() and (s == rs).all()
    # fp32 chain and N-body go through the same walk
    n = 1 << 16
    x = torch.from_numpy(synth.vector(1, n)).cuda()
    w = torch.from_numpy(synth.vector(2, n)).cuda()
    vroot = sk.image_chain([("saxpy", {"a": 2.0}), ("mirror", {})], "sum")
    vbest, vus, vt = sk.tune_pruned(vroot, [x, w, torch.empty_like(x), torch.empty(1, device="cuda")], None, reps=2)
    assert vbest["wg"] in (64, 256, 1024) and vus > 0 and vt >= 1
    pos, vel = synth.nbody(1, 512)
    nargs = [torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda(), torch.empty(512, 4, device="cuda")]
    nbest, nus, nt = sk.tune_pruned(sk.nbody_loop(2), nargs, None, reps=2)
    assert 1 <= nbest["tile_h"] <= 16 and nt >= 1
