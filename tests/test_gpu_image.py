"""GPU parity of the image skeletons against the CPU oracle: bit-exact images,
histograms and sums, for fused, unfused and interpreted kernels, at the full
benchmark sizes, at the paper's odd image sizes and at ragged tiny sizes."""
import numpy as np
import pytest
import torch

import oracle
import paper_1510_06585_amd as sk
import synth
from gpu_helpers import assert_image_equal, run_image

pytestmark = pytest.mark.gpu

PIPE_NSM = [("noise", {"seed": synth.NOISE_SEED}), ("solarise", {}), ("mirror", {})]
PIPE_NSBM = [("noise", {"seed": synth.NOISE_SEED}), ("solarise", {}), ("blur5", {}), ("mirror", {})]


@pytest.mark.parametrize("options", [{"fusion": sk.FUSE_OFF}, {}, {"variant": 1}],
                         ids=["plain", "fused", "interpreter"])
def test_filter_pipeline_1024(options):
    img = synth.image(synth.SEED_PIPE_PLAIN, 1024, 1024)
    ref = oracle.run_image_pipeline(img, PIPE_NSM)
    out, _, _ = run_image(PIPE_NSM, img, None, options)
    assert_image_equal(out, ref, "filter pipeline 1024")


@pytest.mark.parametrize("options", [{}, {"fusion": sk.FUSE_OFF}], ids=["fused", "plain"])
def test_pipeline_mapreduce_8192(options):
    img = synth.image(synth.SEED_PIPE_FUSED, 8192, 8192)
    ref, rh, rs = oracle.run_image_pipeline(img, PIPE_NSBM, "hist_sum")
    out, h, s = run_image(PIPE_NSBM, img, "hist_sum", options)
    assert_image_equal(out, ref, "pipeline+mapreduce 8192")
    assert (h == rh).all() and (s == rs).all()
    assert int(h.sum()) == 4 * 8192 * 8192 and (h[:, 128:] == 0).all()


def test_pipeline_mapreduce_near_the_2gib_limit():
    """22000 x 22000 RGBA (1.94 GB per image, just under the 2^31-byte image
    limit): byte offsets near the top of the 32-bit buffer range, fused chain
    against the full oracle."""
    H = W = 22000
    assert H * W * 4 < (1 << 31)
    img = synth.image(synth.SEED_PIPE_FUSED + 7, H, W)
    out, h, s = run_image(PIPE_NSBM, img, "hist_sum", {})
    ref, rh, rs = oracle.run_image_pipeline(img, PIPE_NSBM, "hist_sum")
    assert_image_equal(out, ref, "pipeline+mapreduce 22000^2")
    assert (h == rh).all() and (s == rs).all()
    del out, ref, img


# Image sizes the paper's Table 5 lists (W x H), plus ragged and tiny shapes.
SIZES = [(4288, 2848), (1800, 1125), (1440, 900), (256, 512), (512, 512), (2048, 2048),
         (1, 1), (3, 5), (5, 3), (257, 9), (300, 7), (251, 40), (252, 33), (253, 31), (508, 17), (4, 1000), (1023, 1)]


@pytest.mark.parametrize("W,H", SIZES, ids=[f"{w}x{h}" for w, h in SIZES])
def test_pipeline_mapreduce_odd_sizes(W, H):
    img = synth.image(W * 7 + H, H, W)
    ref, rh, rs = oracle.run_image_pipeline(img, PIPE_NSBM, "hist_sum")
    for opt in ({}, {"fusion": sk.FUSE_OFF}, {"variant": 1}, {"wg": 64, "tile_h": 7},
                {"wg": 128, "tile_h": 1}):
        out, h, s = run_image(PIPE_NSBM, img, "hist_sum", opt)
        assert_image_equal(out, ref, f"{W}x{H} {opt}")
        assert (h == rh).all() and (s == rs).all(), opt


@pytest.mark.parametrize("W,H", [(1, 1), (2, 2), (3, 7), (260, 3), (1000, 37)])
def test_every_stage_alone_and_mirror_positions(W, H):
    img = synth.image(W + 100 * H, H, W)
    for st in (["noise"], ["solarise"], ["mirror"], ["blur5"], ["mirror", "noise"], ["noise", "mirror", "blur5"],
               ["mirror", "blur5", "noise", "mirror"], ["blur5", "mirror", "noise", "solarise", "mirror"],
               ["mirror", "noise", "blur5", "mirror", "noise"]):
        stages = [(n, {"seed": 77 + i} if n == "noise" else {}) for i, n in enumerate(st)]
        ref = oracle.run_image_pipeline(img, stages)
        for opt in ({}, {"fusion": sk.FUSE_OFF}, {"variant": 1}):
            out, _, _ = run_image(stages, img, None, opt)
            assert_image_equal(out, ref, f"{st} {opt} {W}x{H}")


def test_random_compositions_and_fusion_partitions():
    rng = np.random.default_rng(synth.SEED_SELECT)
    done = 0
    while done < 30:
        comp = synth.composition(rng, log2_lo=6, log2_hi=15)
        if comp["domain"] != "u8":
            continue
        img = synth.image(comp["seed"], comp["H"], comp["W"])
        ref = oracle.run_image_pipeline(img, comp["stages"], comp["reduce"])
        k = len(comp["stages"])
        nbits = k - 1 + (1 if comp["reduce"] else 0)
        masks = sorted(set([0, (1 << nbits) - 1, int(rng.integers(0, 1 << nbits)) if nbits else 0]))
        for m in masks:
            nblur = 0
            ok = True
            for i, (n, _) in enumerate(comp["stages"]):
                nblur += n == "blur5"
                if nblur > 1:
                    ok = False
                if i < k - 1 and (m >> i) & 1:
                    nblur = 0
            opt = {"fusion": sk.FUSE_MASK, "split_mask": m} if ok else {"fusion": sk.FUSE_ON}
            out, h, s = run_image(comp["stages"], img, comp["reduce"], opt)
            if comp["reduce"]:
                ref_img, rh, rs = ref
                assert_image_equal(out, ref_img, f"{comp} {opt}")
                assert (s == rs).all()
                if comp["reduce"] == "hist_sum":
                    assert (h == rh).all()
            else:
                assert_image_equal(out, ref, f"{comp} {opt}")
        done += 1


def test_loop_of_image_stages_runs_depth_first():
    img = synth.image(9, 40, 70)
    stages = [("noise", {"seed": 1}), ("blur5", {}), ("blur5", {}), ("blur5", {}), ("mirror", {})]
    ref = oracle.run_image_pipeline(img, stages)
    root = sk.Pipeline(sk.Map("noise", seed=1), sk.Loop(sk.Map("blur5"), 3), sk.Map("mirror"))
    from gpu_helpers import image_args, image_results
    for opt in ({}, {"fusion": sk.FUSE_OFF}):
        args = image_args(img)
        p = sk.Plan(root, args, opt)
        p.run(args)
        out, _, _ = image_results(args)
        assert_image_equal(out, ref, str(opt))


def test_inplace_pointwise_and_rejections():
    img = synth.image(10, 33, 65)
    st = [("noise", {"seed": 3}), ("solarise", {})]
    out, _, _ = run_image(st, img, None, {}, inplace=True)
    assert_image_equal(out, oracle.run_image_pipeline(img, st), "inplace")
    with pytest.raises(sk.SkelError) as e:
        run_image(PIPE_NSM, img, None, {}, inplace=True)
    assert e.value.status == sk.EINVAL
    # unfused: the mirror kernel reads a scratch image, so in-place is legal
    out, _, _ = run_image(PIPE_NSM, img, None, {"fusion": sk.FUSE_OFF}, inplace=True)
    assert_image_equal(out, oracle.run_image_pipeline(img, PIPE_NSM), "inplace unfused")


def test_empty_images_and_reduce_outputs_overwritten():
    for H, W in ((0, 5), (5, 0)):
        img = np.zeros((H, W, 4), np.uint8)
        out, h, s = run_image(PIPE_NSBM, img, "hist_sum")
        assert (h == 0).all() and (s == 0).all()
    img = synth.image(11, 50, 50)
    from gpu_helpers import image_args, image_results
    args = image_args(img, "hist_sum")
    p = sk.Plan(sk.image_chain(PIPE_NSBM, "hist_sum"), args)
    p.run(args)
    p.run(args)        # a second run overwrites, it does not accumulate
    out, h, s = image_results(args, "hist_sum")
    ref, rh, rs = oracle.run_image_pipeline(img, PIPE_NSBM, "hist_sum")
    assert (h == rh).all() and (s == rs).all()


@pytest.mark.parametrize("options", [{"wg": 64, "tile_h": 8}, {}, {"fusion": sk.FUSE_OFF, "tile_h": 4}],
                         ids=["many-rows", "auto", "plain"])
def test_reduce_rerun_overwrites_with_many_merge_chunks(options):
    """Plans whose histogram rows need several merge chunks (device atomics into
    outputs cleared by the image kernel) and plans with one chunk (plain
    stores), run three times on the same output buffers with new input data."""
    from gpu_helpers import image_args, image_results
    H, W = 1500, 2048
    args = image_args(synth.image(21, H, W), "hist_sum")
    p = sk.Plan(sk.image_chain(PIPE_NSBM, "hist_sum"), args, options)
    for r in range(3):
        img = synth.image(21 + r, H, W)
        args[0].copy_(torch.from_numpy(img).cuda())
        p.run(args)
        out, h, s = image_results(args, "hist_sum")
        ref, rh, rs = oracle.run_image_pipeline(img, PIPE_NSBM, "hist_sum")
        assert_image_equal(out, ref, f"run {r}")
        assert (h == rh).all() and (s == rs).all(), f"run {r}"
    p.destroy()


def test_sum_only_reduce():
    img = synth.image(12, 77, 301)
    ref, _, rs = oracle.run_image_pipeline(img, PIPE_NSBM, "sum")
    for opt in ({}, {"fusion": sk.FUSE_OFF}):
        out, _, s = run_image(PIPE_NSBM, img, "sum", opt)
        assert_image_equal(out, ref, "sum")
        assert (s == rs).all()


def test_wrong_shapes_rejected_at_run():
    img = synth.image(13, 16, 16)
    from gpu_helpers import image_args
    args = image_args(img)
    p = sk.Plan(sk.image_chain(PIPE_NSM), args)
    bad = image_args(synth.image(13, 16, 17))
    with pytest.raises(sk.SkelError) as e:
        p.run(bad)
    assert e.value.status == sk.ESHAPE


@pytest.mark.parametrize("H,W", [(3, 65536), (65536, 3), (2, 65535)], ids=["3x65536", "65536x3", "2x65535"])
def test_image_side_at_the_65536_limit(H, W):
    """Sides at the noise key's 16-bit limit (x and y up to 65535 packed in
    one 32-bit key): the full chain with histogram and sums, fused and
    unfused, against the oracle; a side of 65537 is rejected."""
    img = synth.image(H + 3 * W, H, W)
    ref, rh, rs = oracle.run_image_pipeline(img, PIPE_NSBM, "hist_sum")
    for options in ({}, {"fusion": sk.FUSE_OFF}):
        out, h, s = run_image(PIPE_NSBM, img, "hist_sum", options)
        assert_image_equal(out, ref, f"{H}x{W} {options}")
        assert (h == rh).all() and (s == rs).all()
    big = [sk.proto([H, 65537, 4] if W >= H else [65537, W, 4], sk.U8)] * 2
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.image_chain(PIPE_NSBM), big)
    assert e.value.status == sk.EUNSUPPORTED
