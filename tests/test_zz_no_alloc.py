"""The allocation-free execution request (skel_plan_run_noalloc) against the
ordinary one (skel_plan_run) through the C-ABI: the same plan run both ways
gives the same bytes (images, volumes, histograms, sums) and fp32 results, on
two calls in a row with the second on a smaller input, so anything the first
call left in the shared static scratch must not leak into the second.  The
rejections (plans outside the entry point's scope or larger than its scratch)
are host-side checks and need no GPU."""
import numpy as np
import pytest
import torch

import paper_1510_06585_amd as sk
import synth

PIPE_NSBM = [("noise", {"seed": synth.NOISE_SEED}), ("solarise", {}), ("blur5", {}), ("mirror", {})]
PIPE_BN = [("blur5", {}), ("noise", {"seed": 77}), ("mirror", {})]


def _image_args(img, reduce):
    x = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    a = [x, torch.full_like(x, 3)]
    if reduce == "hist_sum":
        a += [torch.full((4, 256), 7, dtype=torch.int32, device="cuda"),
              torch.full((4,), 7, dtype=torch.int64, device="cuda")]
    elif reduce == "sum":
        a += [torch.full((4,), 7, dtype=torch.int64, device="cuda")]
    return a


def _host(args):
    torch.cuda.synchronize()
    return [t.cpu().numpy().copy() for t in args[1:]]


def _image_both(stages, reduce, H, W, seed, options):
    img = synth.image(seed, H, W)
    root = sk.image_chain(stages, reduce)
    a_ref = _image_args(img, reduce)
    a_new = _image_args(img, reduce)
    plan = sk.Plan(root, a_ref, options)
    plan.run(a_ref)
    ref = _host(a_ref)
    plan.run_noalloc(a_new)
    got = _host(a_new)
    plan.destroy()
    return ref, got


@pytest.mark.gpu
@pytest.mark.parametrize("options", [{}, {"fusion": sk.FUSE_OFF}, {"tile_h": 5, "wg": 128}],
                         ids=["fused", "unfused", "small-tiles"])
@pytest.mark.parametrize("reduce", ["hist_sum", "sum", None])
def test_image_chain_twice_second_smaller(options, reduce):
    for (H, W, seed) in ((1030, 1500, 11), (300, 517, 12)):
        ref, got = _image_both(PIPE_NSBM, reduce, H, W, seed, options)
        for r, g in zip(ref, got):
            assert r.shape == g.shape and (r == g).all(), (H, W, reduce, options)


@pytest.mark.gpu
def test_image_chain_at_the_benchmark_size_then_smaller():
    """The fused 8192^2 Pipeline + MapReduce (1989 work-groups of histogram
    rows in the static scratch), then a 2-kernel split plan on a small image
    whose rows land where the first call's were."""
    ref, got = _image_both(PIPE_NSBM, "hist_sum", 8192, 8192, synth.SEED_PIPE_FUSED, {})
    for r, g in zip(ref, got):
        assert (r == g).all()
    ref, got = _image_both(PIPE_BN, "hist_sum", 129, 1000, 5, {"fusion": sk.FUSE_MASK, "split_mask": 1})
    for r, g in zip(ref, got):
        assert (r == g).all()


@pytest.mark.gpu
@pytest.mark.parametrize("options", [{}, {"fusion": sk.FUSE_OFF}], ids=["fused", "unfused"])
def test_fp32_chain_with_sum_twice_second_smaller(options):
    rng = np.random.default_rng(9)
    a1, a2 = synth.saxpy_coeff(rng), synth.saxpy_coeff(rng)
    root = sk.image_chain([("saxpy", {"a": a1}), ("mirror", {}), ("saxpy", {"a": a2})], "sum")
    for n in (1_000_003, 4097):
        x = torch.from_numpy(synth.vector(21, n)).cuda()
        w1 = torch.from_numpy(synth.vector(22, n)).cuda()
        w2 = torch.from_numpy(synth.vector(23, n)).cuda()
        outs = []
        for k in range(2):
            args = [x, w1, w2, torch.full_like(x, 5.0), torch.full((1,), 9.0, device="cuda")]
            plan = sk.Plan(root, args, options)
            (plan.run if k == 0 else plan.run_noalloc)(args)
            torch.cuda.synchronize()
            outs.append((args[3].cpu().numpy(), float(args[4].cpu()[0])))
            plan.destroy()
        (v_ref, s_ref), (v_got, s_got) = outs
        assert (v_ref.view(np.uint32) == v_got.view(np.uint32)).all(), n
        # the same kernels on the same data: the sum's fixed-order merge is
        # deterministic, so the two results are the same float
        assert s_ref == s_got, (n, s_ref, s_got)


@pytest.mark.gpu
def test_gray_chain_unfused_twice_second_smaller():
    root = sk.image_chain([("segment", {"lo": 0, "hi": 0}), ("segment", {"lo": 100, "hi": 200})])
    for shape in ((40, 300, 301), (3, 17, 19)):
        vol = torch.from_numpy(synth.gray_volume(31, *shape)).cuda()
        outs = []
        for k in range(2):
            out = torch.full_like(vol, 1)
            plan = sk.Plan(root, [vol, out], {"fusion": sk.FUSE_OFF})
            (plan.run if k == 0 else plan.run_noalloc)([vol, out])
            torch.cuda.synchronize()
            outs.append(out.cpu().numpy())
            plan.destroy()
        assert (outs[0] == outs[1]).all(), shape


def _fake(shape, dtype, addr):
    """A buffer descriptor at a made-up device address: the checks under test
    run on the host and reject before any device work."""
    b = sk.proto(shape, dtype)
    b.data = addr
    return b


def test_rejects_plans_beyond_its_scope_or_size():
    lib = sk.lib()
    # unfused 4096^2 chain: two 64 MiB intermediate images > 32 MiB of scratch
    args = [_fake([4096, 4096, 4], sk.U8, 1 << 40), _fake([4096, 4096, 4], sk.U8, 2 << 40)]
    plan = sk.Plan(sk.image_chain(PIPE_NSBM), args, {"fusion": sk.FUSE_OFF})
    arr, n = sk.skel._buf_array(args)
    st = lib.skel_plan_run_noalloc(plan.handle, arr, n, None)
    assert st == sk.skel.EUNSUPPORTED
    assert b"bytes of device scratch" in lib.skel_last_error()
    plan.destroy()
    # N-body Loop: needs a captured graph
    N = 64
    nb = [_fake([N, 4], sk.F32, (k + 1) << 40) for k in range(3)]
    plan = sk.Plan(sk.nbody_loop(2), nb)
    arr, n = sk.skel._buf_array(nb)
    assert lib.skel_plan_run_noalloc(plan.handle, arr, n, None) == sk.skel.EUNSUPPORTED
    plan.destroy()
    # shape mismatch is reported as by skel_plan_run
    plan = sk.Plan(sk.image_chain(PIPE_NSBM), [sk.proto([8, 8, 4], sk.U8)] * 2)
    arr, n = sk.skel._buf_array([_fake([8, 9, 4], sk.U8, 1 << 40), _fake([8, 9, 4], sk.U8, 2 << 40)])
    assert lib.skel_plan_run_noalloc(plan.handle, arr, n, None) == sk.skel.ESHAPE
    plan.destroy()
