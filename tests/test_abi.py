"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, builds and linearises skeleton trees, groups stages into kernels and
rejects malformed requests -- all without a GPU (plan compilation is
host-only; device resources are allocated by a plan's first run)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1510_06585_amd as sk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ensure_built():
    if not os.path.exists(sk.skel.LIB_PATH):
        from paper_1510_06585_amd import build
        build.build()


_ensure_built()


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "skel.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(skel_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 20
    L = ctypes.CDLL(sk.skel.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(sk.skel.EXPORTS)


def img(H, W):
    return [sk.proto([H, W, 4], sk.U8), sk.proto([H, W, 4], sk.U8)]


def hist_args(H, W):
    return img(H, W) + [sk.proto([4, 256], sk.U32), sk.proto([4], sk.U64)]


PIPE_NSBM = [("noise", {"seed": 0x1510}), ("solarise", {}), ("blur5", {}), ("mirror", {})]


def test_fused_nsbm_chain_is_one_kernel_with_mirror_on_the_store():
    p = sk.Plan(sk.image_chain(PIPE_NSBM, "hist_sum"), hist_args(64, 100))
    d = p.describe()
    assert d["stages"] == ["noise", "solarise", "blur5", "mirror"]
    assert len(d["kernels"]) == 1
    k = d["kernels"][0]
    assert k["blur"] and k["reduce"] and k["name"] == "img_noise_sol_blur_reduce"


def test_unfused_is_one_kernel_per_stage_in_depth_first_order():
    # Sec. 2: pipeline(K1, loop(K2), K3) runs K1, then K2 n times, then K3.
    root = sk.MapReduce(sk.Pipeline(sk.Map("noise", seed=1), sk.Loop(sk.Map("blur5"), 3), sk.Map("mirror")),
                        sk.RED_HIST256_SUM)
    p = sk.Plan(root, hist_args(16, 16), {"fusion": sk.FUSE_OFF})
    d = p.describe()
    assert d["stages"] == ["noise", "blur5", "blur5", "blur5", "mirror"]
    assert [k["stages"] for k in d["kernels"]] == [[0, 1], [1, 2], [2, 3], [3, 4], [4, 5], [5, 5]]
    assert d["kernels"][-1]["reduce"] and not d["kernels"][-2]["reduce"]
    assert d["sct"] == "mapreduce(pipeline(noise,loop[3](blur5),mirror),hist256_sum)"


def test_fusion_splits_at_second_stencil():
    root = sk.image_chain([("noise", {"seed": 1}), ("blur5", {}), ("solarise", {}), ("blur5", {}), ("mirror", {})])
    d = sk.Plan(root, img(32, 300)).describe()
    assert [k["stages"] for k in d["kernels"]] == [[0, 3], [3, 5]]


def test_split_mask_partitions_and_rejects_two_stencils():
    root = sk.image_chain(PIPE_NSBM, "hist_sum")
    d = sk.Plan(root, hist_args(8, 8), {"fusion": sk.FUSE_MASK, "split_mask": 0b0010}).describe()
    assert [k["stages"] for k in d["kernels"]] == [[0, 2], [2, 4]]
    d = sk.Plan(root, hist_args(8, 8), {"fusion": sk.FUSE_MASK, "split_mask": 0b1000}).describe()
    assert [k["stages"] for k in d["kernels"]] == [[0, 4], [4, 4]] and d["kernels"][1]["reduce"]
    two = sk.image_chain([("blur5", {}), ("blur5", {})])
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(two, img(8, 8), {"fusion": sk.FUSE_MASK, "split_mask": 0})
    assert e.value.status == sk.EINVAL


def test_generic_variant_selected_on_request():
    root = sk.image_chain(PIPE_NSBM, "hist_sum")
    d = sk.Plan(root, hist_args(8, 8), {"variant": 1}).describe()
    assert d["kernels"][0]["name"] == "img_generic_blur_reduce"


def test_type_and_shape_errors():
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.Pipeline(sk.Map("noise"), sk.Map("saxpy", a=1.0)), img(4, 4))
    assert e.value.status == sk.ETYPE
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.image_chain(PIPE_NSBM, "hist_sum"), img(4, 4))          # missing reduce outputs
    assert e.value.status == sk.EINVAL
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.image_chain(PIPE_NSBM), [sk.proto([4, 4, 4], sk.U8), sk.proto([4, 5, 4], sk.U8)])
    assert e.value.status == sk.ESHAPE
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.image_chain(PIPE_NSBM), img(2, 65537))
    assert e.value.status == sk.EUNSUPPORTED
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.MapReduce(sk.Map("saxpy", a=1.0), sk.RED_HIST256_SUM),
                [sk.proto([8], sk.F32)] * 3 + [sk.proto([1], sk.F32)])
    assert e.value.status == sk.ETYPE
    with pytest.raises(sk.SkelError) as e:      # MapReduce below the root
        sk.Pipeline(sk.MapReduce(sk.Map("noise"), sk.RED_SUM), sk.Map("mirror"))
        sk.Loop(sk.MapReduce(sk.Map("noise"), sk.RED_SUM), 2)
    assert e.value.status == sk.EINVAL
    with pytest.raises(sk.SkelError) as e:
        sk.Map(99)
    assert e.value.status == sk.EINVAL
    with pytest.raises(sk.SkelError):
        sk.Plan(sk.image_chain(PIPE_NSBM), img(8, 8), {"wg": 96})


def test_nbody_structure_checks():
    p = sk.Plan(sk.nbody_loop(20), [sk.proto([128, 4], sk.F32)] * 3)
    d = p.describe()
    assert d["iterations"] == 20 and d["kernels"][0]["name"] == "nbody_force_kick_drift"
    assert d["loop_sync"] == 1 and d["loop_carried"] == 0b011
    d = sk.Plan(sk.nbody_loop(3), [sk.proto([128, 4], sk.F32)] * 3, {"fusion": sk.FUSE_OFF}).describe()
    assert [k["name"] for k in d["kernels"]] == ["nbody_force", "nbody_kick_drift"]
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.Pipeline(sk.Map("leapfrog", dt=1e-3), sk.Map("nbody_force", eps=0.01, G=1.0)),
                [sk.proto([8, 4], sk.F32)] * 3)
    assert e.value.status == sk.ETYPE


def test_vector_chain_grouping():
    st = [("saxpy", {"a": 1.5}), ("mirror", {}), ("saxpy", {"a": -2.0})]
    root = sk.image_chain(st, "sum")
    args = [sk.proto([1000], sk.F32)] * 4 + [sk.proto([1], sk.F32)]
    d = sk.Plan(root, args).describe()
    assert d["domain"] == "f32" and len(d["kernels"]) == 1
    d = sk.Plan(root, args, {"fusion": sk.FUSE_OFF}).describe()
    assert len(d["kernels"]) == 4 and d["kernels"][-1]["reduce"]


def test_mirror_only_chain_takes_domain_from_arguments():
    d = sk.Plan(sk.Map("mirror"), [sk.proto([9], sk.F32)] * 2).describe()
    assert d["domain"] == "f32"
    d = sk.Plan(sk.Map("mirror"), img(3, 3)).describe()
    assert d["domain"] == "u8"


def test_features_reflect_configuration():
    root = sk.image_chain(PIPE_NSBM, "hist_sum")
    f_on = sk.features(root, hist_args(1024, 1024))
    f_off = sk.features(root, hist_args(1024, 1024), {"fusion": sk.FUSE_OFF})
    assert f_on.shape == (24,)
    assert list(f_on[:6]) == [1, 1, 1, 1, 0, 1]
    assert f_on[6] == 4 and f_on[7] == 20 and f_on[8] == 1
    assert f_on[10] == 1 and f_off[10] == 5                 # kernels
    assert f_off[11:15].tolist() == [1, 1, 1, 0]            # stage boundaries after stages 0..2
    assert f_on[21] == 1 and f_off[21] == 0                 # reduce fused
    assert f_off[22] > f_on[22]                             # more algorithmic bytes unfused


def test_kernel_constants_exact():
    # constants the image kernels use in place of divisions
    assert all(b - 33 * ((b * 249) >> 13) == b % 33 for b in range(256))
    assert all((s * 5243) >> 17 == s // 25 for s in range(25 * 255 + 1))
    assert all((s * 671089) >> 24 == s // 25 for s in range(25 * 255 + 1)) and 6375 * 671089 < 2 ** 32
    assert all(b * 249 < 65536 for b in range(256))


def test_gray_chain_structure_and_limits():
    st = [("segment", {}), ("segment", {"lo": 100, "hi": 200}), ("segment", {"lo": 5, "hi": 9})]
    args = [sk.proto([7, 9, 11], sk.U8)] * 2
    d = sk.Plan(sk.image_chain(st), args).describe()
    assert d["domain"] == "gray" and [k["stages"] for k in d["kernels"]] == [[0, 3]]
    d = sk.Plan(sk.image_chain(st), args, {"fusion": sk.FUSE_OFF}).describe()
    assert [k["stages"] for k in d["kernels"]] == [[0, 1], [1, 2], [2, 3]]
    d = sk.Plan(sk.image_chain(st), args, {"fusion": sk.FUSE_MASK, "split_mask": 1}).describe()
    assert [k["stages"] for k in d["kernels"]] == [[0, 1], [1, 3]]
    # 2^31 voxels and more, including shapes whose product overflows 64 bits
    for shape in ([1 << 16, 1 << 15], [1 << 40, 1 << 40], [3, 1 << 31]):
        with pytest.raises(sk.SkelError) as e:
            sk.Plan(sk.image_chain(st), [sk.proto(shape, sk.U8)] * 2)
        assert e.value.status == sk.EUNSUPPORTED
    with pytest.raises(sk.SkelError) as e:      # mixed with image stages
        sk.Plan(sk.image_chain(st + [("noise", {"seed": 1})]), args)
    assert e.value.status == sk.ETYPE
    with pytest.raises(sk.SkelError) as e:      # gray chains have no reduce
        sk.Plan(sk.image_chain(st, "sum"), args + [sk.proto([1], sk.U64)])
    assert e.value.status == sk.ETYPE
    for lo, hi in ((10, 5), (0, 257), (300, 300)):
        with pytest.raises(sk.SkelError) as e:
            sk.Map("segment", lo=lo, hi=hi)
        assert e.value.status == sk.EINVAL


def test_fft_chain_structure_and_limits():
    st = [("fft", {}), ("ifft", {}), ("fft", {})]
    args = [sk.proto([3, 65536, 2], sk.F32)] * 2
    d = sk.Plan(sk.image_chain(st), args).describe()
    assert d["domain"] == "c32" and len(d["kernels"]) == 4        # L + 1 passes when fused
    d = sk.Plan(sk.image_chain(st), args, {"fusion": sk.FUSE_OFF}).describe()
    assert len(d["kernels"]) == 6                                  # two passes per stage
    with pytest.raises(sk.SkelError) as e:                         # 65536-point transforms only
        sk.Plan(sk.image_chain(st), [sk.proto([3, 4096, 2], sk.F32)] * 2)
    assert e.value.status in (sk.ESHAPE, sk.EUNSUPPORTED)
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.image_chain(st), [sk.proto([65536, 65536, 2], sk.F32)] * 2)
    assert e.value.status == sk.EUNSUPPORTED
    with pytest.raises(sk.SkelError) as e:
        sk.Plan(sk.image_chain(st + [("saxpy", {"a": 1.0})]), args)
    assert e.value.status == sk.ETYPE


def test_empty_buffers_with_any_strides_compile():
    # zero-element tensors get strides that are not row-major products (e.g.
    # (3, 0, 2) -> (2, 2, 1)); with no elements any strides are accepted
    b = sk.proto([3, 0, 2], sk.U8)
    b.stride_bytes[0], b.stride_bytes[1], b.stride_bytes[2] = 2, 2, 1
    d = sk.Plan(sk.image_chain([("segment", {})]), [b, b]).describe()
    assert d["kernels"][0]["grid"] == 0


def _dense(shape, dtype, addr):
    """A skel_buffer over a fake device address with explicit dense strides
    (only host-side checks run on it: every request below is rejected before
    the library touches the device)."""
    b = sk.proto(shape, dtype)
    b.data = addr
    es = {sk.U8: 1, sk.U32: 4, sk.U64: 8, sk.F32: 4, sk.F64: 8}[dtype]
    st = es
    for d in range(len(shape) - 1, -1, -1):
        b.stride_bytes[d] = st
        st *= shape[d]
    return b


def _img_req(base, H, W):
    """in, out, hist, sum of one image request laid out back to back from base."""
    n = H * W * 4
    return [_dense([H, W, 4], sk.U8, base), _dense([H, W, 4], sk.U8, base + n),
            _dense([4, 256], sk.U32, base + 2 * n), _dense([4], sk.U64, base + 2 * n + 4096)]


def test_tune_batch_checks_the_request_set_on_the_host():
    """The batch autotuner checks the request set before any device work, so a
    bad request reports its own status (here on a machine with no GPU)."""
    root = sk.image_chain(PIPE_NSBM, "hist_sum")
    H, W = 8, 8
    a = _img_req(1 << 40, H, W)
    a[1].data = a[0].data + 16                       # in and out overlap partially
    with pytest.raises(sk.SkelError) as e:
        sk.tune_batch(root, [a])
    assert e.value.status == sk.EINVAL and "overlap" in str(e.value)
    a, b = _img_req(1 << 40, H, W), _img_req(1 << 41, H, W)
    b[2].data = a[2].data                            # two requests share a histogram
    with pytest.raises(sk.SkelError) as e:
        sk.tune_batch(root, [a, b])
    assert e.value.status == sk.EINVAL
    a, b = _img_req(1 << 40, H, W), _img_req(1 << 41, H, W)
    b[2] = _dense([4, 128], sk.U32, b[2].data)       # wrong histogram shape
    with pytest.raises(sk.SkelError) as e:
        sk.tune_batch(root, [a, b])
    assert e.value.status == sk.ESHAPE


def test_tune_batch_rejects_empty_and_non_image_request_sets():
    root = sk.image_chain(PIPE_NSBM, "hist_sum")
    with pytest.raises(sk.SkelError) as e:       # no requests at all
        sk.tune_batch(root, [])
    assert e.value.status == sk.EINVAL
    n = 1000                                      # an fp32 chain is not a batched image run
    vec = [_dense([n], sk.F32, 1 << 40), _dense([n], sk.F32, (1 << 40) + 4 * n),
           _dense([n], sk.F32, (1 << 40) + 8 * n)]
    with pytest.raises(sk.SkelError) as e:
        sk.tune_batch(sk.Map("saxpy", a=1.0), [vec])
    assert e.value.status == sk.EUNSUPPORTED


def test_mixed_zero_strides_are_rejected():
    # strides may be all zero (dense shorthand) or exactly dense; a zero stride
    # next to non-zero ones would make the kernels read past the allocation
    root = sk.image_chain(PIPE_NSBM, "hist_sum")
    good = _img_req(1 << 40, 6, 5)
    p = sk.Plan(root, good)
    for bad_strides in ([0, 4, 1], [20, 0, 1], [20, 4, 0]):
        a = _img_req(1 << 40, 6, 5)
        a[0].stride_bytes[0], a[0].stride_bytes[1], a[0].stride_bytes[2] = bad_strides
        with pytest.raises(sk.SkelError) as e:
            sk.Plan(root, a)
        assert e.value.status == sk.ESHAPE, bad_strides
        with pytest.raises(sk.SkelError) as e:
            p.run(a, stream=0)
        assert e.value.status == sk.ESHAPE, bad_strides
        with pytest.raises(sk.SkelError) as e:
            p.batch_run([a], stream=0)
        assert e.value.status == sk.ESHAPE, bad_strides
    # a zero stride on an extent-1 dimension is never stepped and is accepted
    one = sk.proto([1, 5, 4], sk.U8)
    one.stride_bytes[0], one.stride_bytes[1], one.stride_bytes[2] = 0, 4, 1
    sk.Plan(sk.image_chain(PIPE_NSBM), [one, one])
    allz = sk.proto([6, 5, 4], sk.U8)
    sk.Plan(sk.image_chain(PIPE_NSBM), [allz, allz])


def test_batch_rejects_overlapping_requests():
    root = sk.image_chain(PIPE_NSBM, "hist_sum")
    p = sk.Plan(root, _img_req(1 << 40, 8, 8))
    H, W = 8, 8
    n = H * W * 4
    # in and out of one request overlap partially
    a = _img_req(1 << 40, H, W)
    a[1].data = a[0].data + 16
    with pytest.raises(sk.SkelError) as e:
        p.batch_run([a], stream=0)
    assert e.value.status == sk.EINVAL
    # a reduce output inside an image
    a = _img_req(1 << 40, H, W)
    a[2].data = a[1].data + 64
    with pytest.raises(sk.SkelError) as e:
        p.batch_run([a], stream=0)
    assert e.value.status == sk.EINVAL
    # two requests writing the same histogram / one's output over another's input
    a, b = _img_req(1 << 40, H, W), _img_req(1 << 41, H, W)
    b[2].data = a[2].data
    with pytest.raises(sk.SkelError) as e:
        p.batch_run([a, b], stream=0)
    assert e.value.status == sk.EINVAL
    a, b = _img_req(1 << 40, H, W), _img_req(1 << 41, H, W)
    b[1].data = a[0].data + n // 2
    with pytest.raises(sk.SkelError) as e:
        p.batch_run([a, b], stream=0)
    assert e.value.status == sk.EINVAL
    # a stencil chain cannot run in place
    a = _img_req(1 << 40, H, W)
    a[1].data = a[0].data
    with pytest.raises(sk.SkelError) as e:
        p.batch_run([a], stream=0)
    assert e.value.status == sk.EINVAL


def test_while_loop_option_rejections():
    """Condition kind and carried_mask are checked when the node is built."""
    body = sk.image_chain([("blur5", {})], "hist_sum")
    body_sum = sk.image_chain([("blur5", {})], "sum")
    for kw in ({"kind": 2}, {"carried_mask": 1 << 4}, {"carried_mask": 1 << 5}):
        with pytest.raises(sk.SkelError) as e:
            sk.LoopWhile(body, 3, 0, ">", 0, **kw)
        assert e.value.status == sk.EINVAL, kw
    with pytest.raises(sk.SkelError):
        sk.LoopWhile(body_sum, 3, 0, ">", 0, carried_mask=1 << 3)      # the count of a SUM body
    # accepted: images (always carried), reduce outputs, both kinds, asynchronous runs
    for kw in ({"carried_mask": 0b1111}, {"kind": "delta", "check_every": -1}):
        sk.LoopWhile(body, 3, 0, ">", 0, **kw)
    sk.LoopWhile(body_sum, 3, 0, ">", 0, carried_mask=0b111)
