"""Helpers of the GPU parity tests: move seeded numpy inputs to the device, run a
plan through the C-ABI binding, bring results back as numpy arrays."""
import numpy as np
import torch

import paper_1510_06585_amd as sk


def cuda(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def image_args(img: np.ndarray, reduce=None, inplace=False):
    x = cuda(img)
    out = x if inplace else torch.empty_like(x)
    args = [x, out]
    if reduce == "hist_sum":
        args += [torch.full((4, 256), 7, dtype=torch.int32, device="cuda"),
                 torch.full((4,), 7, dtype=torch.int64, device="cuda")]
    elif reduce == "sum":
        args += [torch.full((4,), 7, dtype=torch.int64, device="cuda")]
    return args


def image_results(args, reduce=None):
    torch.cuda.synchronize()
    out = args[1].cpu().numpy()
    if reduce == "hist_sum":
        return out, args[2].cpu().numpy().view(np.uint32), args[3].cpu().numpy().view(np.uint64)
    if reduce == "sum":
        return out, None, args[2].cpu().numpy().view(np.uint64)
    return out, None, None


def run_image(stages, img, reduce=None, options=None, inplace=False):
    root = sk.image_chain(stages, reduce)
    args = image_args(img, reduce, inplace)
    plan = sk.Plan(root, args, options)
    plan.run(args)
    res = image_results(args, reduce)
    plan.destroy()
    return res


def assert_image_equal(got, ref, what=""):
    if got.shape != ref.shape:
        raise AssertionError(f"{what}: shape {got.shape} != {ref.shape}")
    bad = np.argwhere(got != ref)
    if bad.size:
        y, x, c = bad[0]
        raise AssertionError(f"{what}: {len(bad)} bytes differ; first at y={y} x={x} c={c}: "
                             f"got {got[y, x, c]} want {ref[y, x, c]}")
