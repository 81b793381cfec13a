"""Benchmark of the skeleton hot path on one MI355X.

Headline workload: the fused Pipeline + MapReduce over an 8192 x 8192 RGBA
uint8 image (noise -> solarise -> 5x5 blur -> mirror, then a per-channel
256-bin histogram and uint64 channel sums), one plan run per step, inputs
resident in HBM.  Prints ONE JSON line with throughput (Gelem/s = Gpixel/s),
the roofline of the dominant kernel measured live with HIP events, the CPU
oracle's throughput on the host, the fused-vs-plain speedup and, under
"extras", the other skeletons (plain filter pipeline, N-body Loop, batched
requests, while Loop, FFT pipeline, Segmentation).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
                  [--no-cpu-baseline] [--selector] [--profile-run] [--filter-pipeline-only]
                  [--while-only] [--mlp-profile-run]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                                   # MI355X HBM3E, GB/s
VALU_LANE_OPS = 256 * 64 * 2.4e9                        # 256 CUs x 64 lanes x 2.4 GHz
NBODY_LANE_OPS_PER_PAIR = 13                            # 13 VALU issues per pair, v_rsq_f32 included
NBODY_FLOPS_PER_PAIR = 20                               # conventional flop count of one pair interaction
FP32_PEAK_TFLOPS = 157.3                                # MI355X FP32 vector (packed FP32)
FP32_NONPACKED_TFLOPS = 78.6                            # the same without packed FP32 instructions
METRIC = "Gelem/s & % HBM roofline per skeleton; fused/learned vs plain speedup"
PIPE_NSBM = [("noise", {"seed": 0x1510}), ("solarise", {}), ("blur5", {}), ("mirror", {})]
PIPE_NSM = [("noise", {"seed": 0x1510}), ("solarise", {}), ("mirror", {})]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Untimed load before every timed region, whatever --warmup says: the GPU
# needs about 0.1 s of load to reach its working clocks (timed steps right
# after 5 warm-up steps of the 8192^2 chain, ~1 ms of work, ran 10-15% slow).
WARM_SECONDS = 0.3


def warm_up(fn, warmup, min_seconds=WARM_SECONDS):
    """fn() `warmup` times, then more calls (in groups of 4, synchronised)
    until at least min_seconds of wall time have passed.  Returns the number
    of calls made."""
    import torch
    t0 = time.perf_counter()
    n = 0
    for _ in range(warmup):
        fn()
        n += 1
    torch.cuda.synchronize()
    while time.perf_counter() - t0 < min_seconds:
        for _ in range(4):
            fn()
            n += 1
        torch.cuda.synchronize()
    return n


def timed_runs(fn, steps, warmup):
    """Warms up (see warm_up), then runs fn() `steps` times bracketed by device
    synchronisation; returns (wall seconds, event milliseconds)."""
    import torch
    warm_up(fn, warmup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, e0.elapsed_time(e1)


def _loaded_hip_runtime():
    """The HIP runtime library already mapped into this process (the one the
    skeleton library and torch use), opened by its exact path."""
    import ctypes
    for line in open("/proc/self/maps"):
        if "libamdhip64.so" in line:
            return ctypes.CDLL(line.split()[-1])
    raise RuntimeError("HIP runtime not loaded")


class HipEvents:
    """hipEvent_t pairs from the HIP runtime (the plan records them itself, so
    they bypass torch's event bookkeeping)."""

    def __init__(self, n):
        import ctypes
        self.hip = _loaded_hip_runtime()
        self.ct = ctypes
        self.ev = []
        for _ in range(2 * n):
            e = ctypes.c_void_p()
            assert self.hip.hipEventCreate(ctypes.byref(e)) == 0
            self.ev.append(e.value)

    def pair(self, i):
        return self.ev[2 * i], self.ev[2 * i + 1]

    def ms(self, i):
        f = self.ct.c_float()
        a, b = self.pair(i)
        assert self.hip.hipEventSynchronize(self.ct.c_void_p(b)) == 0
        assert self.hip.hipEventElapsedTime(self.ct.byref(f), self.ct.c_void_p(a), self.ct.c_void_p(b)) == 0
        return f.value

    def close(self):
        for e in self.ev:
            self.hip.hipEventDestroy(self.ct.c_void_p(e))


def kernel_times(plan, bound, kernel, steps):
    """Durations (ms) of one kernel of a plan over `steps` runs, from HIP
    events the plan records around that kernel on the launch stream (after the
    same warm-up floor as timed_runs)."""
    import torch
    warm_up(lambda: plan.run(bound), 0)
    ev = HipEvents(steps)
    for i in range(steps):
        plan.kernel_events(kernel, *ev.pair(i))
        plan.run(bound)
    torch.cuda.synchronize()
    plan.kernel_events(-1)
    ts = [ev.ms(i) for i in range(steps)]
    ev.close()
    return ts


def kernel_ms(plan, bound, kernel, steps):
    """Average duration of one kernel of a plan (see kernel_times)."""
    ts = kernel_times(plan, bound, kernel, steps)
    return sum(ts) / len(ts)


def traffic_for(kernel: str, algo_bytes: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this
    kernel, or None when there is none or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_1510_06585_amd", "csrc", rec["source"])
    if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(img, budget_s=12.0):
    """The oracle as it stands on the host's cores: the full chain over the
    full 8192 x 8192 image, every stage materialised, repeated for ~budget_s;
    then one run of the same chain on one thread."""
    import oracle
    oracle.lib()
    cores = oracle.max_threads()
    reps, t = 0, 0.0
    while reps < 2 or t < budget_s:
        t0 = time.perf_counter()
        oracle.run_image_pipeline(img, PIPE_NSBM, "hist_sum")
        t += time.perf_counter() - t0
        reps += 1
    px = img.shape[0] * img.shape[1]
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.run_image_pipeline(img, PIPE_NSBM, "hist_sum")
    t1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    return {"value": round(px * reps / t / 1e9, 6), "unit": "Gelem/s", "cores": cores, "kind": "oracle",
            "sample": f"full 8192x8192 image x {reps} runs (noise, solarise, blur5, mirror each materialised, "
                      f"then histogram + sums); OpenMP over rows in noise/blur, other stages single-threaded",
            "seconds": round(t, 3),
            "single_thread": {"value": round(px / t1 / 1e9, 6), "unit": "Gelem/s", "sample": "the same chain, "
                              "one run on one thread", "seconds": round(t1, 3)},
            "host": {"cpu": _cpu_model(), "nproc": os.cpu_count()}}


def image_args(img, reduce="hist_sum"):
    import torch
    x = torch.from_numpy(img).cuda()
    a = [x, torch.empty_like(x)]
    if reduce == "hist_sum":
        a += [torch.zeros(4, 256, dtype=torch.int32, device="cuda"), torch.zeros(4, dtype=torch.int64, device="cuda")]
    return a


def bench_fused_mapreduce_8192(steps, warmup, do_cpu):
    import torch
    import paper_1510_06585_amd as sk
    import synth
    H = W = 8192
    img = synth.image(synth.SEED_PIPE_FUSED, H, W)
    args = image_args(img)
    bound = sk.bind(args)
    root = sk.image_chain(PIPE_NSBM, "hist_sum")
    fused = sk.Plan(root, args)
    plain = sk.Plan(root, args, {"fusion": sk.FUSE_OFF})
    warm_calls = warm_up(lambda: fused.run(bound), warmup)
    wall, ev_ms = timed_runs(lambda: fused.run(bound), steps, 0)
    ms_step = wall * 1e3 / steps
    k_ts = sorted(kernel_times(fused, bound, 0, steps))
    k_ms = sum(k_ts) / len(k_ts)
    _, plain_ms = timed_runs(lambda: plain.run(bound), max(5, steps // 4), 3)
    plain_ms /= max(5, steps // 4)
    # Context: a device-to-device copy of the same image through torch.
    src, dst = args[0], args[1]
    _, copy_ms = timed_runs(lambda: dst.copy_(src), 50, 5)
    copy_gbs = 2.0 * H * W * 4 / (copy_ms / 50 * 1e-3) / 1e9
    desc = fused.describe()
    algo = 2.0 * H * W * 4 + 4 * 256 * 4 + 4 * 8      # read + write image, hist + sums
    achieved = algo / (k_ms * 1e-3) / 1e9
    kname = desc["kernels"][0]["name"]
    traffic = traffic_for(kname, algo)
    out = {
        "metric": METRIC,
        "value": round(H * W * steps / wall / 1e9, 4),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "fused Pipeline+MapReduce, 8192x8192 RGBA u8: noise>solarise>blur5x5>mirror, "
                               "256-bin per-channel histogram + u64 channel sums",
                   "H": H, "W": W, "kernels": len(desc["kernels"]), "tile_h": desc["kernels"][0].get("tile_h"),
                   "wg": desc["kernels"][0].get("wg")},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel_ms": round(k_ms, 5), "kernel_ms_min": round(k_ts[0], 5),
                     "kernel_ms_median": round(k_ts[len(k_ts) // 2], 5), "algorithmic_bytes": int(algo)},
        "copy_reference_gbs": round(copy_gbs, 1),
        "warmup_policy": {"steps": warmup, "min_seconds": WARM_SECONDS, "untimed_calls": warm_calls},
        "event_ms_per_step": round(ev_ms / steps, 5),
        "plain_ms_per_step": round(plain_ms, 5),
        "fused_vs_plain_speedup": round(plain_ms / (ev_ms / steps), 3),
    }
    fused.destroy()
    plain.destroy()
    del args, bound
    torch.cuda.empty_cache()
    return out, img


def bench_filter_pipeline_1024():
    import paper_1510_06585_amd as sk
    import synth
    img = synth.image(synth.SEED_PIPE_PLAIN, 1024, 1024)
    args = image_args(img, None)
    b = sk.bind(args)
    root = sk.image_chain(PIPE_NSM)
    res = {}
    for name, opt in (("plain", {"fusion": sk.FUSE_OFF}), ("fused", {})):
        p = sk.Plan(root, args, opt)
        _, ms = timed_runs(lambda: p.run(b), 200, 20)
        res[f"{name}_ms"] = round(ms / 200, 5)
        res[f"{name}_gelem_s"] = round(1024 * 1024 / (ms / 200 * 1e-3) / 1e9, 3)
        p.destroy()
    res["fused_vs_plain_speedup"] = round(res["plain_ms"] / res["fused_ms"], 3)
    return res


def bench_nbody():
    import torch
    import paper_1510_06585_amd as sk
    import synth
    N, iters = 65536, 20
    pos, vel = synth.nbody(synth.SEED_NBODY, N)
    args = [torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda(), torch.empty(N, 4, device="cuda")]
    b = sk.bind(args)
    res = {}
    for name, opt in (("graph_fused", {}), ("eager_unfused", {"fusion": sk.FUSE_OFF, "variant": 1})):
        p = sk.Plan(sk.nbody_loop(iters), args, opt)
        _, ms = timed_runs(lambda: p.run(b), 3, 1)
        ms /= 3
        pairs = float(N) * N * iters
        res[f"{name}_ms_per_loop"] = round(ms, 4)
        res[f"{name}_ginteractions_s"] = round(pairs / (ms * 1e-3) / 1e9, 2)
        p.destroy()
    rate = float(N) * N * iters / (res["graph_fused_ms_per_loop"] * 1e-3)
    tflops = rate * NBODY_FLOPS_PER_PAIR / 1e12
    res["roofline"] = {"bound": "alu", "achieved": round(tflops, 2), "peak": FP32_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(tflops / FP32_PEAK_TFLOPS, 4),
                       "frac_of_non_packed_fp32_peak": round(tflops / FP32_NONPACKED_TFLOPS, 4),
                       "note": f"{NBODY_FLOPS_PER_PAIR} flops per pair interaction by convention; peak = MI355X "
                               f"published FP32 vector rate (packed FP32), {FP32_NONPACKED_TFLOPS} without "
                               f"packed FP32 instructions, which this library does not emit"}
    issue_peak = VALU_LANE_OPS / NBODY_LANE_OPS_PER_PAIR
    res["issue_efficiency"] = {"achieved_ginteractions_s": round(rate / 1e9, 2),
                               "issue_bound_ginteractions_s": round(issue_peak / 1e9, 2),
                               "frac": round(rate / issue_peak, 4),
                               "note": "the kernel's own instruction count: 13 VALU issues per pair "
                                       "(v_rsq_f32 included) on 256 CUs x 64 lanes x 2.4 GHz"}
    return res


def bench_batch():
    import torch
    import paper_1510_06585_amd as sk
    import synth
    sides = synth.batch_sides(synth.SEED_BATCH, 256)
    reqs = []
    for r, s in enumerate(sides):
        reqs.append(image_args(synth.image(4000 + r, s, s)))
    px = sum(s * s for s in sides)
    algo = sum(2.0 * s * s * 4 + 4128 for s in sides)
    root = sk.image_chain(PIPE_NSBM, "hist_sum")
    proto = [sk.proto([8, 8, 4], sk.U8)] * 2 + [sk.proto([4, 256], sk.U32), sk.proto([4], sk.U64)]
    res = {"requests": 256, "pixels": px}
    bound = sk.bind_batch(reqs)      # marshal the 1024 buffers once, as a serving loop would
    # tile height and work-group size of the persistent launch chosen by the
    # batch autotuner (exhaustive over its 30 points; untimed here)
    t0 = time.perf_counter()
    best, tuned_us, ntimed = sk.tune_batch(root, bound, None, reps=10)
    res["autotune"] = {"tile_h": best["tile_h"], "wg": best["wg"], "points_timed": ntimed,
                       "median_us": round(tuned_us, 2), "seconds": round(time.perf_counter() - t0, 2)}
    bp_default = sk.Plan(root, proto)
    _, ms = timed_runs(lambda: bp_default.batch_run(bound), 30, 5)
    res["default_plan_ms"] = round(ms / 30, 4)
    bp_default.destroy()
    bp = sk.Plan(root, proto, {"tile_h": best["tile_h"], "wg": best["wg"]})
    _, ms = timed_runs(lambda: bp.batch_run(bound), 30, 5)
    ms /= 30
    res["batched_ms"] = round(ms, 4)
    res["batched_gelem_s"] = round(px / (ms * 1e-3) / 1e9, 3)
    res["batched_hbm_frac"] = round(algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    for name, opt in (("sequential_fused", {}), ("sequential_plain", {"fusion": sk.FUSE_OFF})):
        plans = [(sk.Plan(root, a, opt), sk.bind(a)) for a in reqs]

        def run_all():
            for p, b in plans:
                p.run(b)
        _, ms2 = timed_runs(run_all, 3, 1)
        ms2 /= 3
        res[f"{name}_ms"] = round(ms2, 4)
        res[f"batched_vs_{name}_speedup"] = round(ms2 / ms, 3)
        for p, _ in plans:
            p.destroy()
    bp.destroy()
    del reqs
    torch.cuda.empty_cache()
    return res


def bench_while():
    """While Loop with the device-evaluated condition vs the paper's host-side
    evaluation (run the body, read its sums back, test on the host) on the
    noise>solarise>blur>mirror MapReduce body over 8192^2, 10 iterations."""
    import numpy as np
    import torch
    import paper_1510_06585_amd as sk
    import synth
    H = W = 8192
    iters = 10
    img = synth.image(synth.SEED_PIPE_FUSED, H, W)
    x = torch.from_numpy(img).cuda()
    y = torch.empty_like(x)
    hist = torch.zeros(4, 256, dtype=torch.int32, device="cuda")
    sums = torch.zeros(4, dtype=torch.int64, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    body = sk.image_chain(PIPE_NSBM, "hist_sum")
    res = {"iterations": iters}
    wplan = sk.Plan(sk.LoopWhile(body, iters, 0, ">=", 0), [x, y, hist, sums, count])
    wb = sk.bind([x, y, hist, sums, count])
    _, ms = timed_runs(lambda: wplan.run(wb), 10, 3)
    res["device_condition_ms_per_iteration"] = round(ms / 10 / iters, 5)
    assert int(count.cpu().numpy().view(np.uint32)[0]) == iters
    wplan.destroy()
    # asynchronous runs (no host read-back), the convergence form of the
    # condition and both reduce outputs carried (merged by addition)
    aplan = sk.Plan(sk.LoopWhile(body, iters, 0, ">=", 0, -1, carried_mask=0b1100, kind="delta"),
                    [x, y, hist, sums, count])
    _, ms = timed_runs(lambda: aplan.run(wb), 10, 3)
    res["async_delta_carried_ms_per_iteration"] = round(ms / 10 / iters, 5)
    assert int(count.cpu().numpy().view(np.uint32)[0]) == iters
    aplan.destroy()
    bplan = sk.Plan(body, [x, y, hist, sums])
    a, b2 = sk.bind([x, y, hist, sums]), sk.bind([y, x, hist, sums])

    def host_loop():
        for i in range(iters):
            bplan.run(a if i % 2 == 0 else b2)
            s = sums.cpu().numpy().view(np.uint64)       # the host reads the state and tests it
            if not int(s[0]) >= 0:
                break
    _, ms = timed_runs(host_loop, 5, 1)
    res["host_condition_ms_per_iteration"] = round(ms / 5 / iters, 5)

    def counted():
        for i in range(iters):
            bplan.run(a if i % 2 == 0 else b2)
    _, ms = timed_runs(counted, 5, 1)
    res["no_condition_ms_per_iteration"] = round(ms / 5 / iters, 5)
    bplan.destroy()
    return res


def bench_fft():
    """FFT pipelined with its inversion (the paper's FFT benchmark) over 512
    transforms of 65536 complex fp32 points (256 MiB): fused (3 passes) vs one
    kernel per half-stage (4 passes)."""
    import torch
    import paper_1510_06585_amd as sk
    import synth
    B = 512
    x = torch.from_numpy(synth.complex_batch(synth.SEED_FFT, B)).cuda()
    y = torch.empty_like(x)
    root = sk.image_chain([("fft", {}), ("ifft", {})])
    elems = B * 65536
    algo = 2.0 * elems * 8                      # read the input once, write the output once
    res = {"transforms": B, "points": 65536}
    for name, opt in (("fused", {}), ("plain", {"fusion": sk.FUSE_OFF})):
        p = sk.Plan(root, [x, y], opt)
        b = sk.bind([x, y])
        _, ms = timed_runs(lambda: p.run(b), 20, 5)
        ms /= 20
        passes = len(p.describe()["kernels"])
        res[f"{name}_ms"] = round(ms, 4)
        res[f"{name}_passes"] = passes
        res[f"{name}_gelem_s"] = round(elems / (ms * 1e-3) / 1e9, 2)
        res[f"{name}_pass_traffic_gbs"] = round(passes * algo / (ms * 1e-3) / 1e9, 1)
        p.destroy()
    res["fused_vs_plain_speedup"] = round(res["plain_ms"] / res["fused_ms"], 3)
    # the chain's own algorithmic bytes: the input read once and the output
    # written once (every extra pass is the method's cost, not the workload's)
    res["chain_algorithmic_bytes"] = int(algo)
    res["fused_chain_hbm_gbs"] = round(algo / (res["fused_ms"] * 1e-3) / 1e9, 1)
    res["fused_chain_hbm_frac"] = round(res["fused_chain_hbm_gbs"] / HBM_PEAK_GBS, 4)
    res["fused_pass_traffic_frac"] = round(res["fused_pass_traffic_gbs"] / HBM_PEAK_GBS, 4)
    return res


def bench_saxpy():
    """Saxpy (Sec. 4) at the paper's largest size, 5 x 10^7 fp32 elements: one
    stage (read v and w, write out: 12 bytes per element), and a MapReduce of
    two stages with an fp32 sum, fused (one pass, 16 bytes per element) vs
    one kernel per stage."""
    import torch
    import paper_1510_06585_amd as sk
    import synth
    n = 50_000_000
    rng = __import__("numpy").random.default_rng(synth.SEED_SELECT)
    a1, a2 = synth.saxpy_coeff(rng), synth.saxpy_coeff(rng)
    x = torch.from_numpy(synth.vector(11, n)).cuda()
    w1 = torch.from_numpy(synth.vector(12, n)).cuda()
    w2 = torch.from_numpy(synth.vector(13, n)).cuda()
    out = torch.empty_like(x)
    s = torch.zeros(1, device="cuda")
    res = {"elements": n}
    one = sk.Plan(sk.Map("saxpy", a=a1), [x, w1, out])
    b1 = sk.bind([x, w1, out])
    _, ms = timed_runs(lambda: one.run(b1), 200, 50)
    ms /= 200
    res["one_stage_ms"] = round(ms, 4)
    res["one_stage_hbm_gbs"] = round(12.0 * n / (ms * 1e-3) / 1e9, 1)
    res["one_stage_hbm_frac"] = round(res["one_stage_hbm_gbs"] / HBM_PEAK_GBS, 4)
    one.destroy()
    root = sk.image_chain([("saxpy", {"a": a1}), ("saxpy", {"a": a2})], "sum")
    args = [x, w1, w2, out, s]
    for name, opt in (("chain2_sum_fused", {}), ("chain2_sum_plain", {"fusion": sk.FUSE_OFF})):
        p = sk.Plan(root, args, opt)
        b = sk.bind(args)
        _, ms = timed_runs(lambda: p.run(b), 200, 50)
        ms /= 200
        res[f"{name}_ms"] = round(ms, 4)
        res[f"{name}_kernels"] = len(p.describe()["kernels"])
        p.destroy()
    res["chain2_sum_fused_hbm_gbs"] = round(16.0 * n / (res["chain2_sum_fused_ms"] * 1e-3) / 1e9, 1)
    res["chain2_sum_fused_hbm_frac"] = round(res["chain2_sum_fused_hbm_gbs"] / HBM_PEAK_GBS, 4)
    res["chain2_sum_fused_vs_plain_speedup"] = round(res["chain2_sum_plain_ms"] / res["chain2_sum_fused_ms"], 3)
    return res


def bench_segment():
    """Segmentation (Map over a gray volume, Sec. 4) at the paper's largest
    size, 60 MiB (240 x 512 x 512 voxels): one stage, and a chain of three
    stages fused into one pass vs one kernel per stage."""
    import torch
    import paper_1510_06585_amd as sk
    import synth
    vol = torch.from_numpy(synth.gray_volume(synth.SEED_SEGMENT, 240, 512, 512)).cuda()
    out = torch.empty_like(vol)
    n = vol.numel()
    res = {"voxels": n}
    for name, stages, opt in (("one_stage", [(0, 0)], {}), ("chain3_fused", [(0, 0), (100, 200), (50, 150)], {}),
                              ("chain3_plain", [(0, 0), (100, 200), (50, 150)], {"fusion": sk.FUSE_OFF})):
        p = sk.Plan(sk.image_chain([("segment", {"lo": lo, "hi": hi}) for lo, hi in stages]), [vol, out], opt)
        b = sk.bind([vol, out])
        _, ms = timed_runs(lambda: p.run(b), 200, 50)
        ms /= 200
        passes = len(p.describe()["kernels"])
        res[f"{name}_ms"] = round(ms, 4)
        res[f"{name}_gvox_s"] = round(n / (ms * 1e-3) / 1e9, 1)
        res[f"{name}_hbm_gbs"] = round(passes * 2.0 * n / (ms * 1e-3) / 1e9, 1)
        p.destroy()
    res["one_stage_hbm_frac"] = round(res["one_stage_hbm_gbs"] / HBM_PEAK_GBS, 4)
    res["chain3_fused_vs_plain_speedup"] = round(res["chain3_plain_ms"] / res["chain3_fused_ms"], 3)
    return res


def bench_selector(n_train, n_test):
    """The learned-selector experiment (cost-model MLP trained on the GPU on
    autotuner-measured runtimes, scored on held-out compositions against their
    exhaustive best), with the labels' re-timing noise floor."""
    import shutil
    import tempfile
    from paper_1510_06585_amd import selector
    wd = tempfile.mkdtemp(prefix="skel_selector_")
    t0 = time.perf_counter()
    try:
        r = selector.experiment(n_train=n_train, n_test=n_test, workdir=wd, log=log)
    finally:
        shutil.rmtree(wd, ignore_errors=True)
    r.pop("workdir", None)
    r["seconds"] = round(time.perf_counter() - t0, 1)
    r["target"] = {"mean_regret_le": 0.10, "met": r["regret"]["model"]["mean"] <= 0.10,
                   "met_by_ensemble": r["regret"]["model_ensemble3"]["mean"] <= 0.10,
                   "label_noise_median_lt": 0.03,
                   "label_noise_met": bool(r["label_noise"] and r["label_noise"]["rel_diff"]["median"] < 0.03)}
    return r


def profile_run(steps):
    """Short run for hardware-counter passes: the fused 8192^2 Pipeline+MapReduce kernel and a
    plain copy of the same image (the byte-count reference), `steps` each."""
    import torch
    import paper_1510_06585_amd as sk
    import synth
    img = synth.image(synth.SEED_PIPE_FUSED, 8192, 8192)
    args = image_args(img)
    fused = sk.Plan(sk.image_chain(PIPE_NSBM, "hist_sum"), args)
    copy = sk.Plan(sk.Loop(sk.Map("mirror"), 2), args[:2])   # two mirrors = identity: one copy kernel
    for _ in range(steps):
        fused.run(args)
    for _ in range(steps):
        copy.run(args[:2])
    torch.cuda.synchronize()
    print(json.dumps({"fused": fused.describe()["kernels"][0]["name"], "copy": copy.describe()["kernels"][0]["name"],
                      "copy_bytes_per_launch": 2 * 8192 * 8192 * 4}), flush=True)


def counters_run(steps):
    """Short run for the counter passes over the other workloads' kernels:
    a plain copy of an 8192^2 image (the byte-count reference), the
    256-request batch at its default plan, the FFT -> IFFT chain over 512
    transforms (passes A, B+A, B), one saxpy stage over 5 x 10^7 elements, one
    Segmentation stage over 240 x 512 x 512 voxels (`steps` runs each) and
    one 20-step N-body loop over 65536 bodies."""
    import torch
    import paper_1510_06585_amd as sk
    import synth
    img = synth.image(synth.SEED_PIPE_FUSED, 8192, 8192)
    args = image_args(img)
    copy = sk.Plan(sk.Loop(sk.Map("mirror"), 2), args[:2])   # two mirrors = identity: one copy kernel
    for _ in range(steps):
        copy.run(args[:2])
    torch.cuda.synchronize()
    copy.destroy()
    del args
    sides = synth.batch_sides(synth.SEED_BATCH, 256)
    reqs = [image_args(synth.image(4000 + r, s, s)) for r, s in enumerate(sides)]
    proto = [sk.proto([8, 8, 4], sk.U8)] * 2 + [sk.proto([4, 256], sk.U32), sk.proto([4], sk.U64)]
    bp = sk.Plan(sk.image_chain(PIPE_NSBM, "hist_sum"), proto)
    bound = sk.bind_batch(reqs)
    for _ in range(steps):
        bp.batch_run(bound)
    torch.cuda.synchronize()
    bp.destroy()
    del reqs, bound
    x = torch.from_numpy(synth.complex_batch(synth.SEED_FFT, 512)).cuda()
    y = torch.empty_like(x)
    fp = sk.Plan(sk.image_chain([("fft", {}), ("ifft", {})]), [x, y])
    for _ in range(steps):
        fp.run([x, y])
    torch.cuda.synchronize()
    fp.destroy()
    del x, y
    n = 50_000_000
    v = torch.from_numpy(synth.vector(11, n)).cuda()
    w = torch.from_numpy(synth.vector(12, n)).cuda()
    o = torch.empty_like(v)
    sp = sk.Plan(sk.Map("saxpy", a=1.5), [v, w, o])
    for _ in range(steps):
        sp.run([v, w, o])
    torch.cuda.synchronize()
    sp.destroy()
    del v, w, o
    vol = torch.from_numpy(synth.gray_volume(synth.SEED_SEGMENT, 240, 512, 512)).cuda()
    vout = torch.empty_like(vol)
    gp = sk.Plan(sk.image_chain([("segment", {"lo": 0, "hi": 0})]), [vol, vout])
    for _ in range(steps):
        gp.run([vol, vout])
    torch.cuda.synchronize()
    gp.destroy()
    del vol, vout
    N = 65536
    pos, vel = synth.nbody(synth.SEED_NBODY, N)
    nargs = [torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda(), torch.empty(N, 4, device="cuda")]
    npl = sk.Plan(sk.nbody_loop(20), nargs)
    npl.run(nargs)
    torch.cuda.synchronize()
    npl.destroy()
    torch.cuda.empty_cache()
    print(json.dumps({"counters_run": {"steps": steps, "batch_requests": 256, "fft_transforms": 512,
                                       "saxpy_elements": n, "segment_voxels": 240 * 512 * 512,
                                       "nbody_bodies": N, "nbody_steps": 20}}), flush=True)


def mlp_profile_run(n=16384, reps=3):
    """Workload of the MFMA counter pass: the cost-model MLP's forward and
    gradient kernels `reps` times each on n seeded random samples."""
    import torch
    import paper_1510_06585_amd as sk
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    P = sk.mlp_param_count()
    params = (torch.rand(P, device="cuda", generator=g) - 0.5) * 0.2
    X = torch.rand(n, 24, device="cuda", generator=g)
    t = torch.rand(n, device="cuda", generator=g)
    y = torch.empty(n, device="cuda")
    grad = torch.empty(P, device="cuda")
    loss = torch.empty(1, device="cuda")
    for _ in range(reps):
        sk.mlp_forward(params, X, y)
        sk.mlp_grad(params, X, t, grad, loss)
    torch.cuda.synchronize()
    print(json.dumps({"mlp_profile_run": {"samples": n, "reps": reps}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=500,
                    help="untimed steps first; the GPU needs ~0.1 s of load to reach its working clocks")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--selector", action="store_true", help="run the learned-selector experiment instead")
    ap.add_argument("--profile-run", action="store_true", help="short run for rocprofv3 counter passes")
    ap.add_argument("--filter-pipeline-only", action="store_true",
                    help="only the 1024x1024 filter pipeline, plain and fused (for a per-stage kernel trace)")
    ap.add_argument("--counters-run", action="store_true",
                    help="short run of the other workloads' kernels for rocprofv3 counter passes")
    ap.add_argument("--mlp-profile-run", action="store_true",
                    help="only the cost-model MLP forward and gradient kernels on 16384 samples (MFMA counters)")
    ap.add_argument("--while-only", action="store_true",
                    help="only the 8192x8192 x 10 while Loop against its host-checked and unchecked forms "
                         "(for a kernel trace)")
    ap.add_argument("--no-selector", action="store_true", help="leave the learned-selector experiment out of the extras")
    ap.add_argument("--selector-dir", default=None, help="where the selector experiment keeps its databases")
    ap.add_argument("--selector-train", type=int, default=1000)
    ap.add_argument("--selector-sampled-only", action="store_true",
                    help="train on sampled labels only (without each training composition's Algorithm-1 walk)")
    ap.add_argument("--selector-test", type=int, default=200)
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}); runs over several GPUs are "
              f"not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1510_06585_amd as sk
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    sk.lib()
    if a.profile_run:
        profile_run(a.steps)
        return
    if a.mlp_profile_run:
        mlp_profile_run()
        return
    if a.counters_run:
        counters_run(a.steps)
        return
    if a.filter_pipeline_only:
        print(json.dumps(bench_filter_pipeline_1024()), flush=True)
        return
    if a.while_only:
        print(json.dumps(bench_while()), flush=True)
        return
    if a.selector:
        from paper_1510_06585_amd import selector
        print(json.dumps(selector.experiment(n_train=a.selector_train, n_test=a.selector_test,
                                             workdir=a.selector_dir, log=log,
                                             train_pruned=not a.selector_sampled_only)), flush=True)
        return
    log("config 2: fused pipeline + mapreduce 8192x8192")
    out, img = bench_fused_mapreduce_8192(a.steps, a.warmup, not a.no_cpu_baseline)
    if not a.no_extras:
        extras = {}
        log("config 1: filter pipeline 1024x1024 plain vs fused")
        extras["filter_pipeline_1024"] = bench_filter_pipeline_1024()
        log("config 3: n-body 65536 x 20 iterations")
        extras["nbody_65536_x20"] = bench_nbody()
        log("config 4: 256 batched uneven requests")
        extras["batched_256"] = bench_batch()
        log("while Loop: device-evaluated condition, 8192x8192 x 10")
        extras["while_loop_8192x10"] = bench_while()
        log("FFT pipelined with its inverse: 512 x 65536 complex fp32")
        extras["fft_pipeline_512x65536"] = bench_fft()
        log("saxpy: 5e7 fp32 elements, one stage and a two-stage MapReduce with an fp32 sum")
        extras["saxpy_5e7"] = bench_saxpy()
        log("Segmentation: 60 MiB gray volume, one stage and a 3-stage chain")
        extras["segment_60MiB"] = bench_segment()
        if not a.no_selector:
            log("learned selector: 1000 training / 200 held-out compositions")
            extras["selector"] = bench_selector(a.selector_train, a.selector_test)
        out["extras"] = extras
    if not a.no_cpu_baseline:
        log("cpu baseline: oracle on the host")
        out["cpu_baseline"] = cpu_baseline(img)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
