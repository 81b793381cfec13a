"""rocprofv3 harness: turns kernel-trace statistics and hardware-counter passes
into the short text summaries kept under ``profiles/``.

The counter passes are taken one counter group per run (rocprofv3 does not
split counters over passes), from the repository root with TMPDIR=/tmp:

  rocprofv3 --kernel-trace --stats -d DIR -o fused8192 --output-format csv -- python3 bench.py --no-extras --no-cpu-baseline
  rocprofv3 --kernel-trace --stats -d DIR -o all --output-format csv -- python3 bench.py --no-cpu-baseline --no-selector
  rocprofv3 --pmc FETCH_SIZE -d DIR -o fetch --output-format csv -- python3 bench.py --profile-run --steps 5
  rocprofv3 --pmc WRITE_SIZE -d DIR -o write --output-format csv -- python3 bench.py --profile-run --steps 5
  rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_VALU \
      SQ_ACTIVE_INST_LDS SQ_BUSY_CYCLES SQ_WAVE_CYCLES -d DIR -o sq --output-format csv -- \
      python3 bench.py --profile-run --steps 3

``bench.py --profile-run`` launches the fused 8192^2 kernel and a plain copy of
the same image; FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the fused kernel
are scaled by (known bytes / counter reading) of the copy kernel, which
corrects for the share of the memory channels the counters observe.

  python -m paper_1510_06585_amd.rocprof_harness --trace DIR/fused8192_kernel_stats.csv \
      --trace-all DIR/all_kernel_stats.csv --trace-all-dispatches DIR/all_kernel_trace.csv \
      --fetch DIR/fetch_counter_collection.csv \
      --write DIR/write_counter_collection.csv --sq DIR/sq_counter_collection.csv --out profiles/

``--trace-all`` / ``--trace-all-dispatches`` alone rewrite only the whole-run
summary (``bench_all_kernels.md``), and ``--other-fetch`` / ``--other-write`` /
``--other-sq`` the counter summary of the other workloads' kernels.

The while Loop's trace (``bench.py --while-only`` under the trace command in
COMMAND_WHILE, its stdout kept in a file) is summarised with
``--trace-while DIR/while8192_kernel_stats.csv --while-json FILE
--while-dispatches DIR/while8192_kernel_trace.csv``.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
FUSED = "img_band_kernel<9, 0, true, true, 2>"
FUSED_NAME = "img_noise_sol_blur_reduce"
COPY = "img_band_kernel<0, 0, false, false, 0>"
COPY_BYTES = 2 * 8192 * 8192 * 4
COMMANDS = (
    "rocprofv3 --kernel-trace --stats -d DIR -o fused8192 --output-format csv -- python3 bench.py --no-extras "
    "--no-cpu-baseline",
    "rocprofv3 --kernel-trace --stats -d DIR -o all --output-format csv -- python3 bench.py --no-cpu-baseline "
    "--no-selector",
    "rocprofv3 --pmc FETCH_SIZE -d DIR -o fetch --output-format csv -- python3 bench.py --profile-run --steps 5",
    "rocprofv3 --pmc WRITE_SIZE -d DIR -o write --output-format csv -- python3 bench.py --profile-run --steps 5",
    "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_VALU "
    "SQ_ACTIVE_INST_LDS SQ_BUSY_CYCLES SQ_WAVE_CYCLES -d DIR -o sq --output-format csv -- "
    "python3 bench.py --profile-run --steps 3",
    "python -m paper_1510_06585_amd.rocprof_harness --trace DIR/fused8192_kernel_stats.csv "
    "--trace-all DIR/all_kernel_stats.csv --trace-all-dispatches DIR/all_kernel_trace.csv "
    "--fetch DIR/fetch_counter_collection.csv "
    "--write DIR/write_counter_collection.csv --sq DIR/sq_counter_collection.csv --out profiles/",
)


def kernel_stats(path):
    out = []
    for r in csv.DictReader(open(path)):
        out.append({"name": r["Name"], "calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                    "min_ns": float(r["MinNs"]), "max_ns": float(r["MaxNs"]),
                    "pct": float(r["Percentage"])})
    return out


def counters(path):
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        agg[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in agg.items()}


def _find(d, key):
    for k, v in d.items():
        if key in k:
            return v
    raise KeyError(key)


def _find_opt(d, key):
    for k, v in d.items():
        if key in k:
            return v
    return None


def traffic(fetch_csv, write_csv):
    """HBM bytes per launch of the fused kernel, scaled by the copy kernel."""
    f, w = counters(fetch_csv), counters(write_csv)
    cf, cw = _find(f, COPY)["FETCH_SIZE"], _find(w, COPY)["WRITE_SIZE"]
    kf, kw = _find(f, FUSED)["FETCH_SIZE"], _find(w, FUSED)["WRITE_SIZE"]
    sf = (COPY_BYTES / 2) / (cf * 1024.0)
    sw = (COPY_BYTES / 2) / (cw * 1024.0)
    return {"fetch_kib_raw": kf, "write_kib_raw": kw, "copy_fetch_kib_raw": cf, "copy_write_kib_raw": cw,
            "fetch_scale": sf, "write_scale": sw,
            "bytes_per_launch": kf * 1024.0 * sf + kw * 1024.0 * sw}


COMMAND_FILTER_PIPELINE = ("rocprofv3 --kernel-trace --stats -d DIR -o filter1024 --output-format csv -- python3 bench.py "
                   "--filter-pipeline-only")
COMMAND_WHILE = ("rocprofv3 --kernel-trace --stats -d DIR -o while8192 --output-format csv -- python3 bench.py "
                 "--while-only")
COMMAND_MLP = ("rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VALU SQ_BUSY_CYCLES "
               "-d DIR -o mfma --output-format csv -- python3 bench.py --mlp-profile-run")
HBM_PEAK_GBS = 8000.0
NBODY_PEAK_GPAIRS = 256 * 64 * 2.4 / 13.0   # 13 VALU issues per pair


def row_work():
    """(kernel-name key, workload, kind, work per launch, last) for the kernels
    that serve one workload each in the whole bench run; kind "hbm":
    algorithmic bytes, "alu": body pairs; last: how many of the kernel's last
    dispatches are the workload's timed runs (0: all dispatches)."""
    import synth
    sides = synth.batch_sides(synth.SEED_BATCH, 256)
    batch_bytes = sum(2 * s * s * 4 + 4128 for s in sides)
    fft_bytes = 2 * 512 * 65536 * 8
    return [
        # the bench times the batch autotuner's choice last (30 runs), after
        # the tuner's own 30 candidates and the default plan
        ("img_batch_kernel<9, 0, true, true, 2>", "256 uneven requests, noise>solarise>blur>mirror + histogram "
         "(the autotuned plan's 30 timed runs)", "hbm", batch_bytes, 30),
        ("fft_pass_kernel<0>", "pass A, 512 x 65536 complex fp32", "hbm", fft_bytes, 0),
        ("fft_pass_kernel<1>", "fused pass B+A, 512 x 65536 complex fp32", "hbm", fft_bytes, 0),
        ("fft_pass_kernel<2>", "pass B, 512 x 65536 complex fp32", "hbm", fft_bytes, 0),
        ("gray_chain_kernel", "Segmentation, 240 x 512 x 512 u8", "hbm", 2 * 240 * 512 * 512, 0),
        ("nbody_force_kernel<true>", "N-body force + kick-drift, 65536 bodies", "alu", 65536 * 65536, 0),
        ("nbody_force_kernel<false>", "N-body force only, 65536 bodies", "alu", 65536 * 65536, 0),
    ]


def last_dispatches(dispatch_csv, key, last):
    """Mean duration (ns) of the last `last` dispatches of the kernel whose name
    contains `key`, from a per-dispatch trace; None if there are fewer."""
    rows = sorted(csv.DictReader(open(dispatch_csv)), key=lambda r: int(r["Start_Timestamp"]))
    d = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows if key in r["Kernel_Name"]]
    if len(d) < last:
        return None
    return sum(d[-last:]) / last


def row_roofline(stats, dispatch_csv=None):
    out = ["", "## Rooflines of the kernels that serve one workload each", "",
           "Achieved = work per launch / rocprof average duration (of the timed runs' dispatches where the "
           "kernel also serves other runs); peaks: HBM 8 TB/s, N-body 256 CUs x 64 lanes x 2.4 GHz / 13 VALU "
           "issues per pair.", "",
           "| kernel | workload | work per launch | avg us | achieved | peak | frac |", "|---|---|---|---|---|---|---|"]
    for key, what, kind, work, last in row_work():
        r = next((x for x in stats if key in x["name"]), None)
        if r is None:
            continue
        avg_ns = r["avg_ns"]
        if last and dispatch_csv:
            m = last_dispatches(dispatch_csv, key, last)
            if m is not None:
                avg_ns = m
        r = dict(r, avg_ns=avg_ns)
        sec = r["avg_ns"] * 1e-9
        if kind == "hbm":
            ach, peak, unit, wl = work / sec / 1e9, HBM_PEAK_GBS, "GB/s", f"{work} B"
        else:
            ach, peak, unit, wl = work / sec / 1e9, NBODY_PEAK_GPAIRS, "G pairs/s", f"{work} pairs"
        out.append(f"| `{key}` | {what} | {wl} | {r['avg_ns']/1e3:.2f} | {ach:.1f} {unit} | {peak:.1f} | "
                   f"{ach / peak:.3f} |")
    return out


def while_phases(path):
    """Image-kernel durations of the traced while run split by loop form.  The
    while plan's dispatches end with its last final-copy launch; after it, an
    iteration whose merge is followed by a device-to-host copy belongs to the
    host-checked loop, any other to the unchecked one."""
    import statistics
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    seq = [(r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows]
    last_copy = max(i for i, x in enumerate(seq) if "while_copy_kernel" in x[0])
    phase = {"while plan": [], "host-checked": [], "unchecked": []}
    step = []
    for i, (name, t0, t1) in enumerate(seq):
        if "while_step_kernel" in name:
            step.append(t1 - t0)
        if "img_" not in name:
            continue
        if i < last_copy:
            phase["while plan"].append(t1 - t0)
            continue
        nxt = [x[0] for x in seq[i + 1:i + 4]]
        phase["host-checked" if any("copyBuffer" in n for n in nxt) else "unchecked"].append(t1 - t0)
    out = ["", "Image kernel per dispatch, by loop form (from the per-dispatch trace of the same run):", "",
           "| loop form | dispatches | median us | mean us |", "|---|---|---|---|"]
    for k, v in phase.items():
        if v:
            out.append(f"| {k} | {len(v)} | {statistics.median(v)/1e3:.2f} | {statistics.mean(v)/1e3:.2f} |")
    if step:
        out += ["", f"Step kernel: {len(step)} dispatches, median {statistics.median(step)/1e3:.2f} us."]
    return out


COMMAND_DRIVER = ("rocprofv3 --kernel-trace --stats -d DIR -o driver --output-format csv -- python3 bench.py "
                  "--gpus 1 --steps 20 --warmup 5")
PLAIN_FIRST = "img_band_kernel<1, 0, false, false, 0>"   # noise alone: the plain plan's first kernel


def driver_phase(dispatch_csv, steps):
    """Durations (ns) of the fused 8192^2 kernel's dispatches in the headline
    measurement of a default bench run: every dispatch of the fused kernel
    before the plain plan's first kernel (warm-up, timed steps, then the
    `steps` launches whose HIP events give roofline.kernel_ms, last)."""
    rows = sorted(csv.DictReader(open(dispatch_csv)), key=lambda r: int(r["Start_Timestamp"]))
    out = []
    for r in rows:
        if PLAIN_FIRST in r["Kernel_Name"]:
            break
        if FUSED in r["Kernel_Name"]:
            out.append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out, out[-steps:]


def driver_summary(stats_csv, dispatch_csv, bench_json):
    import statistics
    line = json.loads([ln for ln in open(bench_json) if ln.startswith("{")][-1])
    steps = int(line["steps"])
    allf, last = driver_phase(dispatch_csv, steps)
    algo = line["roofline"]["algorithmic_bytes"]
    mean = statistics.mean(last)
    out = ["# rocprofv3 summary: the default bench command, fused Pipeline+MapReduce 8192x8192 RGBA u8 "
           "(headline kernel) and every other kernel of the run", "",
           "Command (repository root on the MI355X host, TMPDIR=/tmp):", "", "```", COMMAND_DRIVER, "```", "",
           "## Headline kernel in this run", "",
           f"The bench line printed under the profiler: value {line['value']} {line['unit']}, ms_per_step "
           f"{line['ms_per_step']}, roofline.kernel_ms {line['roofline']['kernel_ms']} (HIP events around the "
           f"last {steps} launches), frac {line['roofline']['frac']}.", "",
           f"From the per-dispatch trace, the fused kernel `{FUSED}` ran {len(allf)} times before the plain plan "
           f"started (the untimed warm-up floor, the {steps} timed steps, then the {steps} launches the HIP "
           "events bracket):", "",
           "| dispatches | mean us | median us | min us | max us | frac of 8 TB/s (algorithmic bytes / mean) |",
           "|---|---|---|---|---|---|",
           f"| last {steps} | {mean/1e3:.2f} | {statistics.median(last)/1e3:.2f} | {min(last)/1e3:.2f} | "
           f"{max(last)/1e3:.2f} | {algo / (mean * 1e-9) / 1e9 / HBM_PEAK_GBS:.4f} |",
           f"| first 20 (clock ramp) | {statistics.mean(allf[:20])/1e3:.2f} | {statistics.median(allf[:20])/1e3:.2f} "
           f"| {min(allf[:20])/1e3:.2f} | {max(allf[:20])/1e3:.2f} | "
           f"{algo / (statistics.mean(allf[:20]) * 1e-9) / 1e9 / HBM_PEAK_GBS:.4f} |",
           f"| all {len(allf)} | {statistics.mean(allf)/1e3:.2f} | {statistics.median(allf)/1e3:.2f} | "
           f"{min(allf)/1e3:.2f} | {max(allf)/1e3:.2f} | "
           f"{algo / (statistics.mean(allf) * 1e-9) / 1e9 / HBM_PEAK_GBS:.4f} |", "",
           f"Algorithmic bytes per launch: {algo} (image read and written once, 4 x 256 x 4 B histogram, 4 x 8 B "
           "sums).", "",
           "## Kernel statistics of the whole run (--stats; averages mix workloads where one kernel serves "
           "several)", "", "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for r in kernel_stats(stats_csv)[:25]:
        out.append(f"| `{r['name'][:90]}` | {r['calls']} | {r['avg_ns']/1e3:.2f} | {r['min_ns']/1e3:.2f} | "
                   f"{r['max_ns']/1e3:.2f} |")
    return out


COMMANDS_OTHER = (
    "rocprofv3 --pmc FETCH_SIZE -d DIR -o ofetch --output-format csv -- python3 bench.py --counters-run --steps 5",
    "rocprofv3 --pmc WRITE_SIZE -d DIR -o owrite --output-format csv -- python3 bench.py --counters-run --steps 5",
    "rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_VALU "
    "SQ_BUSY_CYCLES SQ_WAVE_CYCLES -d DIR -o osq --output-format csv -- python3 bench.py --counters-run --steps 3",
    "python -m paper_1510_06585_amd.rocprof_harness --other-fetch DIR/ofetch_counter_collection.csv "
    "--other-write DIR/owrite_counter_collection.csv --other-sq DIR/osq_counter_collection.csv --out profiles/",
)
SIMDS = 256 * 4          # 4 SIMDs per CU
SQ_ENGINES = 32          # shader engines summed by SQ_BUSY_CYCLES


def other_work():
    """(kernel-name key, workload, algorithmic bytes per launch, work units per
    launch, unit name) of the kernels `bench.py --counters-run` launches."""
    import synth
    sides = synth.batch_sides(synth.SEED_BATCH, 256)
    n_fft = 512 * 65536
    N = 65536
    return [
        ("img_batch_kernel<9, 0, true, true, 2>", "256 uneven requests, noise>solarise>blur>mirror + histogram",
         sum(2 * s * s * 4 + 4128 for s in sides), sum(s * s for s in sides), "pixel"),
        ("fft_pass_kernel<0>", "FFT pass A, 512 x 65536 complex fp32", 2 * n_fft * 8, n_fft, "element"),
        ("fft_pass_kernel<1>", "FFT fused pass B+A", 2 * n_fft * 8, n_fft, "element"),
        ("fft_pass_kernel<2>", "FFT pass B", 2 * n_fft * 8, n_fft, "element"),
        ("vec_chain_kernel", "saxpy, 5 x 10^7 fp32 (read v, w; write out)", 12 * 50_000_000, 50_000_000,
         "element"),
        ("gray_chain_kernel", "Segmentation, 240 x 512 x 512 u8", 2 * 240 * 512 * 512, 240 * 512 * 512, "voxel"),
        ("nbody_force_kernel<true>", "N-body force + kick-drift, 65536 bodies (one step)",
         4 * N * 16, N * N, "pair"),
    ]


def other_summary(fetch_csv, write_csv, sq_csv):
    """Counter summary of the other workloads' kernels: bytes moved between L2
    and the memory fabric (FETCH_SIZE / WRITE_SIZE scaled by the copy kernel),
    and VALU instructions per work unit with their share of the busy cycles."""
    f, w = counters(fetch_csv), counters(write_csv)
    sq = counters(sq_csv) if sq_csv else {}
    cf, cw = _find(f, COPY)["FETCH_SIZE"], _find(w, COPY)["WRITE_SIZE"]
    sf = (COPY_BYTES / 2) / (cf * 1024.0)
    sw = (COPY_BYTES / 2) / (cw * 1024.0)
    out = ["# rocprofv3 counters: the kernels of the batched, FFT, saxpy, Segmentation and N-body workloads", "",
           "Commands (repository root on the MI355X host, TMPDIR=/tmp):", "", "```"] + list(COMMANDS_OTHER) + [
           "```", "",
           "`bench.py --counters-run` runs a plain copy of an 8192^2 RGBA image (the byte reference), the "
           "256-request batch at its default plan, the FFT -> IFFT chain over 512 transforms, one saxpy stage, "
           "one Segmentation stage (5 runs each in the byte passes, 3 in the SQ pass) and one 20-step N-body "
           "loop.  FETCH_SIZE and WRITE_SIZE (KiB per dispatch) count what leaves and enters the L2; both are "
           f"scaled by the copy kernel's known 256 MiB each way (fetch x {sf:.4f}, write x {sw:.4f}).  Where "
           "the input fits the 256 MB MALL (Segmentation's 60 MiB), fetched bytes may be served there rather "
           "than by HBM.", "",
           "## Bytes per launch", "",
           "| kernel | workload | algorithmic B | fetched B | written B | measured / algorithmic |",
           "|---|---|---|---|---|---|"]
    for key, what, algo, units, unit in other_work():
        fk, wk = _find_opt(f, key), _find_opt(w, key)
        if not fk or not wk:
            continue
        fb = fk["FETCH_SIZE"] * 1024.0 * sf
        wb = wk["WRITE_SIZE"] * 1024.0 * sw
        out.append(f"| `{key}` | {what} | {algo} | {fb:.0f} | {wb:.0f} | {(fb + wb) / algo:.3f} |")
    if sq:
        out += ["", "## VALU work (SQ counters, mean per dispatch)", "",
                "VALU lane-instructions per unit = SQ_INSTS_VALU x 64 / units.  Issue share = "
                f"(SQ_INSTS_VALU x 4 cycles / {SIMDS} SIMDs) / (SQ_BUSY_CYCLES / {SQ_ENGINES} engines): the "
                "fraction of the busy cycles in which each SIMD issues a VALU instruction.", "",
                "| kernel | units | SQ_WAVES | SQ_INSTS_VALU | VALU per unit | SQ_INSTS_SALU | SQ_INSTS_LDS | "
                "SQ_LDS_BANK_CONFLICT | SQ_BUSY_CYCLES | issue share |", "|---|---|---|---|---|---|---|---|---|---|"]
        for key, what, algo, units, unit in other_work() + [(COPY, "copy", 0, 8192 * 8192, "pixel")]:
            c = _find_opt(sq, key)
            if not c:
                continue
            valu = c.get("SQ_INSTS_VALU", 0.0)
            busy = c.get("SQ_BUSY_CYCLES", 0.0)
            share = (valu * 4.0 / SIMDS) / (busy / SQ_ENGINES) if busy else float("nan")
            out.append(f"| `{key}` | {units} {unit}s | {c.get('SQ_WAVES', 0):.0f} | {valu:.0f} | "
                       f"{valu * 64 / units:.2f} | {c.get('SQ_INSTS_SALU', 0):.0f} | {c.get('SQ_INSTS_LDS', 0):.0f} | "
                       f"{c.get('SQ_LDS_BANK_CONFLICT', 0):.0f} | {busy:.0f} | {share:.3f} |")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--driver-stats", help="kernel stats of the default bench command under the profiler")
    ap.add_argument("--driver-dispatches", help="the per-dispatch kernel trace of the same run")
    ap.add_argument("--driver-json", help="the JSON line that run printed")
    ap.add_argument("--trace")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--sq")
    ap.add_argument("--trace-all", help="kernel stats of the whole bench run (every skeleton)")
    ap.add_argument("--trace-all-dispatches", help="the per-dispatch kernel trace of the same run")
    ap.add_argument("--trace-filter-pipeline", help="kernel stats of the 1024x1024 filter-pipeline run alone (per-stage times)")
    ap.add_argument("--mlp-counters", help="MFMA counter pass over the cost-model MLP kernels")
    ap.add_argument("--trace-while", help="kernel stats of the 8192x8192 x 10 while Loop run alone")
    ap.add_argument("--while-json", help="the JSON line the traced while run printed (per-iteration wall times)")
    ap.add_argument("--while-dispatches", help="the per-dispatch kernel trace of the same while run")
    ap.add_argument("--other-fetch", help="FETCH_SIZE pass over bench.py --counters-run")
    ap.add_argument("--other-write", help="WRITE_SIZE pass over bench.py --counters-run")
    ap.add_argument("--other-sq", help="SQ counter pass over bench.py --counters-run")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    os.makedirs(a.out, exist_ok=True)
    if a.driver_stats and a.driver_dispatches and a.driver_json:
        d = driver_summary(a.driver_stats, a.driver_dispatches, a.driver_json)
        open(os.path.join(a.out, "driver_command_8192.md"), "w").write("\n".join(d) + "\n")
    if a.trace_filter_pipeline:
        c1 = ["# rocprofv3 summary: filter pipeline 1024x1024 RGBA u8 (noise > solarise > mirror), plain plan "
              "(one kernel per stage) and fused plan, 220 runs each", "",
              "Command (repository root on the MI355X host, TMPDIR=/tmp):", "", "```", COMMAND_FILTER_PIPELINE, "```", "",
              "Kernels: `img_band_kernel<1, 0, false, false, 0>` is the noise stage, `<2, 0, false, false, 0>` "
              "solarise, `<0, 0, false, false, 2>` mirror (a copy with the store flipped), "
              "`<9, 0, false, false, 2>` the fused chain.", "",
              "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
        for r in kernel_stats(a.trace_filter_pipeline):
            c1.append(f"| `{r['name'][:90]}` | {r['calls']} | {r['avg_ns']/1e3:.2f} | {r['min_ns']/1e3:.2f} | "
                      f"{r['max_ns']/1e3:.2f} |")
        open(os.path.join(a.out, "img_filter_pipeline_1024.md"), "w").write("\n".join(c1) + "\n")
    if a.trace_while:
        stats = kernel_stats(a.trace_while)
        cw = ["# rocprofv3 summary: while Loop, noise > solarise > blur > mirror + histogram body over "
              "8192x8192 RGBA u8, 10 iterations", "",
              "Command (repository root on the MI355X host, TMPDIR=/tmp):", "", "```", COMMAND_WHILE, "```", "",
              "The run times, 10 iterations each, the while plan with host checks in blocks of 8 and then the "
              "asynchronous while plan with the convergence condition and both reduce outputs carried (each "
              "after the warm-up floor, then 10 timed runs; both count as \"while plan\" below), the same body "
              "with the sums read back by the host after every iteration and the body alone, unchecked.  Per "
              "iteration a while plan launches the image kernel, the histogram merge and the step kernel "
              "(one work-group: the carried merges, the count and the condition); per run one init kernel "
              "and one final guarded copy.", "",
              "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
        for r in stats:
            cw.append(f"| `{r['name'][:90]}` | {r['calls']} | {r['avg_ns']/1e3:.2f} | {r['min_ns']/1e3:.2f} | "
                      f"{r['max_ns']/1e3:.2f} |")
        busy = {}
        for key in ("img_", "hist_merge_kernel", "while_step_kernel"):
            r = [x for x in stats if key in x["name"]]
            if r:
                busy[key] = sum(x["avg_ns"] * x["calls"] for x in r) / max(sum(x["calls"] for x in r), 1) / 1e3
        if busy:
            cw += ["", "Mean per dispatch over all three loop forms: " +
                   ", ".join(f"{k.strip('_')} {v:.2f} us" for k, v in busy.items()) +
                   f"; total {sum(busy.values()):.2f} us."]
        if a.while_dispatches:
            cw += while_phases(a.while_dispatches)
        if a.while_json:
            w = json.loads([ln for ln in open(a.while_json) if ln.startswith("{")][-1])
            asy = w.get("async_delta_carried_ms_per_iteration")
            cw += ["", "Wall time per iteration under the profiler (ms): "
                   f"while plan {w['device_condition_ms_per_iteration']}"
                   + (f", asynchronous while plan (convergence condition, carried outputs) {asy}" if asy else "")
                   + f", host-checked body {w['host_condition_ms_per_iteration']}, unchecked body "
                   f"{w['no_condition_ms_per_iteration']}."]
        open(os.path.join(a.out, "while_loop_8192.md"), "w").write("\n".join(cw) + "\n")
    if a.other_fetch and a.other_write:
        oc = other_summary(a.other_fetch, a.other_write, a.other_sq)
        open(os.path.join(a.out, "other_kernels_counters.md"), "w").write("\n".join(oc) + "\n")
    if a.mlp_counters:
        cm = counters(a.mlp_counters)
        n = 16384
        fwd_flops = 2 * n * (24 * 64 + 64 * 64 + 64)
        ml = ["# rocprofv3 counters: cost-model MLP kernels on the matrix cores (16384 samples, 24->64->64->1)", "",
              "Command (repository root on the MI355X host, TMPDIR=/tmp):", "", "```", COMMAND_MLP, "```", "",
              "`bench.py --mlp-profile-run` runs `skel_mlp_forward` and `skel_mlp_grad` three times each on 16384 random "
              f"samples.  The forward pass's layer products are {fwd_flops} flops; one "
              "SQ_INSTS_VALU_MFMA_MOPS_F32 count is 512 flops.", "",
              "| kernel | counter | mean per dispatch |", "|---|---|---|"]
        for kern in sorted(cm):
            if "mlp" not in kern:
                continue
            short = kern.split("(")[0].replace("skel::", "")
            for c, v in sorted(cm[kern].items()):
                ml.append(f"| `{short}` | {c} | {v:.0f} |")
            mops = cm[kern].get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0)
            if mops:
                ml.append(f"| `{short}` | MFMA flops (MOPS x 512) | {mops * 512:.0f} |")
        open(os.path.join(a.out, "mlp_mfma_16384.md"), "w").write("\n".join(ml) + "\n")
    if a.trace_all:
        al = ["# rocprofv3 kernel trace of the whole bench run (every skeleton's kernels)", "",
              "Command (repository root on the MI355X host, TMPDIR=/tmp):", "", "```", COMMANDS[1], "```", "",
              "Averages mix workloads where one kernel serves several (e.g. the fused image kernel runs the "
              "8192^2 image and, in the sequential baseline of the batch, 256 smaller ones).", "",
              "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
        stats_all = kernel_stats(a.trace_all)
        for r in stats_all:
            al.append(f"| `{r['name'][:90]}` | {r['calls']} | {r['avg_ns']/1e3:.2f} | {r['min_ns']/1e3:.2f} | "
                      f"{r['max_ns']/1e3:.2f} |")
        al += row_roofline(stats_all, a.trace_all_dispatches)
        open(os.path.join(a.out, "bench_all_kernels.md"), "w").write("\n".join(al) + "\n")
    if not (a.trace and a.fetch and a.write):
        return
    st = kernel_stats(a.trace)
    tr = traffic(a.fetch, a.write)
    src = os.path.join(HERE, "csrc", "kern_img.hip")
    rec = {"kernel": FUSED_NAME, "source": "kern_img.hip",
           "source_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(),
           "bytes_per_launch": round(tr["bytes_per_launch"]),
           "algorithmic_bytes": 2 * 8192 * 8192 * 4 + 4128, **{k: round(v, 4) for k, v in tr.items()}}
    json.dump(rec, open(os.path.join(a.out, f"traffic_{FUSED_NAME}.json"), "w"), indent=1)
    lines = ["# rocprofv3 summary: fused Pipeline+MapReduce, 8192x8192 RGBA u8 (the bench run of this workload: fused "
             "plan, plain plan, copy reference)",
             "", "Commands (repository root on the MI355X host, TMPDIR=/tmp):", "", "```"] + list(COMMANDS)
    lines += ["```", "", "## Kernel trace (--kernel-trace --stats)", "",
              "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for r in st:
        lines.append(f"| `{r['name'][:90]}` | {r['calls']} | {r['avg_ns']/1e3:.2f} | {r['min_ns']/1e3:.2f} | "
                     f"{r['max_ns']/1e3:.2f} |")
    lines += ["", "## HBM traffic per launch (FETCH_SIZE, WRITE_SIZE; scaled by a copy kernel of 512 MiB)", ""]
    for k, v in rec.items():
        lines.append(f"- {k}: {v}")
    if a.sq:
        sq = counters(a.sq)
        lines += ["", "## SQ counters (mean per dispatch)", "", "| kernel | counter | value |", "|---|---|---|"]
        for kern in (FUSED, COPY):
            for c, v in sorted(_find(sq, kern).items()):
                lines.append(f"| `{kern}` | {c} | {v:.0f} |")
    open(os.path.join(a.out, f"{FUSED_NAME}_8192.md"), "w").write("\n".join(lines) + "\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
