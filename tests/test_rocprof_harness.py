"""CPU tests of the rocprofv3 summary harness's parsers on small synthetic
trace files: the per-kernel statistics table and the split of the while-Loop
run's image-kernel dispatches by loop form."""
import csv

from paper_1510_06585_amd import rocprof_harness as rh


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_ALL)
        w.writerow(header)
        w.writerows(rows)


def test_kernel_stats_reads_rocprof_columns(tmp_path):
    p = tmp_path / "k_kernel_stats.csv"
    _write(p, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
           [["skel::a(int)", "3", "300", "100.0", "75.0", "90", "110", "8.1"],
            ["skel::b(int)", "1", "100", "100.0", "25.0", "100", "100", "0"]])
    st = rh.kernel_stats(str(p))
    assert [r["name"] for r in st] == ["skel::a(int)", "skel::b(int)"]
    assert st[0]["calls"] == 3 and st[0]["avg_ns"] == 100.0 and st[0]["min_ns"] == 90.0 and st[0]["pct"] == 75.0


def test_while_phases_splits_by_loop_form(tmp_path):
    t = [0]

    def d(name, dur):
        row = ["KERNEL_DISPATCH", name, str(t[0]), str(t[0] + dur)]
        t[0] += dur + 10
        return row

    rows = []
    for _ in range(2):                      # while plan: 3 iterations per run, then the final copy
        rows.append(d("skel::while_init_kernel(unsigned int*)", 5))
        for _ in range(3):
            rows += [d("void skel::img_band_kernel<9>(skel::ImgGroupArgs)", 1300),
                     d("skel::hist_merge_kernel(skel::HistFinArgs)", 60),
                     d("skel::while_step_kernel(unsigned int*)", 48)]
        rows.append(d("skel::while_copy_kernel(unsigned int const*)", 40))
    for _ in range(4):                      # host-checked: sums read back after every merge
        rows += [d("void skel::img_band_kernel<9>(skel::ImgGroupArgs)", 1270),
                 d("skel::hist_merge_kernel(skel::HistFinArgs)", 60),
                 d("__amd_rocclr_copyBuffer", 30)]
    for _ in range(5):                      # unchecked body
        rows += [d("void skel::img_band_kernel<9>(skel::ImgGroupArgs)", 1250),
                 d("skel::hist_merge_kernel(skel::HistFinArgs)", 60)]
    p = tmp_path / "w_kernel_trace.csv"
    _write(p, ["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    out = "\n".join(rh.while_phases(str(p)))
    assert "| while plan | 6 | 1.30 | 1.30 |" in out
    assert "| host-checked | 4 | 1.27 | 1.27 |" in out
    assert "| unchecked | 5 | 1.25 | 1.25 |" in out
    assert "Step kernel: 6 dispatches, median 0.05 us." in out


def test_driver_phase_takes_the_headline_launches(tmp_path):
    """The headline kernel's dispatches are those before the plain plan's
    first kernel; the last `steps` of them are the ones the bench's HIP
    events bracket."""
    t = [0]

    def d(name, dur):
        row = ["KERNEL_DISPATCH", name, str(t[0]), str(t[0] + dur)]
        t[0] += dur + 10
        return row

    fused = "void skel::img_band_kernel<9, 0, true, true, 2>(skel::ImgGroupArgs)"
    rows = []
    for k in range(30):                     # warm-up (clock ramp), timed steps, event-bracketed launches
        rows += [d(fused, 2000 if k < 10 else (1300 if k < 20 else 1200)),
                 d("skel::hist_merge_kernel(skel::HistFinArgs)", 50)]
    rows.append(d("void skel::img_band_kernel<1, 0, false, false, 0>(skel::ImgGroupArgs)", 900))
    rows.append(d(fused, 5000))             # the same kernel later in the run (another workload)
    p = tmp_path / "driver_kernel_trace.csv"
    _write(p, ["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    allf, last = rh.driver_phase(str(p), 10)
    assert len(allf) == 30 and last == [1200] * 10


def test_last_dispatches_mean(tmp_path):
    rows = [["KERNEL_DISPATCH", "void skel::img_batch_kernel<9>(x)", str(100 * i), str(100 * i + d)]
            for i, d in enumerate([50, 60, 10, 20, 30])]
    p = tmp_path / "t.csv"
    _write(p, ["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    assert rh.last_dispatches(str(p), "img_batch_kernel", 3) == 20.0
    assert rh.last_dispatches(str(p), "img_batch_kernel", 6) is None


def test_other_summary_scales_bytes_by_the_copy_kernel(tmp_path):
    """Bytes are the counter readings times (known copy bytes / the copy
    kernel's reading), per direction; VALU per unit and the issue share
    follow from the SQ readings."""
    copy = "void skel::img_band_kernel<0, 0, false, false, 0>(skel::ImgGroupArgs)"
    seg = "skel::gray_chain_kernel(skel::GrayArgs)"
    half = rh.COPY_BYTES // 2
    vox = 240 * 512 * 512
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    # the copy reads back half its bytes in FETCH_SIZE and all of them in
    # WRITE_SIZE: scales 2 and 1; the Segmentation kernel reads 30 and 20 MiB
    _write(tmp_path / "f.csv", hdr, [[copy, "FETCH_SIZE", str(half / 2048)], [copy, "FETCH_SIZE", str(half / 2048)],
                                     [seg, "FETCH_SIZE", str(30 * 1024)]])
    _write(tmp_path / "w.csv", hdr, [[copy, "WRITE_SIZE", str(half / 1024)], [seg, "WRITE_SIZE", str(20 * 1024)]])
    busy = 32 * 1000.0
    valu = 1024 * 500 / 4.0          # each SIMD issues for 500 of its 1000 busy cycles
    _write(tmp_path / "s.csv", hdr, [[seg, "SQ_INSTS_VALU", str(valu)], [seg, "SQ_BUSY_CYCLES", str(busy)],
                                     [seg, "SQ_WAVES", "4096"]])
    out = "\n".join(rh.other_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "s.csv")))
    mib = 1 << 20
    algo = 2 * vox
    assert (f"| `gray_chain_kernel` | Segmentation, 240 x 512 x 512 u8 | {algo} | {60 * mib} | {20 * mib} | "
            f"{80 * mib / algo:.3f} |") in out
    assert f"| {valu:.0f} | {valu * 64 / vox:.2f} |" in out
    assert out.rstrip().endswith("| 0.500 |")
    assert "fetch x 2.0000, write x 1.0000" in out
