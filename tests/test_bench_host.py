"""Host logic of the benchmark's profile pipeline (CPU only), on synthetic
rocprofv3 CSV files: the kernel-trace summary splits the run into its
workloads, and the counter summary scales FETCH_SIZE / WRITE_SIZE by the copy
probe and assigns the transform's dispatches to passes in launch order."""
import csv
import json
import os

import pytest

import bench

KERNELS = ["void pf::k_r2c_p2<512, 0>(pf::PassArgs)",
           "void pf::k_c2c_p2<1024, 16, -1, 0, 0, 0>(pf::PassArgs)",
           "void pf::k_c2c_p2<1024, 16, -1, 0, 1, 0>(pf::PassArgs)",
           "void pf::k_c2c_p2<1024, 16, 1, 1, 0, 0>(pf::PassArgs)",
           "void pf::k_c2c_p2<1024, 16, 1, 0, 0, 0>(pf::PassArgs)",
           "void pf::k_c2r_p2<512, 0>(pf::PassArgs)"]


@pytest.fixture
def tmp_root(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernels_digest", lambda: "digest")
    return tmp_path


def write_trace(path, names_ms):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 1000
        for i, (name, ms) in enumerate(names_ms):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Start_Timestamp": t,
                        "End_Timestamp": t + int(ms * 1e6)})
            t += int(ms * 1e6) + 10


def test_trace_summary_splits_the_workloads(tmp_root):
    trace = tmp_root / "kt.csv"
    names = [(KERNELS[0], 2.0), (KERNELS[0], 1.0), (KERNELS[1], 1.5),
             ("void pf::k_c2c_tile<float, -1>(pf::PassArgs)", 0.02),       # the batch begins
             ("void pf::k_c2c_tile_b<float, -1>(pf::BatchArgs)", 0.3),
             ("void pf::k_r2c_p2<256, 0>(pf::PassArgs)", 0.11),             # the spectral step begins
             ("void pf::k_spec_p2<512, 16, 0>(pf::PassArgs, int, float)", 0.23),
             ("pf::k_fill(pf::FillArgs)", 0.09),                            # the share-only leg begins
             (KERNELS[0], 0.28),
             ("void pf::k_r2c_p2d<256>(pf::PassArgs)", 0.41),               # the FP64 plan begins
             ("void pf::k_c2c_p2d<512, -1, 0, 0>(pf::PassArgs)", 0.44),
             ("void pf::k_c2r_p2d<256, true>(pf::PassArgs)", 0.48),
             ("void pf::k_r2c_p2<256, 0>(pf::PassArgs)", 0.4),              # the other grids begin
             ("void pf::k_mr_x<20, 24, 1>(pf::MrArgs)", 0.1),
             ("void pf::k_r2c_p2<1024, 0>(pf::PassArgs)", 0.9),             # the fused comparison begins
             ("void pf::k_xy_fused<1024, 512, 1>(pf::FusedArgs)", 1.7)]
    write_trace(trace, names)
    bench.summarize_trace(str(trace), "CMD", steps=10, warmup=2)
    prof = tmp_root / "profiles"
    main = (prof / "kernels_fft_1024cubed.txt").read_text()
    batch = (prof / "kernels_batch64_mixed.txt").read_text()
    spec = (prof / "kernels_cheb_spectral_512x512x257.txt").read_text()
    assert "command: CMD" in main and "command: CMD" in batch and "command: CMD" in spec
    # the 1024^3 table: two launches of the X kernel averaging 1.5 ms, then the share leg
    head, share = main.split("share-only leg")
    row = next(line for line in head.splitlines() if line.startswith(KERNELS[0]))
    assert row.split()[-5:-3] == ["2", "1.500"]
    assert "k_fill" in share and "k_fill" not in head and "k_c2c_tile" not in main
    assert "k_c2c_tile_b" in batch and "k_spec_p2" not in batch and "k_r2c_p2<512" not in batch
    assert "k_spec_p2" in spec and "k_fill" not in spec
    other = (prof / "kernels_fft_512cubed_480x360x250.txt").read_text()
    assert "k_r2c_p2<256" in other and "k_mr_x<20, 24, 1>" in other and "k_fill" not in other
    assert "k_xy_fused" not in other and "k_r2c_p2<1024" not in other
    assert "k_mr_x" not in share and "p2d" not in share
    f64 = (prof / "kernels_fft_512cubed_f64.txt").read_text()
    assert "k_r2c_p2d<256>" in f64 and "k_c2r_p2d<256, true>" in f64 and "k_r2c_p2<256" not in f64
    assert "p2d" not in other
    fused = (prof / "kernels_fft_2048x512x512_fused.txt").read_text()
    assert "k_r2c_p2<1024" in fused and "k_xy_fused<1024, 512, 1>" in fused and "k_mr_x" not in fused


def write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_counter_summary_scales_by_the_copy_probe_and_assigns_passes(tmp_root):
    n = 16
    copy_kib = bench.COPY_BYTES(n) / 1024.0
    # FETCH reads half of the copy's bytes (scale 2), WRITE all of them (scale 1)
    for counter, copy_val, path in (("FETCH_SIZE", copy_kib / 2, "fetch.csv"), ("WRITE_SIZE", copy_kib, "write.csv")):
        rows = []
        for rep in range(2):  # two forward + backward pairs: pass i reads i + 1 KiB
            rows += [(k, float(i + 1)) for i, k in enumerate(KERNELS)]
        rows += [("void pf::k_c2c_p2<1024, 16, -1, 0, 1, 1>(pf::PassArgs)", 99.0)]  # a later variant: not counted
        rows += [("pf::k_copy(HIP_vector_type<float, 4u> const*, HIP_vector_type<float, 4u>*, unsigned long)",
                  copy_val)]
        write_counters(tmp_root / path, counter, rows)
    bench.summarize_pmc(str(tmp_root / "fetch.csv"), str(tmp_root / "write.csv"), n, ["A", "B"])
    rec = json.loads((tmp_root / "profiles" / f"traffic_fft_{n}cubed.json").read_text())
    assert rec["kernels_sha256"] == "digest"
    assert rec["FETCH_SIZE"]["scale"] == pytest.approx(2.0) and rec["WRITE_SIZE"]["scale"] == pytest.approx(1.0)
    for i, name in enumerate(bench.PASS_ORDER):
        e = rec["passes"][name]
        assert e["kernel"] == KERNELS[i] and e["dispatches"] == 2
        assert e["fetch_bytes"] == pytest.approx(2 * 1024 * (i + 1))
        assert e["write_bytes"] == pytest.approx(1024 * (i + 1))
        assert e["hbm_bytes"] == pytest.approx(3 * 1024 * (i + 1))
    assert os.path.exists(tmp_root / "profiles" / f"traffic_fft_{n}cubed.txt")


def test_sq_summary_normalises_by_each_sections_grid(tmp_root):
    """VALU lane slots per complex mode use the grid of the dispatch's section: 1024^3 for the
    leading plans, 480 x 360 x 250 for the mixed-radix kernels of the other grids."""
    m1024 = 513 * 1024 * 1024
    m480 = 241 * 360 * 250
    plan = [("void pf::k_c2c_p2<1024, 16, 1, 1, 0, 0>(pf::PassArgs)", m1024 * 40 / 64),
            ("void pf::k_c2c_tile_b<float, 1>(pf::BatchArgs)", 1e6),              # the batch begins
            ("void pf::k_r2c_p2<256, 0>(pf::PassArgs)", 1e6),                     # the spectral step
            ("pf::k_fill(pf::FillArgs)", 1e6),                                    # the share-only leg
            ("void pf::k_r2c_p2<256, 0>(pf::PassArgs)", 1e6),                     # the other grids
            ("void pf::k_mr_c2c<18, 20, -1>(pf::MrArgs)", m480 * 150 / 64)]
    path = tmp_root / "sq.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
                               "End_Timestamp", "VGPR_Count", "Scratch_Size"])
        w.writeheader()
        for i, (name, valu) in enumerate(plan):
            for c in bench.SQ_COUNTERS:
                v = valu if c == "SQ_INSTS_VALU" else 1000.0
                w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v,
                            "Start_Timestamp": 0, "End_Timestamp": 1000000, "VGPR_Count": 128,
                            "Scratch_Size": 0})
    bench.summarize_sq(str(path), "CMD")
    text = (tmp_root / "profiles" / "counters_sq_fft.txt").read_text()
    assert "command: CMD" in text

    def row(prefix, after):
        part = text.split(after, 1)[1]
        return next(line for line in part.splitlines() if line.startswith(prefix)).split()

    r = row("void pf::k_c2c_p2<1024", "1024^3")
    assert float(r[-4]) == pytest.approx(40.0, abs=0.05)
    r = row("void pf::k_mr_c2c<18, 20, -1>", "other grids")
    assert float(r[-4]) == pytest.approx(150.0, abs=0.05)
    assert "k_fill" not in text  # the share-only leg is not summarised
    # the batch has no fixed grid: no per-element figure
    assert row("void pf::k_c2c_tile_b", "batched")[-4] == "-"


def test_mfma_summary_per_wave_and_busy_fraction(tmp_root):
    """MFMA instructions per wave and busy fraction against one XCD's active cycles (the CSV holds
    GRBM_GUI_ACTIVE summed over 8 XCDs)."""
    name = "void pf::k_c2c_p2<1024, 16, -1, 0, 0, 1>(pf::PassArgs)"
    vals = {"SQ_WAVES": 2048.0, "SQ_INSTS_VALU": 2048.0 * 300.0, "SQ_INSTS_LDS": 2048.0 * 20.0,
            "SQ_INSTS_MFMA": 2048.0 * 12.0, "SQ_VALU_MFMA_BUSY_CYCLES": 0.05 * 1024 * 1e6,
            "SQ_BUSY_CYCLES": 1.0, "GRBM_GUI_ACTIVE": 8e6}
    path = tmp_root / "mfma.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
                               "End_Timestamp"])
        w.writeheader()
        for c, v in vals.items():
            w.writerow({"Dispatch_Id": 1, "Kernel_Name": name, "Counter_Name": c, "Counter_Value": v,
                        "Start_Timestamp": 0, "End_Timestamp": 2000000})
    bench.summarize_mfma(str(path), "CMD")
    text = (tmp_root / "profiles" / "counters_mfma_fft.txt").read_text()
    row = next(line for line in text.splitlines() if line.startswith(name)).split()
    assert row[-4] == "12.0" and row[-3] == "5.00%" and row[-2] == "300.0" and row[-1] == "20.0"
    assert "command: CMD" in text


def test_more_than_one_gpu_is_refused():
    """One GPU only: --gpus N > 1 exits with status 2 and says so, before touching a GPU."""
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
