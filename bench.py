"""Benchmark: 3D R2C + C2R pencil FFT on one MI355X, FP32, 1024^3.

One step = one forward (R2C) and one backward (C2R) transform of a 1024^3
float32 real Gaussian random field (shell spectrum |k|^-5/3), out-of-place,
STRIDE1 (Z-pencil output [nxh][ny][nz]).  Inputs are resident in HBM before
the timed region.  Flops follow the 5 N log2 N convention per forward+backward
pair (2.5 N log2 N per real transform, the paper's Eq. 3 per-point count).

Prints one JSON line with the throughput, a roofline object for the dominant
kernel (algorithmic bytes / measured HIP-event duration per launch), and the
CPU FP64 oracle timed on the host as a reported baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import statistics
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024, help="grid edge (default 1024)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=1024, help="grid edge of the CPU baseline sample")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs of this benchmark (FETCH_SIZE, WRITE_SIZE) "
                         "into profiles/ and exit")
    ap.add_argument("--pmc-commands", nargs=2, default=None, help="the two commands that produced the CSVs")
    ap.add_argument("--kt-summary", nargs=2, metavar=("TRACE_CSV", "COMMAND"),
                    help="write the per-kernel summaries under profiles/ from a rocprofv3 kernel trace of this "
                         "benchmark (COMMAND: the rocprofv3 command that produced it), then exit")
    ap.add_argument("--mfma-workload", action="store_true",
                    help="run only the plain and matrix-core FP32 plans at the grid edge --n (one warm-up and "
                         "--steps pairs each), for a rocprofv3 --pmc run with MFMA_COUNTERS, then exit")
    ap.add_argument("--mfma-summary", nargs=2, metavar=("COUNTER_CSV", "COMMAND"),
                    help="write profiles/counters_mfma_fft.txt from a rocprofv3 --pmc run of --mfma-workload, "
                         "then exit")
    ap.add_argument("--sq-summary", nargs=2, metavar=("COUNTER_CSV", "COMMAND"),
                    help="write profiles/counters_sq_fft.txt from a rocprofv3 --pmc run of this benchmark with "
                         "the SQ instruction counters (COMMAND: the rocprofv3 command that produced it), then exit")
    return ap.parse_args()


KERNEL_SOURCES = ("kernels.hip", "kernels_p2.hip", "fft_device.h", "pf_internal.h")
PASS_ORDER = ("fwd_x_r2c", "fwd_y_c2c", "fwd_z_c2c", "bwd_z_c2c", "bwd_y_c2c", "bwd_x_c2r")


def kernels_digest() -> str:
    """sha256 over the kernel sources: counters taken from other kernels do not apply."""
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1905_02803_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_path(n: int) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_fft_{n}cubed.json")


def traffic_from_profile(pass_name: str, n: int):
    """Measured HBM bytes per launch of a pass from the committed counter summary, if the kernels match."""
    path = traffic_path(n)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernels_sha256") != kernels_digest():
        return None
    p = rec.get("passes", {}).get(pass_name)
    return None if p is None else p["hbm_bytes"]


def section_starts(names):
    """Dispatch indices where the benchmark's sections start, from the kernel names in launch order:
    the batch (first runtime-radix or mixed-radix launch), the spectral step (its first k_r2c_p2<256, ...>), the
    share-only leg (its first fill), the FP64 512^3 plan (its first FP64 kernel) and the other grids
    (the next k_r2c_p2<256, ...>)."""

    def first(pred, start=0):
        return next((i for i in range(start, len(names)) if pred(names[i])), len(names))

    generic = ("k_c2c_tile", "k_r2c_x", "k_c2r_x", "k_mr_")
    b0 = first(lambda k: any(g in k for g in generic))
    s0 = first(lambda k: "k_r2c_p2<256" in k, b0)
    h0 = first(lambda k: "k_fill" in k, s0)
    o0 = first(lambda k: "k_r2c_p2<256" in k, h0)
    # the FP64 512^3 plan (its FP64 kernels: k_*_p2d, or a runtime-radix <double, ...>) runs
    # between the share-only leg and the other grids
    f0 = first(lambda k: "_p2d<" in k or "<double" in k, h0)
    # the fused comparison at 2048 x 512 x 512 (its X kernel k_r2c_p2<1024, ...>) runs last
    c0 = first(lambda k: "k_r2c_p2<1024" in k, o0)
    return b0, s0, h0, min(f0, o0), o0, c0


def summarize_trace(trace_csv: str, command: str, steps: int, warmup: int) -> None:
    """Per-kernel statistics from a rocprofv3 kernel trace of this benchmark, one file per workload.

    Dispatches are split where each section of the run starts: the 1024^3 plans
    (plain, matrix-core variants, layout variants) up to the first generic-kernel
    launch, which opens the batched section; the spectral step from its first
    X launch (k_r2c_p2<256, ...>); the share-only leg from its first fill; the
    other grids (512^3, then 480 x 360 x 250) from the next k_r2c_p2<256, ...>.
    """
    import csv

    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    b0, s0, h0, f0, o0, c0 = section_starts([r["Kernel_Name"] for r in rows])

    def table(rs):
        d = {}
        for r in rs:
            d.setdefault(r["Kernel_Name"], []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
        tot = sum(sum(v) for v in d.values()) or 1.0
        out = [f"{'kernel':60s} {'calls':>7s} {'avg ms':>9s} {'min ms':>9s} {'max ms':>9s} {'% time':>7s}"]
        for k, v in sorted(d.items(), key=lambda kv: -sum(kv[1])):
            n = k if len(k) <= 60 else k[:57] + "..."
            out.append(f"{n:60s} {len(v):7d} {statistics.mean(v):9.3f} {min(v):9.3f} {max(v):9.3f} "
                       f"{100 * sum(v) / tot:7.2f}")
        return out

    pairs = steps + warmup
    head = [f"command: {command}", "durations from the kernel trace (End - Start per dispatch), MI355X", ""]
    files = {
        "kernels_fft_1024cubed.txt": [
            "rocprofv3 kernel-trace statistics, 1024^3 FP32 R2C+C2R, STRIDE1, out-of-place", *head,
            f"full-grid plans: plain FP32 kernels <.., 0>: {pairs} pairs = {warmup} warm-up + {steps} timed; "
            "matrix-core variants",
            f"<.., 1> = FP16x2 and <.., 2> = BF16x2: {pairs} pairs each plus one forward for the error check; "
            "the copy probe;",
            f"the layout variants (Z-pencil without STRIDE1, in place, empty third transform: {pairs} pairs each, "
            "their plain",
            "kernels <.., 0> add to the counts above); torch kernels of the error checks and input copies",
            *table(rows[:b0]), "",
            "share-only leg: rank (0, 3) of a 1 x 8 grid, X-pencil [128][1024][1024] -> Z-pencil [513][128][1024],",
            f"{pairs} pairs (the same transform kernels on the rank's share, plus fills and block copies)",
            *table(rows[h0:f0])],
        "kernels_fft_512cubed_f64.txt": [
            "rocprofv3 kernel-trace statistics, FP64 R2C+C2R at 512^3, STRIDE1, out-of-place", *head,
            f"{pairs} pairs (k_c2c_p2d: the FP64 power-of-two Y / Z kernel; k_r2c_p2d / k_c2r_p2d: the X passes, "
            "<.., true> on the transposed workspace), then one forward for the oracle comparison",
            *table(rows[f0:o0])],
        "kernels_fft_512cubed_480x360x250.txt": [
            "rocprofv3 kernel-trace statistics, FP32 R2C+C2R at 512^3 (power-of-two kernels) and "
            "480 x 360 x 250 (mixed-radix kernels), STRIDE1, out-of-place", *head,
            f"{warmup + 2 * steps} pairs each ({warmup} warm-up, {steps} timed, {steps} timed with events "
            "between the passes)", *table(rows[o0:c0])],
        "kernels_fft_2048x512x512_fused.txt": [
            "rocprofv3 kernel-trace statistics, FP32 R2C+C2R at 2048 x 512 x 512, STRIDE1, out-of-place: "
            "the three-pass plan, then the fused X-Y plan", *head,
            f"{pairs} pairs each; k_xy_fused<1024, 512, FWD>: the fused X-Y pass", *table(rows[c0:])],
        "kernels_batch64_mixed.txt": [
            "rocprofv3 kernel-trace statistics, 64 batched FP32 R2C+C2R transforms "
            "(synth.batch_sizes(4, 64), 7-smooth sizes in [48, 320]^3)", *head,
            f"modes serial, serial + hipGraph, serial on 4 streams, fused, fused + hipGraph, fused on 4 "
            f"streams, with default and tuned plans: {pairs} pairs each;",
            "k_mr_c2c<N1, N2, DIR> / k_mr_x<N1, N2, FWD>: the compile-time mixed-radix passes (length N1 N2; "
            "one launch per transform and pass in",
            "the serial modes, per pass and length in the fused ones); k_*_b: fused launches of the runtime-radix "
            "passes (one per pass and block size),",
            "k_c2c_tile / k_r2c_x / k_c2r_x their serial launches", *table(rows[b0:s0])],
        "kernels_cheb_spectral_512x512x257.txt": [
            "rocprofv3 kernel-trace statistics, Chebyshev spectral step on 512 x 512 x 257 FP32 "
            "(type-I DCT along z)", *head,
            f"L u, L^T g and autograd forward + backward ({pairs} each), then {pairs} forward + backward "
            "transform pairs",
            "k_spec_sr<256, ADJ>: the fused z pass (split-radix DCT, product, inverse DCT); "
            "k_c2c_p2<512, .., 4>: the DCT Z passes (even extension)", *table(rows[s0:h0])],
    }
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    for name, lines in files.items():
        with open(os.path.join(ROOT, "profiles", name), "w") as f:
            f.write("\n".join(lines) + "\n")
        print(f"wrote profiles/{name} ({len(lines)} lines)")


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INSTS_LDS",
               "SQ_INSTS_SALU", "SQ_BUSY_CYCLES", "SQ_ACTIVE_INST_VALU")
# MI355X: 256 CUs of 4 SIMDs; without packed FP32 a wave64 VALU instruction holds its SIMD 4 cycles
VALU_SIMDS, VALU_CYCLES_PER_INST, CLOCK_GHZ = 1024, 4, 2.4


MFMA_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_MFMA", "SQ_VALU_MFMA_BUSY_CYCLES",
                 "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE")


def mfma_workload(n: int, steps: int) -> None:
    """The plain, FP16x2 and BF16x2 plans at n^3: one warm-up pair and `steps` pairs each."""
    import torch

    import paper_1905_02803_amd as pf

    u = torch.empty((n, n, n), device="cuda", dtype=torch.float32).uniform_(-1.0, 1.0)
    for math_ in (pf.PF_PLAIN, pf.PF_MFMA_FP16X2, pf.PF_MFMA_BF16X2):
        plan = pf.Plan(n, n, n, pf.Layout(math=math_))
        U = plan.empty_complex()
        r = plan.empty_real()
        for _ in range(1 + steps):
            plan.ftran(u, U)
            plan.btran(U, r)
        torch.cuda.synchronize()
        plan.destroy()
        print(f"bench: mfma workload, math {math_} done", file=sys.stderr, flush=True)


def summarize_mfma(counter_csv: str, command: str) -> None:
    """profiles/counters_mfma_fft.txt from a rocprofv3 --pmc run of --mfma-workload with MFMA_COUNTERS.

    Per kernel, per-dispatch averages: MFMA instructions per wave, the fraction of the SIMDs' active cycles
    the matrix cores were busy (rocprofv3's MfmaUtil: SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE of one
    XCD x 1024 SIMDs); the counter CSV holds GRBM_GUI_ACTIVE summed over the 8 XCDs), VALU and LDS
    instructions per wave, and the dispatch duration under counter collection.
    """
    import csv

    disp = {}
    for r in csv.DictReader(open(counter_csv)):
        d = disp.setdefault(int(r["Dispatch_Id"]), {
            "name": r["Kernel_Name"], "ms": (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6, "c": {}})
        d["c"][r["Counter_Name"]] = d["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    by = {}
    for d in disp.values():
        if "pf::k_" in d["name"] and "k_copy" not in d["name"]:
            by.setdefault(d["name"], []).append(d)
    lines = ["rocprofv3 matrix-core counters per dispatch, 1024^3 FP32 plans: plain (<.., 0>), FP16x2 (<.., 1>) "
             "and BF16x2 (<.., 2>), MI355X",
             f"command: {command}",
             "counters: " + " ".join(MFMA_COUNTERS),
             "mfma/wave, valu/wave, lds/wave: instructions per wave; mfma busy: SQ_VALU_MFMA_BUSY_CYCLES / "
             f"(GRBM_GUI_ACTIVE / 8 XCDs x {VALU_SIMDS} SIMDs) in %; avg ms: duration under counter collection",
             "",
             f"{'kernel':60s} {'calls':>5s} {'avg ms':>7s} {'mfma/wave':>9s} {'mfma busy':>9s} {'valu/wave':>9s} "
             f"{'lds/wave':>8s}"]
    for name, ds in sorted(by.items(), key=lambda kv: kv[0]):
        def avg(c):
            return sum(d["c"].get(c, 0.0) for d in ds) / len(ds)
        waves = avg("SQ_WAVES") or 1.0
        gui = (avg("GRBM_GUI_ACTIVE") or 8.0) / 8.0  # one XCD's active cycles
        busy = 100.0 * avg("SQ_VALU_MFMA_BUSY_CYCLES") / (gui * VALU_SIMDS)
        n = name if len(name) <= 60 else name[:57] + "..."
        lines.append(f"{n:60s} {len(ds):5d} {sum(d['ms'] for d in ds) / len(ds):7.3f} "
                     f"{avg('SQ_INSTS_MFMA') / waves:9.1f} {busy:8.2f}% {avg('SQ_INSTS_VALU') / waves:9.1f} "
                     f"{avg('SQ_INSTS_LDS') / waves:8.1f}")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "counters_mfma_fft.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote profiles/counters_mfma_fft.txt")


def summarize_sq(counter_csv: str, command: str) -> None:
    """Per-kernel instruction counts from a rocprofv3 --pmc run of this benchmark with SQ_COUNTERS.

    Writes profiles/counters_sq_fft.txt: for each section of the run (split as
    in the kernel-trace summary) and each of the library's kernels, the
    per-dispatch averages of the counters, and where the grid is fixed by the
    section, VALU lane slots per complex mode of the pass (SQ_INSTS_VALU x 64 /
    M, inactive lanes included) and the time the VALU instructions alone hold
    the SIMDs (SQ_INSTS_VALU x 4 cycles / 1024 SIMDs at 2.4 GHz) next to the
    dispatch's duration.  A kernel whose VALU time is near its duration is
    bound by VALU issue, one far below it by memory.
    """
    import csv

    disp = {}
    for r in csv.DictReader(open(counter_csv)):
        d = disp.setdefault(int(r["Dispatch_Id"]), {
            "name": r["Kernel_Name"], "ms": (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6,
            "scratch": r.get("Scratch_Size", ""), "c": {}})
        d["c"][r["Counter_Name"]] = float(r["Counter_Value"])
    ds = [disp[k] for k in sorted(disp)]
    b0, s0, h0, f0, o0, c0 = section_starts([d["name"] for d in ds])

    def modes(nx, ny, nz):
        return (nx // 2 + 1) * ny * nz

    m1024, m512 = modes(1024, 1024, 1024), modes(512, 512, 512)
    sections = [
        ("1024^3 FP32 plans (plain, matrix-core and layout variants; M = 513 x 1024 x 1024 complex modes)",
         ds[:b0], lambda k: m1024),
        ("64 batched transforms, 7-smooth sizes in [48, 320]^3 (serial and fused launches; sizes vary per "
         "dispatch)", ds[b0:s0], lambda k: None),
        ("Chebyshev spectral step on 512 x 512 x 257 (M = 257 x 512 x 257)", ds[s0:h0],
         lambda k: modes(512, 512, 257)),
        ("FP64 512^3 (M = 257 x 512 x 512)", ds[f0:o0], lambda k: m512),
        ("other grids: 512^3 on the power-of-two kernels (M = 257 x 512 x 512), 480 x 360 x 250 on the "
         "compile-time mixed-radix kernels k_mr_* (M = 241 x 360 x 250)", ds[o0:c0],
         lambda k: modes(480, 360, 250) if "k_mr_" in k else m512),
        ("2048 x 512 x 512, three-pass and fused X-Y plans (M = 1025 x 512 x 512)", ds[c0:],
         lambda k: modes(2048, 512, 512)),
    ]
    lines = ["rocprofv3 SQ instruction counters per dispatch, FP32 R2C+C2R workloads of the benchmark, MI355X",
             f"command: {command}",
             "counters: " + " ".join(SQ_COUNTERS),
             "avg ms: dispatch duration under counter collection (kernels serialised); waves: SQ_WAVES;",
             "valu/wave, vmem/wave (reads + writes), lds/wave: instructions per wave; lanes/elem: SQ_INSTS_VALU x 64 "
             "per complex mode;",
             f"valu ms: SQ_INSTS_VALU x {VALU_CYCLES_PER_INST} cycles / {VALU_SIMDS} SIMDs at {CLOCK_GHZ} GHz; "
             "valu/dur: valu ms over avg ms; scratch: bytes per lane", ""]
    hdr = (f"{'kernel':60s} {'calls':>5s} {'avg ms':>7s} {'waves':>9s} {'valu/wave':>9s} {'vmem/wave':>9s} "
           f"{'lds/wave':>8s} {'lanes/elem':>10s} {'valu ms':>8s} {'valu/dur':>8s} {'scratch':>7s}")
    for title, rs, elems in sections:
        by = {}
        for d in rs:
            if "pf::k_" in d["name"] and "k_copy" not in d["name"]:
                by.setdefault(d["name"], []).append(d)
        if not by:
            continue
        lines += [title, hdr]
        for k, v in sorted(by.items(), key=lambda kv: -sum(d["ms"] for d in kv[1])):
            def avg(c):
                return statistics.mean(d["c"].get(c, 0.0) for d in v)
            waves = avg("SQ_WAVES") or 1.0
            valu = avg("SQ_INSTS_VALU")
            ms = statistics.mean(d["ms"] for d in v)
            valu_ms = valu * VALU_CYCLES_PER_INST / (VALU_SIMDS * CLOCK_GHZ * 1e6)
            m = elems(k)
            per = f"{valu * 64 / m:10.1f}" if m else f"{'-':>10s}"
            name = k if len(k) <= 60 else k[:57] + "..."
            lines.append(f"{name:60s} {len(v):5d} {ms:7.3f} {waves:9.0f} {valu / waves:9.1f} "
                         f"{(avg('SQ_INSTS_VMEM_RD') + avg('SQ_INSTS_VMEM_WR')) / waves:9.1f} "
                         f"{avg('SQ_INSTS_LDS') / waves:8.1f} {per} {valu_ms:8.3f} "
                         f"{(valu_ms / ms if ms > 0 else 0.0):8.2f} {v[0]['scratch']:>7s}")
        lines.append("")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "counters_sq_fft.txt"), "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def summarize_pmc(fetch_csv: str, write_csv: str, n: int, commands) -> None:
    """Turn two rocprofv3 --pmc runs of this benchmark into profiles/traffic_fft_<n>cubed.{json,txt}.

    FETCH_SIZE / WRITE_SIZE are read per dispatch (KiB) and scaled by what the
    same counters read for the plain copy kernel k_copy, whose bytes are known.
    The transform's own kernels are assigned to passes in launch order
    (forward X, Y, Z, backward Z, Y, X, repeated), over the leading run of
    dispatches that repeats the first pair's six kernels: the plain 1024^3
    plan; the matrix-core variants and the share-only leg come later.
    """
    import csv

    def read(path):
        rows = list(csv.DictReader(open(path)))
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return rows

    out = {"kernels_sha256": kernels_digest(), "grid": n, "commands": commands, "passes": {}}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in read(path) if r["Counter_Name"] == counter]
        copies = [float(r["Counter_Value"]) * 1024.0 for r in rows if "k_copy(" in r["Kernel_Name"]]
        ours = [r for r in rows if "pf::k_" in r["Kernel_Name"] and "k_copy" not in r["Kernel_Name"]]
        period = [r["Kernel_Name"] for r in ours[:len(PASS_ORDER)]]
        run = 0
        while run < len(ours) and ours[run]["Kernel_Name"] == period[run % len(PASS_ORDER)]:
            run += 1
        ours = ours[:run - run % len(PASS_ORDER)]
        copy_bytes = COPY_BYTES(n)
        factor = copy_bytes / statistics.mean(copies) if copies else None
        out[counter] = {"copy_bytes_per_dispatch": copy_bytes,
                        "copy_counter_bytes": statistics.mean(copies) if copies else None,
                        "scale": factor}
        per = {}
        for i, r in enumerate(ours):
            name = PASS_ORDER[i % len(PASS_ORDER)]
            per.setdefault(name, {"kernel": r["Kernel_Name"], "vals": []})["vals"].append(
                float(r["Counter_Value"]) * 1024.0)
        for name, d in per.items():
            e = out["passes"].setdefault(name, {"kernel": d["kernel"]})
            key = "fetch" if counter == "FETCH_SIZE" else "write"
            raw = statistics.mean(d["vals"])
            e[key + "_raw_bytes"] = raw  # the counter as read, KiB x 1024
            e[key + "_bytes"] = raw * (factor or 1.0)  # scaled by the copy probe's factor
            e["dispatches"] = len(d["vals"])
    for e in out["passes"].values():
        e["hbm_bytes"] = e.get("fetch_bytes", 0.0) + e.get("write_bytes", 0.0)
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(traffic_path(n), "w") as f:
        json.dump(out, f, indent=1)
    lines = [f"HBM traffic per launch, {n}^3 FP32 R2C+C2R (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by k_copy)",
             f"commands: {commands}",
             f"copy probe: {COPY_BYTES(n)} B read and written per dispatch; "
             f"scale FETCH {out['FETCH_SIZE']['scale']}, WRITE {out['WRITE_SIZE']['scale']}",
             "the scales are measured on the copy probe alone (16-byte loads and stores of whole lines); the",
             "raw counter values are listed beside the scaled ones",
             f"{'pass':<12} {'fetch raw':>9} {'write raw':>9} {'fetch GB':>9} {'write GB':>9} {'total GB':>9}  kernel"]
    for name in PASS_ORDER:
        e = out["passes"].get(name)
        if e:
            lines.append(f"{name:<12} {e.get('fetch_raw_bytes', 0) / 1e9:9.3f} {e.get('write_raw_bytes', 0) / 1e9:9.3f} "
                         f"{e.get('fetch_bytes', 0) / 1e9:9.3f} {e.get('write_bytes', 0) / 1e9:9.3f} "
                         f"{e['hbm_bytes'] / 1e9:9.3f}  {e['kernel']}")
    with open(traffic_path(n).replace(".json", ".txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def COPY_BYTES(n: int) -> int:
    """Bytes the copy probe moves each way: the n^3 float32 real array."""
    return 4 * n ** 3


def forward_errors(pairs):
    """Part of the CPU-baseline leg: relative L2 error of GPU forward outputs (STRIDE1 Z-pencils) against
    the FP64 oracle's forward transform of the same real inputs; pairs: {name: (input, output)}."""
    import oracle

    errs = {}
    for name, (u, got) in pairs.items():
        ref = oracle.to_stride1(oracle.r2c3d(u))
        errs[name] = float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))
    return errs


def cpu_baseline(n: int, u=None, forward_outputs=None):
    """The oracle, untuned, on one forward+backward pair of an n^3 GRF (the benchmark's own input if given).

    forward_outputs: {name: host array [nxh][ny][nz]} of GPU forward results on
    the same input; their relative L2 error against the oracle's FP64 forward
    is returned next to the timing.
    """
    import oracle
    import synth

    if u is None or u.shape != (n, n, n):
        u = synth.grf(3, (n, n, n))
    t0 = time.perf_counter()
    U = oracle.r2c3d(u)
    oracle.c2r3d(U, n)
    dt = time.perf_counter() - t0
    N = float(n) ** 3
    errs = {}
    shells = {}
    # |k| shells [1, 2), [2, 4), ... [n/2, inf): the power-law input puts most of
    # the energy at low |k|, so the global error hides the high-|k| one (mode 0
    # of the input is zero by construction and is left out of the shells)
    edges = [2.0 ** j for j in range(0, int(math.log2(n)))] + [math.inf]
    kyz = np.fft.fftfreq(n, 1.0 / n)
    k2_yz = kyz[:, None] ** 2 + kyz[None, :] ** 2  # [ky][kz]
    for name, got in (forward_outputs or {}).items():
        if got is None or got.shape != (U.shape[2], U.shape[1], U.shape[0]):
            continue
        num = np.zeros(len(edges) - 1)
        den = np.zeros(len(edges) - 1)
        tot_num = tot_den = 0.0
        for kx in range(got.shape[0]):  # plane by plane: got[kx] is [ky][kz], U[:, :, kx] is [kz][ky]
            ref = U[:, :, kx].T
            e2 = np.abs(got[kx].astype(np.complex128) - ref) ** 2
            r2 = np.abs(ref) ** 2
            tot_num += float(e2.sum())
            tot_den += float(r2.sum())
            b = (np.digitize(np.sqrt(kx * kx + k2_yz), edges) - 1).ravel()
            ok = b >= 0
            num += np.bincount(b[ok], weights=e2.ravel()[ok], minlength=len(num))[:len(num)]
            den += np.bincount(b[ok], weights=r2.ravel()[ok], minlength=len(den))[:len(den)]
        errs[name] = math.sqrt(tot_num / tot_den)
        shells[name] = [{"k_lo": edges[i], "k_hi": edges[i + 1] if math.isfinite(edges[i + 1]) else None,
                         "rel_l2": math.sqrt(num[i] / den[i]) if den[i] > 0 else None}
                        for i in range(len(num))]
    errs["_shells"] = shells
    return {
        "value": 5.0 * N * math.log2(N) / dt / 1e9,
        "unit": "GFLOP/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"one R2C+C2R pair at {n}^3 (FP64, OpenMP over lines), {dt:.2f} s wall",
        "nproc": os.cpu_count(),
        "cpus_allowed": len(os.sched_getaffinity(0)),
        "one_core": cpu_baseline_one_core(min(n, 384)),
    }, errs


ONE_CORE_SCRIPT = """
import json, math, sys, time
sys.path.insert(0, sys.argv[1])
import oracle, synth
n = int(sys.argv[2])
u = synth.grf(2, (n, n, n))
t0 = time.perf_counter()
U = oracle.r2c3d(u)
oracle.c2r3d(U, n)
dt = time.perf_counter() - t0
N = float(n) ** 3
print(json.dumps({"value": 5.0 * N * math.log2(N) / dt / 1e9, "unit": "GFLOP/s", "cores": oracle.num_threads(),
                  "kind": "oracle", "sample": f"one R2C+C2R pair at {n}^3 (FP64), {dt:.2f} s wall"}))
"""


def cpu_baseline_one_core(n: int):
    """The same oracle on one host thread (OMP_NUM_THREADS=1, a child process that touches no GPU), on one
    pair of an n^3 GRF (n = 384: about 10 s)."""
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", ONE_CORE_SCRIPT, ROOT, str(n)], env=env, capture_output=True,
                       text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def other_grid_timings(pf, args, dev, stream):
    """The other FP32 grids of the plain path (STRIDE1, out-of-place, uniform[-1, 1] data): 512^3, all on
    the power-of-two kernels, and the uneven 480 x 360 x 250, all on the compile-time mixed-radix ones: ms
    per pair, GFLOP/s and algorithmic HBM GB/s; then, in a second timed loop with events between the
    passes, each pass's kernel family, average ms and algorithmic GB/s."""
    import torch

    out = {}
    g = torch.Generator(device=dev)
    g.manual_seed(2)
    for nx, ny, nz in ((512, 512, 512), (480, 360, 250)):
        plan = pf.Plan(nx, ny, nz, pf.Layout())
        u = torch.empty((nz, ny, nx), device=dev, dtype=torch.float32).uniform_(-1.0, 1.0, generator=g)
        U = plan.empty_complex(dev)
        r = plan.empty_real(dev)
        for _ in range(args.warmup):
            plan.ftran(u, U)
            plan.btran(U, r)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            plan.ftran(u, U)
            plan.btran(U, r)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        N = float(nx) * ny * nz
        nbytes = sum(plan.pass_bytes(d, i) for d in (pf.PF_DIR_FORWARD, pf.PF_DIR_BACKWARD)
                     for i in range(plan.num_passes(d)))
        rec = {"ms_per_pair": ms, "gflops": 5.0 * N * math.log2(N) / (ms * 1e-3) / 1e9,
               "alg_GBps": nbytes / (ms * 1e-3) / 1e9}
        plan.set_timing(True)
        for _ in range(args.steps):
            plan.ftran(u, U)
            plan.btran(U, r)
        torch.cuda.synchronize()
        passes = []
        for d in (pf.PF_DIR_FORWARD, pf.PF_DIR_BACKWARD):
            for i in range(plan.num_passes(d)):
                tot, cnt = plan.get_timing(d, i)
                pms = tot / max(cnt, 1)
                passes.append({"pass": plan.pass_name(d, i), "kernel": plan.pass_kernel(d, i), "avg_ms": pms,
                               "alg_GBps": plan.pass_bytes(d, i) / (pms * 1e-3) / 1e9})
        plan.set_timing(False)
        rec["passes"] = passes
        # the intermediate between the passes of each direction: blocked rows or the transposed workspace
        rec["workspace_layout"] = {dn: ("transposed" if plan.workspace_layout(d) == pf.PF_WS_TRANSPOSED else "blocked")
                                   for d, dn in ((pf.PF_DIR_FORWARD, "fwd"), (pf.PF_DIR_BACKWARD, "bwd"))}
        out[f"{nx}x{ny}x{nz}"] = rec
        plan.destroy()
    return out


def fused_timing(pf, nx, ny, nz, args, dev, stream, u, plain_passes):
    """The slab form (pf_layout.fused_xy): X and Y stages in one persistent pass per direction.  Pair time,
    per-pass times, and the fused pass's bandwidth under two accountings: its own algorithmic bytes (the
    real array and the complex array once each, what a two-pass transform must move) and the bytes the
    separate X and Y passes move (the three-pass accounting)."""
    import torch

    plan = pf.Plan(nx, ny, nz, pf.Layout(fused_xy=1))
    U = plan.empty_complex(dev)
    r = plan.empty_real(dev)
    for _ in range(args.warmup):
        plan.ftran(u, U)
        plan.btran(U, r)
    plan.set_timing(True)
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s0.record(stream)
    for _ in range(args.steps):
        plan.ftran(u, U)
        plan.btran(U, r)
    s1.record(stream)
    torch.cuda.synchronize()
    pf.pf_check_status(plan.handle)
    three = {p["pass"]: p["alg_bytes"] for p in plain_passes}
    out = {"ms_per_step": s0.elapsed_time(s1) / args.steps, "passes": []}
    for d in (pf.PF_DIR_FORWARD, pf.PF_DIR_BACKWARD):
        for i in range(plan.num_passes(d)):
            tot, cnt = plan.get_timing(d, i)
            avg = tot / max(cnt, 1)
            name = plan.pass_name(d, i)
            e = {"pass": name, "avg_ms": avg, "alg_bytes": plan.pass_bytes(d, i)}
            e["alg_GBps"] = e["alg_bytes"] / (avg * 1e-3) / 1e9
            if "fused" in name:
                sep = three["fwd_x_r2c"] + three["fwd_y_c2c"] if d == 0 else three["bwd_y_c2c"] + three["bwd_x_c2r"]
                e["three_pass_bytes"] = sep
                e["three_pass_GBps"] = sep / (avg * 1e-3) / 1e9
            out["passes"].append(e)
    plan.set_timing(False)
    plan.destroy()
    return out


def fused_compare_timing(pf, args, dev, stream, nx=2048, ny=512, nz=512):
    """Pair times of the three-pass and the fused X-Y plans on a grid whose X pass (2048-point lines)
    outweighs its Y pass.  Runs last: the trace summary splits on its first launch."""
    import torch

    u = torch.empty((nz, ny, nx), device=dev, dtype=torch.float32).uniform_(-1.0, 1.0)
    out = {"grid": [nx, ny, nz]}
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    for name, lay in (("three_pass_ms", pf.Layout()), ("fused_ms", pf.Layout(fused_xy=1))):
        plan = pf.Plan(nx, ny, nz, lay)
        U = plan.empty_complex(dev)
        r = plan.empty_real(dev)
        for _ in range(args.warmup):
            plan.ftran(u, U)
            plan.btran(U, r)
        torch.cuda.synchronize()
        s0.record(stream)
        for _ in range(args.steps):
            plan.ftran(u, U)
            plan.btran(U, r)
        s1.record(stream)
        torch.cuda.synchronize()
        pf.pf_check_status(plan.handle)
        out[name] = s0.elapsed_time(s1) / args.steps
        plan.destroy()
    return out


def f64_timing(pf, args, dev, stream, n=512, check=True):
    """FP64 R2C+C2R at n^3 (uniform[-1, 1] data, STRIDE1, out-of-place; the paper's runs are double
    precision): ms per pair, GFLOP/s, per-pass algorithmic GB/s and fraction of 8 TB/s, and the forward
    relative L2 error against the FP64 oracle."""
    import torch

    plan = pf.Plan(n, n, n, pf.Layout(precision=pf.PF_F64))
    g = torch.Generator(device=dev)
    g.manual_seed(64)
    u = torch.empty((n, n, n), device=dev, dtype=torch.float64).uniform_(-1.0, 1.0, generator=g)
    U = plan.empty_complex(dev)
    r = plan.empty_real(dev)
    for _ in range(args.warmup):
        plan.ftran(u, U)
        plan.btran(U, r)
    plan.set_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        plan.ftran(u, U)
        plan.btran(U, r)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    N = float(n) ** 3
    passes, nbytes = [], 0.0
    for d in (pf.PF_DIR_FORWARD, pf.PF_DIR_BACKWARD):
        for i in range(plan.num_passes(d)):
            tot, cnt = plan.get_timing(d, i)
            avg = tot / max(cnt, 1)
            b = plan.pass_bytes(d, i)
            nbytes += b
            gbs = b / (avg * 1e-3) / 1e9
            passes.append({"pass": plan.pass_name(d, i), "avg_ms": avg, "alg_GBps": gbs,
                           "frac_of_peak": gbs / HBM_PEAK_GBS})
    plan.set_timing(False)
    out = {"grid": [n, n, n], "precision": "f64", "ms_per_pair": ms,
           "gflops": 5.0 * N * math.log2(N) / (ms * 1e-3) / 1e9, "alg_GBps": nbytes / (ms * 1e-3) / 1e9,
           "frac_of_peak": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "passes": passes}
    rt = (torch.linalg.vector_norm(r / N - u) / torch.linalg.vector_norm(u)).item()
    out["round_trip_rel_l2"] = rt
    if check:  # host copies of the input and forward output, compared in the CPU-baseline leg
        plan.ftran(u, U)
        torch.cuda.synchronize()
        out["_check"] = {"512^3": (u.cpu().numpy(), U.cpu().numpy())}
    plan.destroy()
    return out


def layout_timings(pf, nx, ny, nz, args, dev, stream, u):
    """Pair time and per-pass times of the layout variants off the measured one:
    Z-pencil without STRIDE1, in-place, and the empty third transform."""
    import torch

    out = {}
    for name, lay in (("stride1_undefined", pf.Layout(stride1=0)),
                      ("inplace", pf.Layout(inplace=1)),
                      ("third_empty", pf.Layout(third=pf.PF_THIRD_EMPTY))):
        plan = pf.Plan(nx, ny, nz, lay)
        nb = max(nx * ny * nz * 4, (nx // 2 + 1) * ny * nz * 8)
        if lay.inplace:
            buf = torch.empty(nb // 4, dtype=torch.float32, device=dev)

            def step():
                buf[: u.numel()].copy_(u.reshape(-1))  # the input is consumed in place
                pf.pf_ftran_r2c(plan.handle, buf.data_ptr(), buf.data_ptr(), stream.cuda_stream)
                pf.pf_btran_c2r(plan.handle, buf.data_ptr(), buf.data_ptr(), stream.cuda_stream)
        else:
            U = plan.empty_complex(dev)
            r = plan.empty_real(dev)

            def step():
                plan.ftran(u, U)
                plan.btran(U, r)
        for _ in range(args.warmup):
            step()
        plan.set_timing(True)
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s0.record(stream)
        for _ in range(args.steps):
            step()
        s1.record(stream)
        torch.cuda.synchronize()
        passes = {}
        for d in (pf.PF_DIR_FORWARD, pf.PF_DIR_BACKWARD):
            for i in range(plan.num_passes(d)):
                tot, cnt = plan.get_timing(d, i)
                passes[plan.pass_name(d, i)] = tot / max(cnt, 1)
        plan.set_timing(False)
        out[name] = {"ms_per_step": s0.elapsed_time(s1) / args.steps, "pass_ms": passes}
        if lay.inplace:
            out[name]["note"] = "includes one device copy of the input per step (the input is overwritten)"
        plan.destroy()
    return out


def batch_timing(pf, args, dev, stream, count=64, seed=4, check=True):
    """64 independent R2C+C2R FP32 transforms of 7-smooth sizes in [48, 320] (uniform[-1, 1] data):
    ms per batch pair in each execution mode, default and autotuned plans, and the forward error of a
    sample of transforms against the FP64 oracle."""
    import torch

    import synth
    from paper_1905_02803_amd import autotune

    dims = synth.batch_sizes(seed, count)
    Ns = [float(nx) * ny * nz for nx, ny, nz in dims]
    flops = sum(5.0 * N * math.log2(N) for N in Ns)
    nbytes = sum(2 * (N * 4 + (nx // 2 + 1) * ny * nz * 8) + 8 * (nx // 2 + 1) * ny * nz * 8
                 for N, (nx, ny, nz) in zip(Ns, dims))  # both directions: X, Y, Z passes
    serial_modes = (("serial", pf.PF_BATCH_SERIAL), ("serial_graph", pf.PF_BATCH_SERIAL | pf.PF_BATCH_GRAPH),
                    ("serial_streams", pf.PF_BATCH_SERIAL | pf.PF_BATCH_STREAMS))
    fused_modes = (("fused", pf.PF_BATCH_FUSED), ("fused_graph", pf.PF_BATCH_FUSED | pf.PF_BATCH_GRAPH),
                   ("fused_streams", pf.PF_BATCH_FUSED | pf.PF_BATCH_STREAMS))
    # the cached plans of each mode: radix orders and tiles (serial), radix orders alone (fused)
    runs = (("default", None, serial_modes + fused_modes),
            ("tuned", autotune.tune_for(dims, mode="serial"), serial_modes),
            ("tuned", autotune.tune_for(dims, mode="fused"), fused_modes))
    out = {"count": count, "sizes": f"synth.batch_sizes({seed}, {count}): 7-smooth, each dimension in [48, 320]",
           "points": sum(Ns), "gflop_per_pair": flops / 1e9, "alg_bytes_per_pair": nbytes, "modes": {}}
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    for tname, tune, modes in runs:
        if tname == "tuned" and tune is None:
            out["modes"]["tuned_" + modes[0][0]] = "no cached plans for these sizes"
            continue
        b = pf.Batch(dims, tune=tune)
        R = b.empty(0).zero_()
        C = b.empty(1).zero_()
        R2 = b.empty(0)
        for i in range(count):
            v = b.view(R, 0, i)
            v.copy_(torch.rand(v.shape, generator=g, device=dev) * 2 - 1)
        for mname, mode in modes:
            b.set_mode(mode)
            for _ in range(args.warmup):
                b.ftran(R, C)
                b.btran(C, R2)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(args.steps):
                b.ftran(R, C)
                b.btran(C, R2)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            out["modes"][f"{tname}_{mname}"] = {"ms_per_pair": ms, "gflops": flops / (ms * 1e-3) / 1e9,
                                                "alg_GBps": nbytes / (ms * 1e-3) / 1e9,
                                                "transforms_per_s": count / (ms * 1e-3)}
        if check and tname == "default":  # host copies of a sample, compared in the CPU-baseline leg
            b.set_mode(pf.PF_BATCH_FUSED)
            b.ftran(R, C)
            torch.cuda.synchronize()
            out["_check"] = {"x".join(map(str, dims[i])): (b.view(R, 0, i).cpu().numpy(), b.view(C, 1, i).cpu().numpy())
                             for i in sorted(set([0, 1, 2, int(max(range(count), key=lambda j: Ns[j]))]))}
        b.destroy()
    return out


def spectral_timing(pf, args, dev, stream, nx=512, ny=512, nz=257):
    """The differentiable spectral step on the 512 x 512 x 257 Chebyshev grid (FP32): L u, L^T g and one
    autograd forward + backward; per-pass times of the plan's transforms (the type-I DCT runs as the generic
    kernel on the even extension, length 2 (nz - 1) = 512)."""
    import torch

    plan = pf.Plan(nx, ny, nz, pf.Layout(third=pf.PF_THIRD_CHEB))
    u = (torch.rand((nz, ny, nx), generator=torch.Generator(device=dev).manual_seed(5), device=dev) * 2 - 1)
    spec = plan.empty_complex(dev)
    out = {"grid": [nx, ny, nz], "third": "type-I DCT (Chebyshev) along z"}

    def timeit(fn):
        for _ in range(args.warmup):
            fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    out["ms_step"] = timeit(lambda: pf.spectral_step(plan, u, spec))
    out["ms_adjoint"] = timeit(lambda: pf.spectral_step(plan, u, spec, adjoint=True))
    ug = u.clone().requires_grad_(True)

    def fb():
        ug.grad = None
        pf.spectral_step_autograd(ug, plan).sum().backward()

    out["ms_autograd_fwd_bwd"] = timeit(fb)
    U = plan.empty_complex(dev)
    r = plan.empty_real(dev)
    for _ in range(args.warmup):
        plan.ftran(u, U)
        plan.btran(U, r)
    plan.set_timing(True)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        plan.ftran(u, U)
        plan.btran(U, r)
    torch.cuda.synchronize()
    passes = []
    for d in (pf.PF_DIR_FORWARD, pf.PF_DIR_BACKWARD):
        for i in range(plan.num_passes(d)):
            tot, cnt = plan.get_timing(d, i)
            avg = tot / max(cnt, 1)
            nbytes = plan.pass_bytes(d, i)
            passes.append({"pass": plan.pass_name(d, i), "avg_ms": avg, "alg_GBps": nbytes / (avg * 1e-3) / 1e9})
    plan.set_timing(False)
    out["passes"] = passes
    plan.destroy()
    return out


def share_only_timing(pf, nx, ny, nz, args, dev, stream, m2=8, r2=3):
    """One rank's share of the grid on a 1 x m2 slab grid (share-only plan): per-pass times."""
    import torch

    lay = pf.Layout(precision=pf.PF_F32, stride1=1, m1=1, m2=m2, share_only=1, r1=0, r2=r2)
    plan = pf.Plan(nx, ny, nz, lay)
    ub = torch.randn(plan.real_shape, dtype=torch.float32, device=dev)
    Ub = plan.empty_complex(dev)
    rb = plan.empty_real(dev)
    for _ in range(args.warmup):
        plan.ftran(ub, Ub)
        plan.btran(Ub, rb)
    plan.set_timing(True)
    s0 = torch.cuda.Event(enable_timing=True)
    s1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s0.record(stream)
    for _ in range(args.steps):
        plan.ftran(ub, Ub)
        plan.btran(Ub, rb)
    s1.record(stream)
    torch.cuda.synchronize()
    passes = []
    for d in (pf.PF_DIR_FORWARD, pf.PF_DIR_BACKWARD):
        for i in range(plan.num_passes(d)):
            tot, cnt = plan.get_timing(d, i)
            avg = tot / max(cnt, 1)
            nbytes = plan.pass_bytes(d, i)
            passes.append({"pass": plan.pass_name(d, i), "avg_ms": avg, "alg_bytes": nbytes,
                           "alg_GBps": nbytes / (avg * 1e-3) / 1e9 if avg > 0 else None})
    plan.set_timing(False)
    out = {"grid": f"1x{m2}", "rank": [0, r2], "x_pencil": list(plan.real_shape),
           "z_pencil": list(plan.complex_shape), "ms_per_step": s0.elapsed_time(s1) / args.steps,
           "passes": passes}
    plan.destroy()
    return out


def main():
    args = parse()
    if args.kt_summary:
        summarize_trace(args.kt_summary[0], args.kt_summary[1], args.steps, args.warmup)
        return
    if args.pmc_summary:
        summarize_pmc(args.pmc_summary[0], args.pmc_summary[1], args.n, args.pmc_commands)
        return
    if args.sq_summary:
        summarize_sq(args.sq_summary[0], args.sq_summary[1])
        return
    if args.mfma_summary:
        summarize_mfma(args.mfma_summary[0], args.mfma_summary[1])
        return
    if args.mfma_workload:
        mfma_workload(args.n, args.steps)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is a design "
              "note, not built", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1905_02803_amd as pf
    import synth

    n = args.n
    nx = ny = nz = n
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    u_host = synth.grf(3, (nz, ny, nx))
    plan = pf.Plan(nx, ny, nz, pf.Layout(precision=pf.PF_F32, stride1=1))
    u = torch.from_numpy(u_host).to(dev)
    U = plan.empty_complex(dev)
    r = plan.empty_real(dev)
    stream = torch.cuda.current_stream()

    def step():
        plan.ftran(u, U)
        plan.btran(U, r)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # round-trip error of the last warm-up step (GPU only): ||btran(ftran u)/N - u|| / ||u||
    Nf = float(nx) * ny * nz
    rt_err = (torch.linalg.vector_norm((r.double() / Nf - u.double())) / torch.linalg.vector_norm(u.double())).item()

    # HBM ceilings: copies of the real array (the same bytes in and out as one pass of it) in the
    # passes' access shapes -- the one-shot copy, 128 KB tiles between two arrays (the X and Z passes),
    # 128 KB tiles in place (the Y pass)
    probes = {}
    for pname, kind, dst in (("copy", pf.PF_PROBE_COPY, r), ("tiles", pf.PF_PROBE_TILES, r),
                             ("tiles_inplace", pf.PF_PROBE_TILES_INPLACE, u)):
        copy_reps = 5
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        pf.pf_probe(kind, dst.data_ptr(), u.data_ptr(), COPY_BYTES(n), stream.cuda_stream)
        c0.record(stream)
        for _ in range(copy_reps):
            pf.pf_probe(kind, dst.data_ptr(), u.data_ptr(), COPY_BYTES(n), stream.cuda_stream)
        c1.record(stream)
        torch.cuda.synchronize()
        probes[pname] = 2.0 * COPY_BYTES(n) / (c0.elapsed_time(c1) / copy_reps * 1e-3) / 1e9
    copy_GBps = probes["copy"]

    plan.set_timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    marks[0].record(stream)
    for i in range(args.steps):
        step()
        marks[i + 1].record(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    step_ms = [marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps)]

    passes = []
    for d, dname in ((pf.PF_DIR_FORWARD, "fwd"), (pf.PF_DIR_BACKWARD, "bwd")):
        for i in range(plan.num_passes(d)):
            tot, cnt = plan.get_timing(d, i)
            avg = tot / max(cnt, 1)
            nbytes = plan.pass_bytes(d, i)
            passes.append({"pass": plan.pass_name(d, i), "avg_ms": avg, "launches": cnt,
                           "alg_bytes": nbytes, "alg_GBps": nbytes / (avg * 1e-3) / 1e9 if avg > 0 else None})
    plan.set_timing(False)
    for p_ in passes:  # against the probe of the pass's own access shape
        own = probes["tiles_inplace"] if "_y_" in p_["pass"] else probes["tiles"]
        p_["frac_of_own_probe"] = p_["alg_GBps"] / own if p_["alg_GBps"] else None
    dom = max(passes, key=lambda p: p["avg_ms"])
    keep_host = not args.no_cpu_baseline
    fwd_host = {"plain": U.cpu().numpy() if keep_host else None}

    # the matrix-core precision variants on the same input, same protocol
    mfma = {}
    for name, mth in (("fp16x2", pf.PF_MFMA_FP16X2), ("bf16x2", pf.PF_MFMA_BF16X2)):
        pm = pf.Plan(nx, ny, nz, pf.Layout(precision=pf.PF_F32, stride1=1, math=mth))
        Um = pm.empty_complex(dev)
        for _ in range(args.warmup):
            pm.ftran(u, Um)
            pm.btran(Um, r)
        torch.cuda.synchronize()
        m0 = torch.cuda.Event(enable_timing=True)
        m1 = torch.cuda.Event(enable_timing=True)
        m0.record(stream)
        for _ in range(args.steps):
            pm.ftran(u, Um)
            pm.btran(Um, r)
        m1.record(stream)
        torch.cuda.synchronize()
        mms = m0.elapsed_time(m1) / args.steps
        mfma[name] = {"ms_per_step": mms, "value": 5.0 * Nf * math.log2(Nf) / (mms * 1e-3) / 1e9,
                      "speedup_vs_plain": ms / mms}
        pm.ftran(u, Um)
        torch.cuda.synchronize()
        if keep_host:
            fwd_host[name] = Um.cpu().numpy()
        del Um
        pm.destroy()
    def step(name):  # a progress line per section, on stderr (the JSON line is the only stdout)
        print(f"bench: {name}", file=sys.stderr, flush=True)

    step("fused X-Y plan")
    fused = fused_timing(pf, nx, ny, nz, args, dev, stream, u, passes)
    step("layout variants")
    layouts = layout_timings(pf, nx, ny, nz, args, dev, stream, u)
    step("batch")
    batched = batch_timing(pf, args, dev, stream, check=not args.no_cpu_baseline)
    step("spectral step")
    spectral = spectral_timing(pf, args, dev, stream)
    step("share-only rank")
    share = share_only_timing(pf, nx, ny, nz, args, dev, stream)
    step("FP64 512^3")
    f64 = f64_timing(pf, args, dev, stream, check=not args.no_cpu_baseline)
    step("other grids")
    other_grids = other_grid_timings(pf, args, dev, stream)  # the trace summary splits on its first launch
    step("fused X-Y against three passes at 2048 x 512 x 512")
    fused_cmp = fused_compare_timing(pf, args, dev, stream)  # last, likewise
    flops = 5.0 * Nf * math.log2(Nf)
    alg_bytes = sum(p["alg_bytes"] for p in passes)
    gflops = flops / (ms * 1e-3) / 1e9

    cpu = None
    errs = {}
    f64_check, batch_check = f64.pop("_check", None), batched.pop("_check", None)
    if not args.no_cpu_baseline:  # the CPU-baseline leg: the oracle's timing and every oracle comparison
        cpu, errs = cpu_baseline(min(args.cpu_n, n), u_host, fwd_host)
        if f64_check:
            f64["rel_l2_fwd_vs_fp64_oracle"] = forward_errors(f64_check)["512^3"]
        if batch_check:
            batched["rel_l2_fwd_vs_fp64_oracle"] = forward_errors(batch_check)
    del u_host, fwd_host, f64_check, batch_check
    for name in mfma:
        mfma[name]["rel_l2_fwd_vs_fp64_oracle"] = errs.get(name)

    out = {
        "metric": "3D R2C+C2R GFLOP/s & HBM GB/s at 1024^3; MFMA-mixed vs FP32 at stated err",
        "value": gflops,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3D R2C+C2R FP32 {nx}x{ny}x{nz}, GRF |k|^-5/3, STRIDE1, out-of-place",
                   "grid": [nx, ny, nz], "precision": "f32", "math": "plain", "layout": "1x1"},
        "hbm_GBps_alg": alg_bytes / (ms * 1e-3) / 1e9,
        "copy_probe_GBps": copy_GBps,
        "probes_GBps": probes,
        "ms_per_step_median": statistics.median(step_ms),
        "ms_per_step_min": min(step_ms),
        "round_trip_rel_l2": rt_err,
        "rel_l2_fwd_vs_fp64_oracle": errs.get("plain"),
        "rel_l2_fwd_by_k_shell": errs.get("_shells", {}).get("plain"),
        "mfma": mfma,
        "roofline": {
            "bound": "hbm",
            "kernel": dom["pass"],
            "achieved": dom["alg_GBps"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom["alg_GBps"] / HBM_PEAK_GBS,
            "frac_of_copy_probe": dom["alg_GBps"] / copy_GBps,
            "frac_of_own_probe": dom["frac_of_own_probe"],
            "traffic": traffic_from_profile(dom["pass"], n),
        },
        "passes": passes,
        "fused_xy": fused,
        "share_only": share,
        "layouts": layouts,
        "other_grids": other_grids,
        "fused_xy_2048x512x512": fused_cmp,
        "f64_512cubed": f64,
        "batched": batched,
        "spectral_step": spectral,
        "cpu_baseline": cpu,
        "wall_s_timed": wall,
    }
    plan.destroy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
