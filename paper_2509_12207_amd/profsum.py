"""Summarise a rocprofv3 CSV output directory into a short markdown report.

    python -m paper_2509_12207_amd.profsum <rocprof dir> --kernel <regex> \
        --last N [--skip S] [--title T] [--command C] [--pmc] > summary.md

Reports the top kernels by total time (the --stats view: calls, total, mean)
and, for the kernel matching --kernel, the mean duration of its last N
dispatches excluding the final S ... i.e. the dispatches of a timed leg that
runs after everything else (e.g. the roofline leg of bench.py).  With --pmc
the counter columns (FETCH_SIZE, WRITE_SIZE, ...) of those same dispatches
are averaged too.

    python -m paper_2509_12207_amd.profsum --traffic <FETCH_SIZE dir> \
        <WRITE_SIZE dir> <roofline-only json> > profiles/traffic.json

builds the per-kernel HBM traffic table that bench.py reports: for every
kernel of the roofline leg, FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of
its timed launches, each scaled to bytes by what the same counter reads for
the leg's 1 GiB device-to-device copy, next to the kernel's algorithmic bytes
and the hash of its source file (a changed source invalidates the entry).

    python -m paper_2509_12207_amd.profsum --sq <pass dir> [<pass dir> ...] > table.md

tabulates SQ / GRBM counters of the roofline leg's kernels (mean per
dispatch over each kernel's last 5 dispatches, from every pass directory)
with two derived columns: MFMA busy, SQ_VALU_MFMA_BUSY_CYCLES over the
SIMD-cycles of the dispatch (1024 SIMDs; GRBM_GUI_ACTIVE summed over the
eight XCDs, so / 8 gives the dispatch's cycles), and the waves' waiting
share, SQ_WAIT_ANY / SQ_WAVE_CYCLES.
"""

import argparse
import csv
import glob
import os
import re
import sys


def _rows(d, pattern):
    out = []
    for path in sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True)):
        with open(path, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def _dur(r):
    return int(r["End_Timestamp"]) - int(r["Start_Timestamp"])


# roofline-leg op -> (kernel-name regex, dispatches per launch, source file)
TRAFFIC_KERNELS = {
    "gemm": (r"gemm_f32_kernel<2, 2, 2, 2, 1, true>", 1,
             "paper_2509_12207_amd/csrc/kernels/gemm_f32.hip"),
    "conv3x3": (r"conv3x3_f32_kernel<2, 2, 2, 2, 1, 8, 16>", 1,
                "paper_2509_12207_amd/csrc/kernels/conv3x3_f32.hip"),
    "bias_relu": (r"bias_relu_vec<0", 1, "paper_2509_12207_amd/csrc/kernels/pointwise.hip"),
    "rowsum": (r"rowsum_block", 1, "paper_2509_12207_amd/csrc/kernels/pointwise.hip"),
    "softmax": (r"softmax_reg<4, 4, ", 1, "paper_2509_12207_amd/csrc/kernels/pointwise.hip"),
    "voxel": (r"voxel_(init|scatter|finalize|bin|tile_reduce|merge)", 3,
              "paper_2509_12207_amd/csrc/kernels/voxel.hip"),
    "gemm_fp8": (r"gemm_fp8_kernel|gemm_ring<0, false>", 1,
                 "paper_2509_12207_amd/csrc/kernels/gemm_lowp.hip"),
    "gemm_bf16": (r"gemm_ring<1, false>", 1, "paper_2509_12207_amd/csrc/kernels/gemm_lowp.hip"),
    "conv3x3_bf16": (r"gemm_ring<1, true>", 1, "paper_2509_12207_amd/csrc/kernels/gemm_lowp.hip"),
}


def _counter_per_dispatch(d, name):
    """[(kernel name, value)] in dispatch order for counter ``name``."""
    rows = _rows(d, "*counter_collection.csv")
    by = {}
    for r in rows:
        if r["Counter_Name"] == name:
            k = int(r["Dispatch_Id"])
            nm, v = by.get(k, (r["Kernel_Name"], 0.0))
            by[k] = (nm, v + float(r["Counter_Value"]))
    return [by[k] for k in sorted(by)]


def traffic(fetch_dir, write_dir, roof_json, root):
    import hashlib
    import json
    roof = None
    for line in open(roof_json):
        if line.startswith("{"):
            roof = json.loads(line)
    recs = {r["kernel"]: r for r in roof["kernels"]}
    fetch = _counter_per_dispatch(fetch_dir, "FETCH_SIZE")
    write = _counter_per_dispatch(write_dir, "WRITE_SIZE")
    copy_kib = roof["copy_bytes_each_way"] / 1024.0
    copies_f = [v for n, v in fetch if "copyBuffer" in n]
    copies_w = [v for n, v in write if "copyBuffer" in n]
    fs = copy_kib / (sum(copies_f[-3:]) / len(copies_f[-3:]))
    ws = copy_kib / (sum(copies_w[-3:]) / len(copies_w[-3:]))
    out = {"source": "rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, of `python3 bench.py "
                     "--roofline-only` (the timed launches of each kernel at its roofline "
                     "shape); scale factors from the run's 1 GiB device-to-device copy",
           "fetch_scale": round(fs, 4), "write_scale": round(ws, 4), "kernels": {}}
    for op, (rx, per, src) in TRAFFIC_KERNELS.items():
        if op not in recs:
            continue
        reps = recs[op]["reps"]
        pat = re.compile(rx)
        f = [v for n, v in fetch if pat.search(n)][-reps * per:]
        w = [v for n, v in write if pat.search(n)][-reps * per:]
        fk, wk = sum(f) / reps, sum(w) / reps
        sha = hashlib.sha256(open(os.path.join(root, src), "rb").read()).hexdigest()
        out["kernels"][op] = {
            "kernel_regex": rx, "dispatches_per_launch": per, "launches": reps,
            "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
            "traffic_bytes": int(round((fk * fs + wk * ws) * 1024)),
            "algorithmic_bytes": recs[op]["bytes"], "source_file": src, "source_sha256": sha}
    return out


SQ_KERNELS = [("voxel bin", r"voxel_bin"), ("voxel tile_reduce", r"voxel_tile_reduce"),
              ("FP32 GEMM 4096^3", r"gemm_f32_kernel<2, 2, 2, 2, 1, true>"),
              ("FP32 conv C256 256^2", r"conv3x3_f32_kernel<2, 2, 2, 2, 1, 8, 16>"),
              ("BF16 GEMM 4096^3", r"gemm_ring<1, false>"),
              ("BF16 conv C256 256^2", r"gemm_ring<1, true>"),
              ("FP8 GEMM 8192^3", r"gemm_ring<0, false>"),
              ("bias+ReLU 16384^2", r"bias_relu_vec<0")]


def sq_table(dirs, last=5):
    by = {}
    for d in dirs:
        rows = _rows(d, "*counter_collection.csv")
        for label, rx in SQ_KERNELS:
            pat = re.compile(rx)
            disp = {}
            for r in rows:
                if pat.search(r.get("Kernel_Name", "")):
                    disp.setdefault(int(r["Dispatch_Id"]), {}).setdefault(r["Counter_Name"], 0.0)
                    disp[int(r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
            tail = [disp[k] for k in sorted(disp)][-last:]
            for d_ in tail:
                for n, v in d_.items():
                    by.setdefault(label, {}).setdefault(n, []).append(v)
    names = sorted({n for v in by.values() for n in v})
    out = ["| kernel | MFMA busy | waves waiting | " + " | ".join(names) + " |",
           "|---|---|---|" + "---|" * len(names)]
    for label, _ in SQ_KERNELS:
        if label not in by:
            continue
        m = {n: sum(v) / len(v) for n, v in by[label].items()}
        cyc = m.get("GRBM_GUI_ACTIVE", 0) / 8
        busy = m.get("SQ_VALU_MFMA_BUSY_CYCLES", 0) / (1024 * cyc) if cyc else float("nan")
        wait = m.get("SQ_WAIT_ANY", 0) / m["SQ_WAVE_CYCLES"] if m.get("SQ_WAVE_CYCLES") else float("nan")
        out.append(f"| {label} | {busy:.2f} | {wait:.2f} | " +
                   " | ".join(f"{m[n]:.4g}" if n in m else "" for n in names) + " |")
    return "\n".join(out)


def main(argv=None):
    if argv is None:
        argv = sys.argv[1:]
    if argv and argv[0] == "--sq":
        print(sq_table(argv[1:]))
        return 0
    if argv and argv[0] == "--traffic":
        import json
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        print(json.dumps(traffic(argv[1], argv[2], argv[3], root), indent=1))
        return 0
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--kernel", required=True, help="regex selecting the timed kernel")
    ap.add_argument("--last", type=int, default=20)
    ap.add_argument("--skip", type=int, default=0, help="dispatches to drop from the end")
    ap.add_argument("--title", default="rocprofv3 summary")
    ap.add_argument("--command", default="")
    ap.add_argument("--top", type=int, default=12)
    ap.add_argument("--pmc", action="store_true", help="counter collection output")
    a = ap.parse_args(argv)

    pat = re.compile(a.kernel)
    if a.pmc:
        rows = _rows(a.dir, "*counter_collection.csv")
        sel = [r for r in rows if pat.search(r.get("Kernel_Name", ""))]
        by_disp = {}
        for r in sel:
            by_disp.setdefault(r["Dispatch_Id"], {})[r["Counter_Name"]] = float(r["Counter_Value"])
        disp = [by_disp[k] for k in sorted(by_disp, key=int)]
        tail = disp[len(disp) - a.last - a.skip: len(disp) - a.skip] if a.skip else disp[-a.last:]
        print(f"# {a.title}\n")
        if a.command:
            print(f"Command:\n\n```\n{a.command}\n```\n")
        print(f"Kernel regex `{a.kernel}`: {len(disp)} dispatches with counters; "
              f"mean over the last {len(tail)} (skipping {a.skip} at the end):\n")
        names = sorted({n for d in tail for n in d})
        print("| counter | mean per dispatch |\n|---|---|")
        for n in names:
            vals = [d[n] for d in tail if n in d]
            print(f"| {n} | {sum(vals) / len(vals):.1f} |")
        return 0

    rows = _rows(a.dir, "*kernel_trace.csv")
    if not rows:
        print(f"no kernel_trace.csv under {a.dir}", file=sys.stderr)
        return 1
    tot = {}
    for r in rows:
        k = r["Kernel_Name"]
        n, s = tot.get(k, (0, 0))
        tot[k] = (n + 1, s + _dur(r))
    grand = sum(s for _, s in tot.values())
    print(f"# {a.title}\n")
    if a.command:
        print(f"Command:\n\n```\n{a.command}\n```\n")
    print(f"{len(rows)} dispatches, {grand / 1e6:.1f} ms of kernel time.\n")
    print("| kernel | calls | total ms | mean us | share |\n|---|---|---|---|---|")
    for k, (n, s) in sorted(tot.items(), key=lambda kv: -kv[1][1])[: a.top]:
        short = k if len(k) < 110 else k[:107] + "..."
        print(f"| `{short}` | {n} | {s / 1e6:.2f} | {s / n / 1e3:.2f} | {s / grand:.3f} |")
    sel = sorted((r for r in rows if pat.search(r["Kernel_Name"])), key=lambda r: int(r["Start_Timestamp"]))
    tail = sel[len(sel) - a.last - a.skip: len(sel) - a.skip] if a.skip else sel[-a.last:]
    if tail:
        d = [_dur(r) for r in tail]
        g = tail[-1]
        grid = "x".join(g.get(f"Grid_Size_{c}", "?") for c in "XYZ")
        wg = "x".join(g.get(f"Workgroup_Size_{c}", "?") for c in "XYZ")
        print(f"\nTimed leg: kernel regex `{a.kernel}`, last {len(tail)} dispatches "
              f"(grid {grid}, workgroup {wg}): mean {sum(d) / len(d) / 1e3:.2f} us, "
              f"min {min(d) / 1e3:.2f} us, max {max(d) / 1e3:.2f} us.")
    return 0


if __name__ == "__main__":
    sys.exit(main())
