"""Tile-shape autotuner for the FP32 GEMM and 3x3 convolution launchers.

For every distinct (op, shape) of those two operations in the given
workloads, every tile variant of the launcher is timed on the GPU (HIP
events on one stream around `reps` back-to-back launches, median of
`rounds` such loops, after warm-up), and the fastest goes into a table
file that ``ug_tile_load`` / ``ug_config.tile_table`` reads: one line
"op M N K 0 variant" (GEMM) or "op N C H W variant" (convolution), with
the measured microseconds of every variant as a comment.  Ties within 2 %
keep the launcher's own rule (no entry), so the table only records
measured wins.

    python -m paper_2509_12207_amd.autotune --workloads cfg1:0 cfg1:1 cfg3:0 \\
        --out paper_2509_12207_amd/tiles_gfx950.txt
"""

import argparse
import os
import sys
import time

import numpy as np

from . import capi, synth

OPS = ("gemm", "conv3x3")


def workload_shapes(wl):
    """Distinct (op, shape) of the tunable operations in a workload (per-frame
    sizes at every size a frame may take are not enumerated: the registered
    shape stands for them)."""
    out = set()
    for ch in wl.chains:
        for t in ch.tasks:
            for k in t["kernels"]:
                if k["op"] in OPS:
                    out.add((k["op"], tuple(int(v) for v in k["shape"])))
    return sorted(out)


def _buffers(torch, op, shape):
    if op == "gemm":
        M, N, K = shape[:3]
        sizes = (M * K, K * N, M * N)
    else:
        n, c, h, w = shape
        sizes = (n * c * h * w, c * c * 9, n * c * h * w)
    return [torch.rand(s, device="cuda") * 2 - 1 for s in sizes]


def time_variants(torch, op, shape, reps=10, rounds=5):
    """Median microseconds per launch of every variant of (op, shape)."""
    k = {"op": op, "shape": shape, "in": (0, 1), "out": (2,)}
    bufs = _buffers(torch, op, shape)
    ptrs = [b.data_ptr() for b in bufs]
    s = torch.cuda.Stream()
    out = []
    for v in range(capi.tile_variants(op)):
        for _ in range(2):
            capi.kernel_launch_variant(k, ptrs, v, s.cuda_stream)
        ts = []
        for _ in range(rounds):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                capi.kernel_launch_variant(k, ptrs, v, s.cuda_stream)
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e3 / reps)
        out.append(float(np.median(ts)))
    del bufs
    return out


def rule_variant(op, shape):
    capi.tile_clear()
    return capi.tile_get({"op": op, "shape": shape, "in": (0, 1), "out": (2,)})


def tune(torch, shapes, margin=0.02, log=None):
    rows = []
    for i, (op, shape) in enumerate(shapes):
        us = time_variants(torch, op, shape)
        rule = rule_variant(op, shape)
        best = int(np.argmin(us))
        keep = us[best] < (1.0 - margin) * us[rule]
        rows.append({"op": op, "shape": shape, "us": us, "rule": rule,
                     "variant": best if keep else None})
        if log:
            log(f"[{i + 1}/{len(shapes)}] {op} {shape}: " + " ".join(f"{u:.1f}" for u in us)
                + f" us; rule {rule}, best {best}" + ("" if keep else " (kept the rule)"))
    return rows


def write_table(path, rows, header=""):
    with open(path, "w") as fh:
        fh.write("# tile-variant table for the FP32 GEMM and 3x3 convolution on gfx950,\n"
                 "# written by paper_2509_12207_amd.autotune: op s0 s1 s2 s3 variant\n"
                 "# (us per launch of every variant, and the launcher rule's choice)\n")
        if header:
            fh.write(f"# {header}\n")
        for r in rows:
            if r["variant"] is None:
                continue
            s = list(r["shape"]) + [0] * (4 - len(r["shape"]))
            fh.write(f"{capi.OP_IDS[r['op']]} {s[0]} {s[1]} {s[2]} {s[3]} {r['variant']}"
                     f"  # us {' '.join(f'{u:.1f}' for u in r['us'])}; rule {r['rule']}\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", nargs="+", default=["cfg1:0"],
                    help="workload:seed pairs (cfg1, cfg3)")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("the autotuner needs a GPU", file=sys.stderr)
        sys.exit(1)
    capi.lib()
    shapes = set()
    for spec in args.workloads:
        name, seed = spec.split(":")
        gen = {"cfg1": synth.config1, "cfg3": synth.config3}[name]
        shapes |= set(workload_shapes(gen(seed=int(seed), window_s=1.0)))
    shapes = sorted(shapes)
    t0 = time.time()

    def log(m):
        print(m, file=sys.stderr, flush=True)
    log(f"{len(shapes)} shapes")
    rows = tune(torch, shapes, log=log)
    capi.tile_clear()
    write_table(args.out, rows, header=f"workloads {' '.join(args.workloads)}; "
                f"{len(shapes)} shapes in {time.time() - t0:.0f} s")
    won = [r for r in rows if r["variant"] is not None]
    gain = sum(r["us"][r["rule"]] - r["us"][r["variant"]] for r in won)
    log(f"{len(won)} of {len(rows)} shapes changed; {gain:.0f} us saved over one launch of each")


if __name__ == "__main__":
    main()
