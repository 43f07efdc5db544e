"""Seeded synthetic workloads: chain structure, arrival times and input data.

This module holds none of the method's arithmetic; it only describes what to
run and with which inputs.  Tests (for the oracle and the HIP path alike) and
``bench.py`` draw from it.

The paper's chains are closed-source perception, localisation, calibration
and language pipelines (Sec. 5, Tab. "Characteristics of an example
workflow" and Tab. "GPU task profiling results"); they are replaced by chains
of the six synthetic operations with the same structure: 11 chains of 2-6
tasks, 50-300 kernels per task, modality-specific operation mixes, per-chain
GPU work proportional to the paper's E_gpu column, periods of 33-500 ms,
40 % of chains with halved deadlines (f_tight, Sec. 6.2) and 15 ms arrival
jitter (Sec. 5).
"""

import dataclasses
import math

import numpy as np

MS = 1_000_000
US = 1_000

# name, modality, period (ms), E_gpu of the matching chain in the paper (ms)
CHAINS_CFG1 = [
    ("c0_lidar_det", "lidar_det", 100, 28.4),
    ("c1_lidar_det", "lidar_det", 100, 28.4),
    ("c2_cam_det", "camera", 67, 27.0),
    ("c3_cam_det", "camera", 33, 30.2),
    ("c4_cam_face", "camera", 67, 19.5),
    ("c5_cam_det", "camera", 33, 30.2),
    ("c6_cam_sign", "camera", 67, 19.5),
    ("c7_cam_seg", "camera", 67, 27.0),
    ("c8_lidar_loc", "lidar_loc", 200, 19.7),
    ("c9_calib", "calib", 500, 46.1),
    ("c10_text", "text", 500, 6.7),
]

VOXEL_GRID = (512, 512)
VOXEL_FPARAM = (-51.2, -51.2, 5.0)


@dataclasses.dataclass
class Buffer:
    name: str
    kind: str        # "f32", "i32", "u8" (FP8 E4M3 codes) or "bf16" (bfloat16 codes)
    n: int           # elements
    role: str        # "in" (read-only, shared by every frame), "out" (one
    #                  copy per buffer set), "host" (pinned host memory, one
    #                  copy per buffer set, filled with each frame's own data
    #                  before it is submitted) or "state" (device memory
    #                  shared by every frame, updated in frame order)
    init: tuple = ("uniform", -1.0, 1.0)   # for inputs: ("uniform", lo, hi) |
    #                                        ("points", sigma) | ("e4m3", e_lo, e_hi)

    @property
    def nbytes(self):
        return {"u8": 1, "bf16": 2}.get(self.kind, 4) * self.n


@dataclasses.dataclass
class Block:
    """One producer (a contraction or a voxel scatter) and its epilogue kernels."""
    kind: str                 # "dense", "conv", "voxel"
    task: int
    kernels: list             # indices into the task's kernel list
    shape: tuple
    outputs: dict             # role -> slot name written by this block


@dataclasses.dataclass
class ChainDef:
    name: str
    period_ns: int
    deadline_ns: int
    tasks: list               # [{"cpu_ns": int, "kernels": [kernel dict]}]
    buffers: list             # [Buffer]; slot index = position
    blocks: list              # [Block]

    def slot(self, name):
        for i, b in enumerate(self.buffers):
            if b.name == name:
                return i
        raise KeyError(name)


@dataclasses.dataclass
class Workload:
    name: str
    chains: list
    arrivals: list            # (chain, frame, t_offset_ns), sorted by time
    seed: int
    meta: dict


# ----------------------------------------------------------------------------
# input data
# ----------------------------------------------------------------------------
def frame_input(seed, chain, frame, slot, buf, n_valid=None):
    """Deterministic host data of a per-frame input (role "host") for frame
    ``frame``: a point cloud of ``n_valid`` points (the rest zero)."""
    rng = np.random.default_rng([seed, chain, slot, frame, 8])
    out = np.zeros(buf.n, np.float32)
    n = buf.n // 4 if n_valid is None else n_valid
    xyz = rng.normal(0.0, buf.init[1], (n, 3))
    inten = rng.uniform(0.0, 1.0, (n, 1))
    out[: 4 * n] = np.concatenate([xyz, inten], axis=1).astype(np.float32).reshape(-1)
    return out


def input_array(seed, chain, slot, buf):
    """Deterministic host data of an input buffer (float32 or int32)."""
    rng = np.random.default_rng([seed, chain, slot, 7])
    kind = buf.init[0]
    if kind == "uniform":
        lo, hi = buf.init[1], buf.init[2]
        return rng.uniform(lo, hi, buf.n).astype(np.float32)
    if kind == "points":
        sigma = buf.init[1]
        n = buf.n // 4
        xyz = rng.normal(0.0, sigma, (n, 3))
        inten = rng.uniform(0.0, 1.0, (n, 1))
        return np.concatenate([xyz, inten], axis=1).astype(np.float32).reshape(-1)
    if kind == "bf16":
        # bfloat16 codes: the upper halves of float32 values uniform in
        # [lo, hi) (every one a bfloat16 value in that range), as int16
        lo, hi = buf.init[1], buf.init[2]
        f = rng.uniform(lo, hi, buf.n).astype(np.float32)
        return (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    if kind == "e4m3":
        # finite FP8 E4M3 codes: random sign and mantissa, exponent field
        # uniform in [e_lo, e_hi]
        e_lo, e_hi = buf.init[1], buf.init[2]
        sign = rng.integers(0, 2, buf.n) << 7
        expo = rng.integers(e_lo, e_hi + 1, buf.n) << 3
        mant = rng.integers(0, 8, buf.n)
        return (sign | expo | mant).astype(np.uint8)
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# kernel descriptors
# ----------------------------------------------------------------------------
def k_gemm(M, N, K, a, b, c):
    return {"op": "gemm", "shape": (M, N, K), "in": (a, b), "out": (c,)}


def k_bias_relu(R, Cn, axis, x, bias, y):
    return {"op": "bias_relu", "shape": (R, Cn, axis), "in": (x, bias), "out": (y,)}


def k_conv(N, Cc, H, W, x, w, y):
    return {"op": "conv3x3", "shape": (N, Cc, H, W), "in": (x, w), "out": (y,)}


def k_rowsum(R, Cn, z, r):
    return {"op": "rowsum", "shape": (R, Cn), "in": (z,), "out": (r,)}


def k_vecadd(N, W, R, a, b, c):
    return {"op": "vecadd", "shape": (N, W, R), "in": (a, b), "out": (c,)}


def k_gemm_fp8(M, N, K, a, bt, c, m0=0):
    return {"op": "gemm_fp8", "shape": (M, N, K, m0), "in": (a, bt), "out": (c,)}


def k_gemm_bf16(M, N, K, a, bt, c):
    return {"op": "gemm_bf16", "shape": (M, N, K), "in": (a, bt), "out": (c,)}


def k_conv_bf16(Cc, H, W, x, w, y):
    return {"op": "conv3x3_bf16", "shape": (1, Cc, H, W), "in": (x, w), "out": (y,)}


def k_softmax(R, L, x, y):
    return {"op": "softmax", "shape": (R, L), "in": (x,), "out": (y,)}


def k_voxel(N, pts, vi, vc, vz, vf, grid=VOXEL_GRID, fparam=VOXEL_FPARAM):
    return {"op": "voxel", "shape": (N, grid[0], grid[1]), "in": (pts,), "out": (vi, vc, vz, vf),
            "fparam": fparam}


# ----------------------------------------------------------------------------
# configuration 0: 2 chains x 3 tasks x (GEMM, bias+ReLU, conv, row sum)
# ----------------------------------------------------------------------------
def config0(seed=0, frames=10):
    """Two chains (periods 100 and 200 ms, deadline = period), three tasks
    each; a task is GEMM 128^3 -> bias+ReLU -> 3x3 conv on 1x16x64x64 -> row
    sum of the conv output viewed as [1024, 64].  Ten frames per chain at
    k * period, inputs U(-1, 1)."""
    chains = []
    for ci, period in enumerate((100, 200)):
        buffers, tasks, blocks = [], [], []
        for j in range(3):
            base = len(buffers)
            names = ["A", "B", "C", "bias", "X", "W", "Z", "r"]
            sizes = [128 * 128, 128 * 128, 128 * 128, 128, 16 * 64 * 64, 16 * 16 * 9,
                     16 * 64 * 64, 1024]
            roles = ["in", "in", "out", "in", "in", "in", "out", "out"]
            for nm, n, rl in zip(names, sizes, roles):
                buffers.append(Buffer(f"t{j}.{nm}", "f32", n, rl))
            A, B, Cb, bias, X, W, Z, r = range(base, base + 8)
            ks = [k_gemm(128, 128, 128, A, B, Cb), k_bias_relu(128, 128, 0, Cb, bias, Cb),
                  k_conv(1, 16, 64, 64, X, W, Z), k_rowsum(1024, 64, Z, r)]
            tasks.append({"cpu_ns": 0, "kernels": ks})
            blocks.append(Block("dense", j, [0, 1], (128, 128, 128), {"C": f"t{j}.C"}))
            blocks.append(Block("conv", j, [2], (1, 16, 64, 64), {"Y": f"t{j}.Z"}))
            blocks.append(Block("rowsum", j, [3], (1024, 64), {"r": f"t{j}.r"}))
        chains.append(ChainDef(f"c{ci}", period * MS, period * MS, tasks, buffers, blocks))
    arrivals = sorted(((c, f, f * chains[c].period_ns) for c in range(2) for f in range(frames)),
                      key=lambda a: (a[2], a[0], a[1]))
    return Workload("cfg0", chains, arrivals, seed, {"frames": frames})


# ----------------------------------------------------------------------------
# configuration 1: 11 chains, 2-6 tasks, 50-300 kernels per task
# ----------------------------------------------------------------------------
def _model_ns(op, shape):
    """Rough time model used only to size the synthetic tasks."""
    floor = 6 * US
    if op == "gemm":
        M, N, K = shape
        return floor + max(2 * M * N * K / 80e12, 4 * (M * K + K * N + M * N) / 4e12) * 1e9
    if op == "conv3x3":
        _, Cc, H, W = shape
        return floor + max(18 * Cc * Cc * H * W / 70e12, 8 * Cc * H * W / 4e12) * 1e9
    if op in ("bias_relu", "softmax"):
        R, Cn = shape[0], shape[1]
        return floor + 8 * R * Cn / 4e12 * 1e9
    if op == "rowsum":
        R, Cn = shape
        return floor + 4 * R * Cn / 4e12 * 1e9
    if op == "voxel":
        return 3 * floor + 20 * shape[0] / 1e12 * 1e9
    if op == "gemm_bf16":
        M, N, K = shape
        return floor + max(2 * M * N * K / 800e12, (2 * (M * K + K * N) + 4 * M * N) / 4e12) * 1e9
    if op == "conv3x3_bf16":
        _, Cc, H, W = shape
        return floor + max(18 * Cc * Cc * H * W / 500e12, 6 * Cc * H * W / 4e12) * 1e9
    if op == "gemm_fp8":
        M, N, K = shape
        return floor + 2 * M * N * K / 2.5e15 * 1e9
    if op == "vecadd":
        # repeated passes over small vectors run from the caches at about
        # 62.5 GB/s per workgroup (measured on MI355X over 2^20 floats:
        # 58-75 GB/s per workgroup for 32..256 workgroups)
        N, W, R = shape
        return floor + 12 * N * max(R, 1) / (16e12 * min(W, 256) / 256) * 1e9
    if op == "upload":        # host-to-device copy over PCIe
        return 2 * floor + shape[0] * shape[1] / 25e9 * 1e9
    if op == "accum_i32":
        return floor + 12 * shape[0] / 4e12 * 1e9
    raise ValueError(op)


def _pow2_pick(lo, hi, q, s, step=1):
    """Value in [lo, hi] (powers of two apart) at quantile q scaled by s."""
    n = int(round(math.log2(hi / lo)))
    i = min(n, int(math.floor(q * s * (n + 1))))
    return lo * (2 ** i)


def _gemm_shape(q, s):
    dims = []
    for qi in q:
        # multiples of 256 in [256, 4096], log-spaced
        v = 256 * (2 ** (qi * s * 4.0))
        dims.append(int(min(4096, max(256, 256 * round(v / 256)))))
    return tuple(dims)


def _draw_task(rng, modality, task_idx, n_tasks, budget_ns):
    """Draw a task's block list (kind and size quantiles) with 50-300 kernels."""
    target = int(round(math.exp(rng.uniform(math.log(50), math.log(300)))))
    blocks = []
    count = 0
    first = True
    while count < target:
        if first and task_idx == 0 and modality in ("lidar_det", "lidar_loc", "calib"):
            kind = "voxel"
        elif modality in ("lidar_det", "calib"):
            kind = "conv" if rng.uniform() < 0.65 else "dense"
        elif modality == "camera":
            kind = "conv" if rng.uniform() < 0.8 else "dense"
        elif modality == "lidar_loc":
            kind = "dense"
        else:                                  # text
            kind = "dense"
        first = False
        b = {"kind": kind, "q": rng.uniform(0, 1, 3).tolist()}
        if kind == "voxel":
            b["n_points"] = int(rng.integers(30_000, 120_001))
            count += 1
        elif kind == "dense":
            b["softmax"] = bool(rng.uniform() < (0.5 if modality == "text" else 0.2))
            b["rowsum"] = bool(rng.uniform() < 0.15)
            count += 2 + b["softmax"] + b["rowsum"]
        else:
            b["rowsum"] = bool(rng.uniform() < 0.15)
            count += 2 + b["rowsum"]
        blocks.append(b)
    return blocks


def _shapes(b, s):
    if b["kind"] == "vecadd":
        return (b["n"], b["w"], b["r"])
    if b["kind"] == "dense":
        return _gemm_shape(b["q"], s)
    if b["kind"] == "conv" and "img" in b:     # serving: fixed image resolution
        return (1, b["ch"], b["img"], b["img"])
    if b["kind"] == "conv":
        Cc = _pow2_pick(32, 256, b["q"][0], s)
        H = _pow2_pick(32, 256, b["q"][1], s)
        return (1, Cc, H, H)
    return (b["n_points"],)


def _block_time(b, s, bf16=False):
    if b["kind"] == "vecadd":
        return b["count"] * _model_ns("vecadd", (b["n"], b["w"], b["r"]))
    shp = _shapes(b, s)
    if b["kind"] == "dense":
        M, N, K = shp
        t = _model_ns("gemm_bf16" if bf16 else "gemm", shp) + _model_ns("bias_relu", (M, N))
        if b["softmax"]:
            t += _model_ns("softmax", (M, N))
        if b["rowsum"]:
            t += _model_ns("rowsum", (M, N))
        return t
    if b["kind"] == "conv":
        _, Cc, H, W = shp
        t = _model_ns("conv3x3_bf16" if bf16 else "conv3x3", shp) + _model_ns("bias_relu",
                                                                             (Cc, H * W))
        if b["rowsum"]:
            t += _model_ns("rowsum", (Cc, H * W))
        return t
    return _model_ns("voxel", shp)


def _custom_block(custom, task_ns, n=1 << 20):
    """Vector-add kernels over n floats with utilisation custom["util"], each
    repeated to take about custom["kernel_us"] under the time model, as many
    as fill task_ns of modelled time."""
    w = max(1, int(round(custom["util"] * 256)))
    t_k = custom["kernel_us"] * US
    per_pass = _model_ns("vecadd", (n, w, 1)) - 6 * US
    r = max(1, int(round((t_k - 6 * US) / per_pass)))
    count = max(1, int(round(task_ns / _model_ns("vecadd", (n, w, r)))))
    return {"kind": "vecadd", "n": n, "w": w, "r": r, "count": count, "q": [0.0, 0.0, 0.0]}


def _fit_scale(blocks, budget_ns, bf16=False):
    lo, hi = 0.0, 1.0
    if sum(_block_time(b, hi, bf16) for b in blocks) <= budget_ns:
        return hi
    if sum(_block_time(b, lo, bf16) for b in blocks) >= budget_ns:
        return lo
    for _ in range(30):
        mid = 0.5 * (lo + hi)
        if sum(_block_time(b, mid, bf16) for b in blocks) > budget_ns:
            hi = mid
        else:
            lo = mid
    return lo


def _build_chain(name, modality, period_ns, deadline_ns, task_blocks, scales, serving=False,
                 private=False, bf16=False):
    """``serving``: voxel blocks take their points per frame (frame dim 1):
    uploaded from pinned host memory by a gated copy, binned, and added to
    the chain's device-resident cell counts; conv blocks with a
    ``frame_shift`` take the frame's image size (frame dim 2).
    ``private``: every block writes buffers of its own (no double-buffered
    outputs, no softmax / row-sum output shared by the task's blocks), so
    that its epilogue may run outside stream order (fused tails).
    ``bf16``: GEMMs and convolutions on bfloat16 operands (A row-major and B
    transposed; NHWC activations and OHWI weights) with FP32 outputs."""
    buffers, tasks, blocks = [], [], []
    for j, (tb, s) in enumerate(zip(task_blocks, scales)):
        shapes = [_shapes(b, s) for b in tb]
        need = {}

        def want(nm, n, role, init=("uniform", -1.0, 1.0), kind="f32"):
            key = f"t{j}.{nm}"
            cur = need.get(key)
            need[key] = (max(n, cur[0]) if cur else n, role, init, kind)

        B16 = ("bf16", -1.0, 1.0)
        for bi, (b, shp) in enumerate(zip(tb, shapes)):
            sfx = str(bi) if private else ""
            if b["kind"] == "dense":
                M, N, K = shp
                if bf16:
                    want("in_a16", M * K, "in", B16, "bf16")
                    want("in_bt16", N * K, "in", B16, "bf16")
                else:
                    want("in_a", M * K, "in")
                    want("in_b", K * N, "in")
                want("bias_col", N, "in")
                if private:
                    want(f"D{bi}", M * N, "out")
                else:
                    want("D0", M * N, "out")
                    want("D1", M * N, "out")
                if b["softmax"]:
                    want("SM" + sfx, M * N, "out")
                if b["rowsum"]:
                    want("RS" + sfx, M, "out")
            elif b["kind"] == "conv":
                _, Cc, H, W = shp
                if bf16:
                    want("in_x16", Cc * H * W, "in", B16, "bf16")
                    want("in_w16", Cc * Cc * 9, "in", B16, "bf16")
                else:
                    want("in_x", Cc * H * W, "in")
                    want("in_w", Cc * Cc * 9, "in")
                want("bias_row", Cc, "in")
                if private:
                    want(f"C{bi}", Cc * H * W, "out")
                else:
                    want("C0", Cc * H * W, "out")
                    want("C1", Cc * H * W, "out")
                if b["rowsum"]:
                    want("RS" + sfx, Cc, "out")
            elif b["kind"] == "vecadd":
                n = shp[0]
                want("VA", n, "in")
                want("VB", n, "in")
                want("VS", n, "out")
            else:
                n = shp[0]
                G = VOXEL_GRID[0] * VOXEL_GRID[1]
                if serving:
                    want("pts_host", 4 * n, "host", ("points", 20.0))
                    want("pts", 4 * n, "out")
                    want("VSTATE", G, "state", kind="i32")
                else:
                    want("pts", 4 * n, "in", ("points", 20.0))
                want("VI", n, "out", kind="i32")
                want("VC", G, "out", kind="i32")
                want("VZ", G, "out")
                want("VF", G, "out", kind="i32")
        base = len(buffers)
        for key, (n, role, init, kind) in need.items():
            buffers.append(Buffer(key, kind, n, role, init))
        slot = {b.name: i for i, b in enumerate(buffers)}
        ks = []
        dn = cn = 0
        for bi, (b, shp) in enumerate(zip(tb, shapes)):
            first = len(ks)
            sfx = str(bi) if private else ""
            if b["kind"] == "dense":
                M, N, K = shp
                dname = f"t{j}.D{bi}" if private else f"t{j}.D{dn % 2}"
                out = slot[dname]
                outs = {"C": dname}
                dn += 1
                if bf16:
                    ks.append(k_gemm_bf16(M, N, K, slot[f"t{j}.in_a16"], slot[f"t{j}.in_bt16"], out))
                else:
                    ks.append(k_gemm(M, N, K, slot[f"t{j}.in_a"], slot[f"t{j}.in_b"], out))
                ks.append(k_bias_relu(M, N, 0, out, slot[f"t{j}.bias_col"], out))
                if b["softmax"]:
                    ks.append(k_softmax(M, N, out, slot[f"t{j}.SM{sfx}"]))
                    outs["SM"] = f"t{j}.SM{sfx}"
                if b["rowsum"]:
                    ks.append(k_rowsum(M, N, out, slot[f"t{j}.RS{sfx}"]))
                    outs["RS"] = f"t{j}.RS{sfx}"
            elif b["kind"] == "conv":
                _, Cc, H, W = shp
                cname = f"t{j}.C{bi}" if private else f"t{j}.C{cn % 2}"
                out = slot[cname]
                outs = {"Y": cname}
                cn += 1
                if bf16:
                    ks.append(k_conv_bf16(Cc, H, W, slot[f"t{j}.in_x16"], slot[f"t{j}.in_w16"], out))
                else:
                    ks.append(k_conv(1, Cc, H, W, slot[f"t{j}.in_x"], slot[f"t{j}.in_w"], out))
                ks.append(k_bias_relu(Cc, H * W, 1, out, slot[f"t{j}.bias_row"], out))
                if b["rowsum"]:
                    ks.append(k_rowsum(Cc, H * W, out, slot[f"t{j}.RS{sfx}"]))
                    outs["RS"] = f"t{j}.RS{sfx}"
                if serving and "frame_shift" in b:
                    # the frame's image size v sets H = W = v >> shift (and
                    # the planes of the bias and the row sum)
                    for k in ks[first:]:
                        k["frame_dim"], k["frame_shift"] = 2, b["frame_shift"]
            elif b["kind"] == "vecadd":
                n, w, rr = shp
                for _ in range(b["count"]):
                    ks.append(k_vecadd(n, w, rr, slot[f"t{j}.VA"], slot[f"t{j}.VB"],
                                       slot[f"t{j}.VS"]))
                outs = {"C": f"t{j}.VS"}
            else:
                n = shp[0]
                if serving:
                    # the frame's points arrive from host memory (a gated
                    # copy), then are binned; the counts are added to the
                    # chain's device-resident state
                    ks.append({"op": "upload", "shape": (n, 16), "in": (slot[f"t{j}.pts_host"],),
                               "out": (slot[f"t{j}.pts"],), "frame_dim": 1})
                ks.append(k_voxel(n, slot[f"t{j}.pts"], slot[f"t{j}.VI"], slot[f"t{j}.VC"],
                                  slot[f"t{j}.VZ"], slot[f"t{j}.VF"]))
                outs = {"VI": f"t{j}.VI", "VC": f"t{j}.VC", "VZ": f"t{j}.VZ", "VF": f"t{j}.VF"}
                if serving:
                    ks[-1]["frame_dim"] = 1
                    G = VOXEL_GRID[0] * VOXEL_GRID[1]
                    ks.append({"op": "accum_i32", "shape": (G,), "in": (slot[f"t{j}.VC"],),
                               "out": (slot[f"t{j}.VSTATE"],)})
                    outs["STATE"] = f"t{j}.VSTATE"
            blocks.append(Block(b["kind"], j, list(range(first, len(ks))), shp, outs))
        tasks.append({"cpu_ns": 0, "kernels": ks})
        del base
    return ChainDef(name, period_ns, deadline_ns, tasks, buffers, blocks)


# E_cpu (ms) of the same rows of Tab. "Characteristics of an example workflow"
ECPU_CFG1 = [17.4, 16.2, 21.0, 20.2, 21.8, 20.2, 21.8, 21.0, 21.3, 11.2, 17.8]


def config1(seed=0, f_a=1.0, f_d=1.0, f_tight=0.4, u_target=1.6, window_s=10.0,
            jitter_ms=15.0, chains_subset=None, custom=None, cpu=0.0, private=False, bf16=False,
            repeat=1):
    """Eleven chains of 2-6 tasks with 50-300 FP32 kernels per task.

    Per-chain GPU work per frame is proportional to the paper's E_gpu of the
    matching chain, scaled so that sum_c E_c / P_c = u_target under the
    generator's own time model at f_a = 1 (the measured utilisation is
    reported by the benchmark).  The default u_target = 1.6 puts the GPU in
    contention at f_a = 1 (plain FIFO launch misses a few per cent of
    deadlines on MI355X) without sustained overload.  ``f_tight`` of the chains (chosen by the
    seed) get half-period deadlines, the rest a deadline equal to the period;
    all deadlines are scaled by f_d.  Arrivals: per-chain phase U[0, P'),
    nominal k * P' with P' = P / f_a, plus uniform jitter of +-jitter_ms/2.

    ``custom = {"util": U, "kernel_us": T}`` (the sensitivity experiments,
    Sec. 6.6): every odd-indexed task of every chain is replaced by custom
    vector-add kernels run by round(U * 256) workgroups (utilisation U on
    256 CUs), each sized to take about T us under the time model, as many as
    keep the task's modelled time (fewer, longer kernels as T grows).

    ``cpu`` > 0 gives every task a CPU segment (the CPU-scheduling
    experiment, Sec. 4.3): a chain's CPU time per frame is cpu times its GPU
    budget times the paper's E_cpu / E_gpu of the matching row, split over
    the tasks like the GPU budget.

    ``private`` and ``bf16``: see _build_chain (configuration 2).

    ``repeat`` > 1 takes the row list that many times (each copy a chain of
    its own, drawn from its own stream) at the same total u_target: more,
    smaller chains (the scheduling-overhead experiment, Sec. 6.5).
    """
    rng = np.random.default_rng([seed, 1])
    rows = CHAINS_CFG1 if chains_subset is None else [CHAINS_CFG1[i] for i in chains_subset]
    rows = rows * repeat
    lam = u_target / sum(e / p for _, _, p, e in rows)
    n = len(rows)
    n_tight = int(round(f_tight * n))
    tight = set(rng.permutation(n)[:n_tight].tolist())
    chains = []
    for ci, (name, modality, period_ms, egpu) in enumerate(rows):
        crng = np.random.default_rng([seed, 2, ci])
        e_chain = lam * egpu * MS
        n_tasks = int(crng.integers(2, 7))
        split = crng.dirichlet(np.full(n_tasks, 2.0))
        task_blocks, scales = [], []
        for j in range(n_tasks):
            budget = e_chain * split[j]
            tb = _draw_task(crng, modality, j, n_tasks, budget)
            if custom is not None and j % 2 == 1:
                tb = [_custom_block(custom, sum(_block_time(b, _fit_scale(tb, budget)) for b in tb))]
            task_blocks.append(tb)
            scales.append(_fit_scale(tb, budget, bf16))
        period = period_ms * MS
        deadline = int(period * (0.5 if ci in tight else 1.0) * f_d)
        ch = _build_chain(name, modality, period, deadline, task_blocks, scales,
                          private=private, bf16=bf16)
        if ci >= len(rows) // repeat:
            ch.name = f"{name}_r{ci // (len(rows) // repeat)}"
        if cpu > 0:
            ecpu = ECPU_CFG1[CHAINS_CFG1.index(rows[ci])]
            for j, task in enumerate(ch.tasks):
                task["cpu_ns"] = int(cpu * e_chain * split[j] * ecpu / egpu)
        chains.append(ch)
    arr = []
    arng = np.random.default_rng([seed, 3])
    window = int(window_s * 1e9)
    half_j = jitter_ms * MS / 2
    for ci, ch in enumerate(chains):
        p = ch.period_ns / f_a
        phase = arng.uniform(0, p)
        k, last = 0, -1
        while True:
            t = phase + k * p + arng.uniform(-half_j, half_j)
            t = int(max(t, last + 1, 0))
            if t >= window:
                break
            arr.append((ci, k, t))
            last = t
            k += 1
    arr.sort(key=lambda a: (a[2], a[0], a[1]))
    meta = {"f_a": f_a, "f_d": f_d, "f_tight": f_tight, "u_target": u_target,
            "tight": sorted(tight), "window_s": window_s, "cpu": cpu, "private": private,
            "bf16": bf16}
    return Workload("cfg1", chains, arr, seed, meta)


def config2(seed=0, f_a=1.0, f_d=1.0, u_target=1.6, window_s=10.0, **kw):
    """Configuration 2: the eleven chains of configuration 1 drawn from the
    same seeded streams, with BF16 GEMMs and convolutions (FP32 outputs) and
    private block outputs, so that every bias+ReLU with its softmax / row
    sum qualifies as a fused tail.  The generator sizes the contractions
    with its BF16 time model, so the same u_target gives larger shapes than
    configuration 1."""
    wl = config1(seed=seed, f_a=f_a, f_d=f_d, u_target=u_target, window_s=window_s,
                 private=True, bf16=True, **kw)
    wl.name = "cfg2"
    return wl


def config4(seed=0, f_a=1.0, f_d=1.0, u_deadline=0.85, be_gemms=4, be_dim=8192, be_depth=2,
            window_s=10.0, be_chunks=1, **kw):
    """Overload: the eleven chains of configuration 1 at a base load of
    ``u_deadline`` plus one best-effort chain (deadline 0) whose frames are
    ``be_gemms`` back-to-back FP8 E4M3 products be_dim^3 with an FP32
    result.  The best-effort chain is a closed loop: ``be_depth`` of its
    frames are outstanding from the start, and each completion submits the
    next one until the window ends, so it takes all the GPU time the
    deadline chains leave (and, without gating, some they need).  Its frames
    are not in ``arrivals``; ``meta`` names the chain and the depth.
    ``be_chunks`` > 1 splits every product into that many row bands, each a
    kernel of its own (a separate gated launch: a preemption point)."""
    wl = config1(seed=seed, f_a=f_a, f_d=f_d, u_target=u_deadline, window_s=window_s, **kw)
    d = be_dim
    bufs = [Buffer("A8", "u8", d * d, "in", ("e4m3", 4, 9)),
            Buffer("Bt8", "u8", d * d, "in", ("e4m3", 4, 9)),
            Buffer("C", "f32", d * d, "out")]
    assert d % (256 * be_chunks) == 0, "row bands are whole 256-row tiles"
    band = d // be_chunks
    kernels = [k_gemm_fp8(band, d, d, 0, 1, 2, m0=i * band)
               for _ in range(be_gemms) for i in range(be_chunks)]
    e_frame = int(be_gemms * _model_ns("gemm_fp8", (d, d, d)))
    be = ChainDef("be_fp8_gemm", e_frame, 0, [{"cpu_ns": 0, "kernels": kernels}], bufs, [])
    meta = dict(wl.meta, u_deadline=u_deadline, be_chain=len(wl.chains), be_depth=be_depth,
                be_gemms=be_gemms, be_dim=d, be_chunks=be_chunks)
    return Workload("cfg4", wl.chains + [be], list(wl.arrivals), seed, meta)


def config3(seed=0, n_chains=20, f_a=1.0, u_target=1.3, window_s=10.0, pts=(20_000, 150_000),
            img=(256, 1024), rate_jitter=0.2, img_typical=672):
    """Serving: ``n_chains`` chains (the rows of configuration 1, repeated),
    built like configuration 1 with per-frame sizes:

    * chains with a voxel scatter take a different point count per frame,
      uniform in ``pts``, as dims[0]: each frame's points are written to
      pinned host memory, uploaded by a gated copy, binned (kernels
      registered at the maximum count), and the cell counts are added to the
      chain's device-resident state;
    * camera chains take a different image size per frame, a multiple of 32
      uniform in ``img``, square, as dims[1]: each conv layer runs at that
      size / 2^(k+1) with 16 * 2^k channels, k in {0, 1, 2} (a stride-2
      stem before the first), registered at the largest size; the task
      budgets are fitted at ``img_typical`` (about the root mean square of
      the size distribution).

    Arrivals are a Poisson process per chain: exponential gaps of mean
    P_c' = P_c * U(1 - rate_jitter, 1 + rate_jitter) / f_a (the rate of each
    chain jittered by +-20 % once).  ``meta["dims"]`` maps (chain, frame) to
    the frame's dims; ``meta["frame_dims"]`` lists the chains that need them.
    """
    rng = np.random.default_rng([seed, 31])
    rows = [CHAINS_CFG1[i % len(CHAINS_CFG1)] for i in range(n_chains)]
    lam = u_target / sum(e / p for _, _, p, e in rows)
    n_tight = int(round(0.4 * n_chains))
    tight = set(rng.permutation(n_chains)[:n_tight].tolist())
    chains, frame_dims = [], []
    for ci, (name, modality, period_ms, egpu) in enumerate(rows):
        crng = np.random.default_rng([seed, 32, ci])
        e_chain = lam * egpu * MS
        n_tasks = int(crng.integers(2, 5))
        split = crng.dirichlet(np.full(n_tasks, 2.0))
        task_blocks, scales = [], []
        for j in range(n_tasks):
            budget = e_chain * split[j]
            tb = _draw_task(crng, modality, j, n_tasks, budget)
            for b in tb:
                if b["kind"] == "voxel":
                    b["n_points"] = pts[1]
                elif b["kind"] == "conv" and modality == "camera":
                    k = int(crng.integers(0, 3))
                    b["img"] = img_typical >> (k + 1)
                    b["ch"] = 16 << k
                    b["frame_shift"] = k + 1
            task_blocks.append(tb)
            scales.append(_fit_scale(tb, budget))
            for b in tb:
                if "frame_shift" in b:
                    b["img"] = img[1] >> b["frame_shift"]    # registered at the largest
        period = period_ms * MS
        deadline = int(period * (0.5 if ci in tight else 1.0))
        ch = _build_chain(f"s{ci}_{name}", modality, period, deadline, task_blocks, scales,
                          serving=True)
        if any(k.get("frame_dim", 0) for t in ch.tasks for k in t["kernels"]):
            frame_dims.append(ci)
        chains.append(ch)
    arr, dims = [], {}
    arng = np.random.default_rng([seed, 33])
    window = int(window_s * 1e9)
    for ci, ch in enumerate(chains):
        mean = ch.period_ns * arng.uniform(1 - rate_jitter, 1 + rate_jitter) / f_a
        t, f = arng.exponential(mean), 0
        has_pts = any(k["op"] == "voxel" for t_ in ch.tasks for k in t_["kernels"])
        has_img = any(k["op"] == "conv3x3" and k.get("frame_dim", 0) == 2
                      for t_ in ch.tasks for k in t_["kernels"])
        while t < window:
            arr.append((ci, f, int(t)))
            if ci in frame_dims:
                n = int(arng.integers(pts[0], pts[1] + 1)) if has_pts else 0
                v = 32 * int(arng.integers(img[0] // 32, img[1] // 32 + 1)) if has_img else 0
                dims[(ci, f)] = [n, v]
            f += 1
            t += arng.exponential(mean)
    arr.sort(key=lambda a: (a[2], a[0], a[1]))
    meta = {"f_a": f_a, "u_target": u_target, "tight": sorted(tight), "window_s": window_s,
            "dims": dims, "frame_dims": frame_dims, "pts": pts, "img": img}
    return Workload("cfg3", chains, arr, seed, meta)


def footprint_bytes(ch):
    """Device bytes one frame of the chain holds: its output buffers (the
    inputs are shared by every frame)."""
    return sum(b.nbytes for b in ch.buffers if b.role == "out")


def model_utilisation(wl, f_a=1.0):
    """sum_c (model GPU time per frame) / P'_c under the generator's model."""
    u = 0.0
    for ch in wl.chains:
        t = 0.0
        for task in ch.tasks:
            for k in task["kernels"]:
                dims = {"conv3x3": 4, "gemm": 3, "gemm_fp8": 3, "voxel": 1, "vecadd": 3,
                        "accum_i32": 1}.get(k["op"], 2)
                t += _model_ns(k["op"], tuple(k["shape"][:dims]))
        u += t / (ch.period_ns / f_a)
    return u


def kernel_counts(wl):
    return [[len(t["kernels"]) for t in ch.tasks] for ch in wl.chains]
