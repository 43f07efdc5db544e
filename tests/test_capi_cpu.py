"""Host-side checks of the C-ABI library (no GPU needed).

* the library loads and exports every function include/ug.h declares;
* the ctypes structures have the C layout (a gcc-compiled probe of ug.h);
* the C++ policy core, replayed offline instant by instant, takes exactly
  the oracle's decisions on randomised workloads (the oracle's DES produces
  the inputs: arrivals and observed event completions);
* the C++ TH_urgent percentile matches the oracle's.
"""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import des
from oracle import policy as OP
from paper_2509_12207_amd import capi

from _trace import inputs_to_records, record_to_tuple

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ug.h")
MS = 1_000_000
US = 1_000


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ug_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = capi.lib()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []
    assert sorted(capi.EXPORTED) == names
    out = subprocess.run(["nm", "-D", "--defined-only", capi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (ug_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_c(tmp_path):
    probe = tmp_path / "probe.c"
    structs = {"ug_kernel": capi.Kernel, "ug_task": capi.Task, "ug_config": capi.Config,
               "ug_completion": capi.Completion, "ug_record": capi.Record,
               "ug_stats": capi.Stats, "ug_metrics": capi.Metrics, "ug_tail": capi.Tail}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ug.h"', 'int main(void){']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            cf = "in" if f == "in_" else f
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0;}")
    probe.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(probe), "-o",
                    str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)
    assert capi.RECORD_DTYPE.itemsize == C.sizeof(capi.Record)
    assert capi.COMPLETION_DTYPE.itemsize == C.sizeof(capi.Completion)


def test_config_defaults_and_errors():
    L = capi.lib()
    cfg = capi.Config()
    L.ug_config_default(C.byref(cfg))
    assert cfg.abi_version == capi.ABI_VERSION
    assert cfg.delta_eval_ns == 500_000 and cfg.delay_poll_ns == 1_000_000
    assert abs(cfg.util_exempt - 0.1) < 1e-7
    assert cfg.flags == capi.F_BIND | capi.F_DELAY | capi.F_BATCH | capi.F_ADMIT | capi.F_PLACE
    assert cfg.own_streams == 0
    assert cfg.admit_tasks == 4
    assert cfg.calib_period_ns == 1_000_000 and list(cfg.lanes[:cfg.n_levels]) == [2, 6]
    bad = capi.Config()
    L.ug_config_default(C.byref(bad))
    bad.abi_version = 99
    h = C.c_void_p()
    assert L.ug_create(C.byref(bad), C.byref(h)) == capi.EINVAL
    g = capi.Gate(device=-1)
    with pytest.raises(capi.UgError) as e:
        g.register_chain(1, 10, [{"kernels": [{"op": "gemm", "shape": (0, 4, 4), "in": (0, 1),
                                               "out": (2,)}]}], 3)
    assert e.value.status == capi.EINVAL
    with pytest.raises(capi.UgError) as e:
        g.register_chain(1, 10, [{"kernels": [{"op": "gemm", "shape": (4, 4, 4), "in": (0, 5),
                                               "out": (2,)}]}], 3)
    assert e.value.status == capi.EINVAL
    with pytest.raises(capi.UgError) as e:
        g.start()
    assert e.value.status == capi.ENODEV
    # the stream pool: the sum of the lanes for the urgency policy; streams
    # need a device
    assert g.streams_needed() == 8
    arr = capi.pointer_array([0x10] * 8)
    assert L.ug_attach_streams(g.h, arr, 8) == capi.ENODEV
    f = capi.Gate("fifo", device=-1)
    assert f.cfg.flags == 0
    f.register_chain(1, 10, [{"kernels": [{"op": "rowsum", "shape": (4, 4), "in": (0,),
                                           "out": (1,)}]}] * 3, 2)
    assert f.streams_needed() == 3
    f.close()
    with pytest.raises(capi.UgError) as e:
        g.submit(0, 0, [1, 2, 3])
    assert e.value.status in (capi.ESTATE, capi.EINVAL)
    g.close()


def test_voxel_workspace_size_and_checks():
    # host-side only: sizes, and the errors returned before anything runs
    def desc(n, nx=512, ny=512):
        return {"op": "voxel", "shape": (n, nx, ny), "in": (0,), "out": (1, 2, 3, 4),
                "fparam": (-51.2, -51.2, 5.0)}
    assert capi.kernel_workspace(desc(100_000)) == 0            # direct path
    assert capi.kernel_workspace(desc(1 << 20, 4096, 4096)) == 0  # grid too large to bin
    n = (1 << 20) + 3
    need = capi.kernel_workspace(desc(n))
    n8 = (n + 7) // 8 * 8
    assert need >= 10 * n8 and need % 256 == 0
    fake = [0x10000 * (i + 1) for i in range(5)]   # never dereferenced
    for ws, nbytes in [(0, need), (0x100000, need - 1), (0x100000 + 16, need)]:
        with pytest.raises(capi.UgError) as e:
            capi.kernel_launch_ws(desc(n), fake, ws, nbytes)
        assert e.value.status == capi.EINVAL


def test_conv3x3_shape_limits():
    # host-side only: the FP32 convolution stages by 32-bit byte offsets, so
    # a plane of 2^26 pixels or more is refused before anything runs
    fake = [0x10000 * (i + 1) for i in range(3)]   # never dereferenced
    for shape in [(1, 4, 8192, 8192), (1, 4, 1 << 26, 1), (1, 0, 8, 8), (1, 40000, 8, 8)]:
        with pytest.raises(capi.UgError) as e:
            capi.kernel_launch({"op": "conv3x3", "shape": shape, "in": (0, 1), "out": (2,)}, fake)
        assert e.value.status == capi.EINVAL, shape


# ----------------------------------------------------------------------------
# C++ policy core == oracle gate model, instant by instant
# ----------------------------------------------------------------------------
def _random_workload(r, n_chains, n_frames):
    chains, arrivals = [], []
    for c in range(n_chains):
        tasks = []
        for j in range(int(r.integers(1, 4))):
            ks = [(int(r.integers(20, 400)) * US, float(r.choice([0.05, 0.09, 0.1, 0.5, 1.0])))
                  for _ in range(int(r.integers(1, 9)))]
            tasks.append({"cpu_ns": int(r.integers(0, 3)) * 150 * US,
                          "est_ns": [e for e, _ in ks], "util": [u for _, u in ks]})
        period = int(r.integers(3, 12)) * MS
        # one chain in four is best-effort (deadline 0)
        deadline = 0 if r.random() < 0.25 else int(period * r.choice([0.5, 1.0]))
        chains.append({"deadline_ns": deadline, "tasks": tasks, "period_ns": period})
        phase = int(r.integers(0, period))
        for f in range(n_frames):
            arrivals.append((c, f, phase + f * period + int(r.integers(0, 500)) * US))
    return chains, arrivals


SHIFT = 10      # sized kernels are registered as 4 x 4 row sums of planes: s = v >> 10 <= 2


def _sized_variant(r, chains, arrivals):
    """Per-frame sizes: in about half of the chains about half of the kernels
    take the frame's size v in [1024, 3071] and have two or three profile
    points there; every frame draws its v."""
    out = []
    for ch in chains:
        ch = dict(ch, tasks=[dict(t) for t in ch["tasks"]])
        sized = r.random() < 0.5
        for t in ch["tasks"]:
            nk = len(t["est_ns"])
            t["frame_dim"], t["prof"] = [], []
            for _ in range(nk):
                if sized and r.random() < 0.5:
                    vs = sorted(r.choice(np.arange(1024, 3072), int(r.integers(2, 4)), replace=False))
                    t["frame_dim"].append(1)
                    t["prof"].append([(int(v), int(r.integers(20, 600)) * US) for v in vs])
                else:
                    t["frame_dim"].append(0)
                    t["prof"].append(None)
        out.append(ch)
    arr = [(c, f, t, (int(r.integers(1024, 3072)),)) for c, f, t in arrivals]
    return out, arr


def _register(g, chains):
    for c, ch in enumerate(chains):
        tasks = []
        for t in ch["tasks"]:
            nk = len(t["est_ns"])
            fds = t.get("frame_dim", [0] * nk)
            ks = [{"op": "rowsum", "shape": (4, 4), "in": (0,), "out": (1,), "est_ns": e,
                   "util": u, "frame_dim": fd, "frame_shift": SHIFT if fd else 0}
                  for e, u, fd in zip(t["est_ns"], t["util"], fds)]
            tasks.append({"cpu_ns": t["cpu_ns"], "kernels": ks})
        g.register_chain(ch.get("period_ns", 0), ch["deadline_ns"], tasks, 2)
        g_idx = 0
        for t in ch["tasks"]:
            for pts in t.get("prof", [None] * len(t["est_ns"])):
                if pts:
                    g.set_profile(c, g_idx, pts)
                g_idx += 1


def _flags(cfg):
    return ((capi.F_BIND if cfg.get("bind", True) else 0) | (capi.F_DELAY if cfg.get("delay", True) else 0)
            | (capi.F_BATCH if cfg.get("batch", True) else 0)
            | (capi.F_CALIBRATE if cfg.get("calibrate", False) else 0)
            | (capi.F_ADMIT if cfg.get("admit", True) else 0)
            | (capi.F_EXIT if cfg.get("exit", False) else 0)
            | (capi.F_NO_OVERLAP if cfg.get("no_overlap", False) else 0)
            | (capi.F_GRAPH if cfg.get("graph", False) else 0)
            | (capi.F_CPU_PRIO if cfg.get("cpu_prio", False) else 0))


def _gate_for(cfg):
    lanes = cfg.get("lanes", [2, 6])
    return capi.Gate(policy=cfg.get("policy", "urgency"), device=-1, lanes=lanes,
                     flags=_flags(cfg), delta_eval_ns=cfg.get("delta_eval_ns", 500_000),
                     delay_poll_ns=cfg.get("delay_poll_ns", 1_000_000),
                     th_slack_ns=cfg.get("th_slack_ns", 0),
                     calib_period_ns=cfg.get("calib_period_ns", 1_000_000),
                     admit_tasks=cfg.get("admit_tasks", 4),
                     order_key=cfg.get("key", "urgency"),
                     est_noise_permille=cfg.get("est_noise_permille", 0),
                     noise_seed=cfg.get("noise_seed", 0),
                     max_hold_ns=cfg.get("max_hold_ns", 0),
                     cpu_cores=cfg.get("cpu_cores", 0))


CFGS = [
    {"policy": "urgency", "th_slack_ns": 3 * MS},
    {"policy": "urgency", "th_slack_ns": 3 * MS, "admit": False},
    {"policy": "urgency", "th_slack_ns": 3 * MS, "delay_poll_ns": 0, "admit": False},
    {"policy": "urgency", "th_slack_ns": 0, "lanes": [1, 1]},
    {"policy": "urgency", "th_slack_ns": 2 * MS, "lanes": [2, 3, 1, 2]},
    {"policy": "urgency", "batch": False, "bind": False, "th_slack_ns": 2 * MS},
    {"policy": "urgency", "delay": False, "th_slack_ns": 0, "calibrate": True},
    {"policy": "urgency", "th_slack_ns": 2 * MS, "calibrate": True, "calib_period_ns": 0},
    {"policy": "urgency", "th_slack_ns": 2 * MS, "admit": True, "admit_tasks": 2},
    {"policy": "urgency", "th_slack_ns": 0, "admit": True, "admit_tasks": 1, "lanes": [1, 2]},
    {"policy": "urgency", "th_slack_ns": 3 * MS, "exit": True},
    {"policy": "urgency", "th_slack_ns": 0, "exit": True, "admit": False, "batch": False},
    {"policy": "urgency", "th_slack_ns": 4 * MS, "lanes": [1]},
    {"policy": "urgency", "th_slack_ns": 2 * MS, "no_overlap": True},
    {"policy": "urgency", "th_slack_ns": 2 * MS, "no_overlap": True, "delta_eval_ns": 0},
    {"policy": "urgency", "th_slack_ns": 2 * MS, "key": "edf"},
    {"policy": "urgency", "th_slack_ns": 2 * MS, "key": "sjf"},
    {"policy": "urgency", "th_slack_ns": 2 * MS, "key": "hrrn"},
    {"policy": "urgency", "th_slack_ns": 0, "key": "lcuf", "lanes": [2, 3, 3]},
    {"policy": "urgency", "th_slack_ns": 2 * MS, "key": "saedf"},
    {"policy": "urgency", "th_slack_ns": 0, "key": "eqdf", "admit_tasks": 2, "lanes": [1, 3]},
    {"policy": "urgency", "th_slack_ns": 3 * MS, "est_noise_permille": 300, "noise_seed": 5},
    {"policy": "urgency", "th_slack_ns": 3 * MS, "graph": True},
    {"policy": "urgency", "th_slack_ns": 0, "graph": True, "admit": False, "delay_poll_ns": 0},
    {"policy": "urgency", "th_slack_ns": 2 * MS, "key": "hrrn", "est_noise_permille": 500,
     "noise_seed": 2 ** 63 + 9},
    {"policy": "urgency", "th_slack_ns": 3 * MS, "max_hold_ns": 2 * MS},
    {"policy": "urgency", "th_slack_ns": 3 * MS, "max_hold_ns": 700_000, "delay_poll_ns": 0},
    {"policy": "urgency", "th_slack_ns": 0, "max_hold_ns": 1 * MS, "admit_tasks": 1},
    {"policy": "urgency", "th_slack_ns": 3 * MS, "cpu_cores": 1},
    {"policy": "urgency", "th_slack_ns": 3 * MS, "cpu_cores": 1, "cpu_prio": True},
    {"policy": "urgency", "th_slack_ns": 0, "cpu_cores": 2, "cpu_prio": True, "key": "edf",
     "admit_tasks": 2},
    {"policy": "fifo", "cpu_cores": 2},
    {"policy": "fifo"},
]


@pytest.mark.parametrize("sized", [False, True])
@pytest.mark.parametrize("seed", range(8))
def test_cpp_policy_replays_oracle_decisions(seed, sized):
    r = np.random.default_rng(500 + seed)
    chains, arrivals = _random_workload(r, int(r.integers(2, 6)), int(r.integers(2, 6)))
    if sized:
        chains, arrivals = _sized_variant(r, chains, arrivals)
    noise = {}

    def dur(c, f, g):
        if (c, f, g) not in noise:
            est = [e for t in chains[c]["tasks"] for e in t["est_ns"]]
            noise[(c, f, g)] = max(1, int(est[g] * r.uniform(0.5, 1.6)))
        return noise[(c, f, g)]

    for cfg in (CFGS[::3] if sized else CFGS):
        res = des.simulate(chains, cfg, arrivals, dur)
        g = _gate_for(cfg)
        _register(g, chains)
        n_dec = 0
        for idx, (t, arr, evs, dec) in enumerate(res["instants"]):
            got = [record_to_tuple(x) for x in g.replay_instant(t, inputs_to_records(arr, evs))]
            assert got == list(dec), (cfg, idx, t)
            n_dec += len(dec)
        assert n_dec > 0
        if cfg.get("calibrate"):
            samples = g.calibration_samples()
            assert samples == res["gate"].samples
            assert g.calibration_threshold(95) == OP.threshold_from_samples(samples)
        g.close()


def test_cpp_replay_rejects_unexpected_event():
    g = _gate_for({"policy": "urgency"})
    _register(g, [{"deadline_ns": 10 * MS, "tasks": [{"cpu_ns": 0, "est_ns": [MS], "util": [1.0]}]}])
    g.replay_instant(0, inputs_to_records([(0, 0, 0)], []))
    with pytest.raises(capi.UgError):
        g.replay_instant(1, inputs_to_records([], [(0, 0, 0, 1, 5)]))
    g.close()


def test_errors_from_many_threads_on_one_context():
    # several threads fail calls on one context (each failure records its
    # message) while others read the message: every read is one of the
    # messages written, never a torn or freed string
    import threading
    L = capi.lib()
    g = capi.Gate(device=-1)
    g.register_chain(1, 10, [{"kernels": [{"op": "rowsum", "shape": (4, 4), "in": (0,),
                                           "out": (1,)}]}], 2)
    ptrs = capi.pointer_array([0x1000, 0x2000])
    seen, bad = set(), []

    def fail_submit():
        for _ in range(2000):
            assert L.ug_frame_submit(g.h, 0, 0, ptrs, 2, None) == capi.ESTATE

    def fail_estimate():
        for _ in range(2000):
            assert L.ug_kernel_set_estimate(g.h, 0, 99, 1, -1.0) == capi.EINVAL

    def read():
        for _ in range(4000):
            m = L.ug_last_error(g.h).decode()
            seen.add(m)
            if m not in ("not started", "no such kernel", ""):
                bad.append(m)

    th = [threading.Thread(target=f) for f in (fail_submit, fail_estimate, read, read)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not bad and seen <= {"not started", "no such kernel", ""}
    g.close()


def _random_task(rng):
    """A task of contraction blocks over a few shared slots: bias+ReLU after
    most contractions (on their output or not), optional softmax / row sum,
    slots reused so that later kernels collide with earlier tails."""
    nslot = int(rng.integers(4, 9))
    ks = []
    for _ in range(int(rng.integers(1, 6))):
        out = int(rng.integers(0, nslot))
        a, b = (int(v) for v in rng.integers(0, nslot, 2))
        R = int(rng.choice([8, 32, 40]))   # 40 x 8192 floats: over the size limit
        C = int(rng.choice([32, 64, 6, 4100, 8192]))
        kind = rng.choice(["gemm", "conv3x3", "gemm_bf16", "conv3x3_bf16", "softmax"])
        if kind == "gemm":
            ks.append({"op": "gemm", "shape": (R, C, 16), "in": (a, b), "out": (out,)})
        elif kind == "gemm_bf16":
            ks.append({"op": "gemm_bf16", "shape": (R, C, 32), "in": (a, b), "out": (out,)})
        elif kind == "conv3x3":
            ks.append({"op": "conv3x3", "shape": (1, 8, 4, 4), "in": (a, b), "out": (out,)})
        elif kind == "conv3x3_bf16":
            ks.append({"op": "conv3x3_bf16", "shape": (1, 32, 4, 4), "in": (a, b), "out": (out,)})
        else:
            ks.append({"op": "softmax", "shape": (R, C), "in": (a,), "out": (out,)})
        if rng.uniform() < 0.8:
            x = out if rng.uniform() < 0.85 else int(rng.integers(0, nslot))
            y = x if rng.uniform() < 0.8 else int(rng.integers(0, nslot))
            bias = int(rng.integers(0, nslot))
            ks.append({"op": "bias_relu", "shape": (R, C, int(rng.integers(0, 2))),
                       "in": (x, bias), "out": (y,)})
            for op in rng.permutation(["softmax", "rowsum", "softmax"])[: int(rng.integers(0, 3))]:
                src = y if rng.uniform() < 0.9 else int(rng.integers(0, nslot))
                shp = (R, C) if rng.uniform() < 0.9 else (R, C + 4)
                ks.append({"op": str(op), "shape": shp, "in": (src,),
                           "out": (int(rng.integers(0, nslot)),)})
    return ks, nslot


def test_chain_tails_match_the_oracle():
    """The tails the gate fuses (ug_chain_tails, C++) are the oracle's
    (oracle.fused.tail_runs) on random tasks with colliding buffers."""
    from oracle import fused as OF
    rng = np.random.default_rng(7)
    g = capi.Gate(device=-1)
    total = 0
    for _ in range(300):
        tasks, expect, off, nb = [], [], 0, 1
        for _ in range(int(rng.integers(1, 4))):
            ks, nslot = _random_task(rng)
            nb = max(nb, nslot)
            tasks.append({"cpu_ns": 0, "kernels": [dict(k, est_ns=1000, util=1.0) for k in ks]})
            expect += [(off + a, off + b) for a, b in OF.tail_runs(ks)]
            off += len(ks)
        cid = g.register_chain(100 * MS, 100 * MS, tasks, nb)
        assert g.chain_tails(cid) == expect
        total += len(expect)
    assert total > 100
    g.close()


def test_tile_table_set_load_and_errors(tmp_path):
    """The tuning table (host logic): variants per op, set / remove / clear,
    a table file with comments, a malformed file adds nothing, and the
    variant a launch would take follows the table."""
    conv = {"op": "conv3x3", "shape": (1, 32, 64, 64), "in": (0, 1), "out": (2,)}
    gemm = {"op": "gemm", "shape": (256, 512, 1024), "in": (0, 1), "out": (2,)}
    capi.tile_clear()
    assert capi.tile_variants("gemm") == 3 and capi.tile_variants("conv3x3") == 5
    assert capi.tile_variants("softmax") == 0
    rule_c, rule_g = capi.tile_get(conv), capi.tile_get(gemm)
    assert 0 <= rule_c < 5 and 0 <= rule_g < 3
    capi.tile_set("conv3x3", conv["shape"], (rule_c + 1) % 5)
    assert capi.tile_get(conv) == (rule_c + 1) % 5 and capi.tile_get(gemm) == rule_g
    capi.tile_set("conv3x3", conv["shape"], -1)
    assert capi.tile_get(conv) == rule_c
    with pytest.raises(capi.UgError):
        capi.tile_set("conv3x3", conv["shape"], 5)
    with pytest.raises(capi.UgError):
        capi.tile_set("softmax", (4, 4), 0)
    good = tmp_path / "tiles.txt"
    good.write_text(f"# a table\n{capi.OP_GEMM_F32} 256 512 1024 0 {(rule_g + 2) % 3}  # us 1 2 3\n"
                    "\n3 1 32 64 64 0\n")
    assert capi.tile_load(str(good)) == 2
    assert capi.tile_get(gemm) == (rule_g + 2) % 3 and capi.tile_get(conv) == 0
    capi.tile_clear()
    bad = tmp_path / "bad.txt"
    bad.write_text("3 1 32 64 64 0\n1 256 512 1024\n")
    with pytest.raises(capi.UgError):
        capi.tile_load(str(bad))
    assert capi.tile_get(conv) == rule_c           # nothing added
    with pytest.raises(capi.UgError):
        capi.tile_load(str(tmp_path / "missing.txt"))
    # a context created with a table reads it
    g = capi.Gate(device=-1, tile_table=str(good))
    assert capi.tile_get(conv) == 0
    g.close()
    with pytest.raises(capi.UgError):
        capi.Gate(device=-1, tile_table=str(bad))
    capi.tile_clear()
