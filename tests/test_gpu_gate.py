"""End-to-end parity of the urgency-gated path on the GPU, through the C-ABI.

* Configuration 0 (2 chains x 3 tasks x {GEMM, bias+ReLU, conv, row sum}):
  every output against the oracle, for the urgency gate and for FIFO launch;
  the gate's decision log replayed through the oracle gate model must give
  identical decisions (launch order bit-exact given the recorded
  observations).
* Configuration 1 (11 chains, full shapes, the launch configuration the
  benchmark times) for a short window: decision-log replay, sampled outputs
  of every task against the oracle, voxel outputs bit-exact.
* A frame alone and the same frame in the mix give bit-identical outputs.
"""

import numpy as np
import pytest
import torch

from oracle import des
from oracle import kernels as OK
from paper_2509_12207_amd import capi, runner, synth

import _trace as T

pytestmark = pytest.mark.gpu
MS = 1_000_000
TOL = 1e-5


def run_workload(wl, policy, n_sets=2, th=5 * MS, arrivals=None, flags=None, profile=True,
                 est_from=None, **cfg):
    dw = runner.DeviceWorkload(wl, n_sets=n_sets)
    kw = dict(trace_capacity=1 << 22, th_slack_ns=th, **cfg)
    if flags is not None:
        kw["flags"] = flags
    g = runner.make_gate(wl, policy, **kw)
    if est_from is not None:
        for (c, k), (e, u) in est_from.items():
            g.set_estimate(c, k, e, u)
    elif profile:
        runner.profile(g, dw, warmup=1, reps=3)
    est = runner.estimates(g, wl)
    g.start()
    comps, t0 = runner.run(g, dw, wl.arrivals if arrivals is None else arrivals)
    g.drain(60.0)
    g.stop()
    trace = g.trace()
    stats = g.stats()
    metrics = g.metrics()
    g.close()
    return dw, comps, trace, est, stats, metrics


def oracle_cfg(policy, th=5 * MS, **kw):
    cfg = {"policy": policy, "th_slack_ns": th}
    cfg.update(kw)
    return cfg


def check_cfg0_outputs(wl, dw, k=0):
    for c, ch in enumerate(wl.chains):
        s = {b.name: i for i, b in enumerate(ch.buffers)}
        for j in range(3):
            A = dw.host_input(c, s[f"t{j}.A"]).reshape(128, 128)
            B = dw.host_input(c, s[f"t{j}.B"]).reshape(128, 128)
            bias = dw.host_input(c, s[f"t{j}.bias"])
            X = dw.host_input(c, s[f"t{j}.X"]).reshape(1, 16, 64, 64)
            W = dw.host_input(c, s[f"t{j}.W"]).reshape(16, 16, 3, 3)
            Cg = dw.output(c, s[f"t{j}.C"], k).reshape(128, 128)
            Zg = dw.output(c, s[f"t{j}.Z"], k).reshape(1, 16, 64, 64)
            rg = dw.output(c, s[f"t{j}.r"], k)
            ref_c = OK.bias_relu_f32(OK.gemm_f64(A, B).astype(np.float32), bias, 0)
            scale = OK.gemm_abs_f64(A, B) + np.abs(bias)
            assert np.all(np.abs(Cg - ref_c) <= TOL * scale)
            Z64 = OK.conv3x3_f64(X, W)
            assert np.all(np.abs(Zg - Z64) <= TOL * OK.conv3x3_abs_f64(X, W))
            r64, ra = OK.rowsum_f64(Zg.reshape(1024, 64))
            assert np.all(np.abs(rg - r64) <= TOL * ra)


@pytest.mark.parametrize("policy", ["urgency", "fifo"])
def test_cfg0_outputs_and_replay(policy):
    wl = synth.config0(frames=10)
    # compress the 100/200 ms periods 10x so the test runs in ~0.2 s
    arr = [(c, f, t // 10) for c, f, t in wl.arrivals]
    dw, comps, trace, est, stats, metrics = run_workload(wl, policy, arrivals=arr)
    assert len(comps) == 20 and stats["trace_dropped"] == 0
    assert sorted((int(c["chain"]), int(c["frame"])) for c in comps) == \
        sorted((c, f) for c, f, _ in arr)
    check_cfg0_outputs(wl, dw, 0)
    check_cfg0_outputs(wl, dw, 1)
    inst = T.instants_from_trace(trace)
    chains = T.oracle_chains(wl, est)
    assert des.replay(chains, oracle_cfg(policy), inst) is None
    if policy == "urgency":
        des.check_log(chains, oracle_cfg(policy), inst)
    # completions agree with the log and with Eq. (3)
    done = {(d[1], d[2]): d[3] for i in inst for d in i[3] if d[0] == "COMPLETE"}
    for c in comps:
        assert done[(int(c["chain"]), int(c["frame"]))] == int(c["t_done_ns"])
        assert int(c["latency_ns"]) == int(c["t_done_ns"]) - int(c["t_arr_ns"])
        assert bool(c["missed"]) == (int(c["latency_ns"]) > wl.chains[int(c["chain"])].deadline_ns)
    assert metrics["frames"] == 20


@pytest.mark.parametrize("mode", ["sync_batched", "sync"])
def test_cfg0_launch_synchronisation_modes(mode):
    # the no-overlap launch variants (a closed batch is waited for until it
    # has finished): every frame completes, outputs match the oracle and the
    # log replays through the oracle gate model with the same flags
    wl = synth.config0(frames=4)
    arr = [(c, f, t // 10) for c, f, t in wl.arrivals]
    delta = 0 if mode == "sync" else 20_000     # small batches: several per task
    flags = capi.F_BIND | capi.F_DELAY | capi.F_BATCH | capi.F_ADMIT | capi.F_NO_OVERLAP
    dw, comps, trace, est, stats, metrics = run_workload(wl, "urgency", arrivals=arr, flags=flags,
                                                         delta_eval_ns=delta)
    assert len(comps) == len(arr) and stats["trace_dropped"] == 0
    check_cfg0_outputs(wl, dw, 0)
    check_cfg0_outputs(wl, dw, 1)
    inst = T.instants_from_trace(trace)
    chains = T.oracle_chains(wl, est)
    cfg = oracle_cfg("urgency", no_overlap=True, delta_eval_ns=delta)
    assert des.replay(chains, cfg, inst) is None
    des.check_log(chains, cfg, inst)
    # at most one batch of a task on the device at a time: every batch after
    # the first is preceded by its own start event, recorded behind the last one
    n_launch = sum(1 for i in inst for d in i[3] if d[0] == "LAUNCH")
    n_start = sum(1 for i in inst for d in i[3] if d[0] == "EVREC" and d[4] == 0)
    if mode == "sync":
        assert n_start == n_launch
    else:
        assert len(arr) * 3 < n_start <= n_launch


@pytest.mark.parametrize("policy", ["urgency", "fifo"])
def test_cfg0_task_graphs(policy):
    # every task launched as one captured graph: outputs match the oracle
    # (both output copies, so each buffer set's graph is exercised) and the
    # log replays through the oracle gate model with graphs on
    wl = synth.config0(frames=4)
    arr = [(c, f, t // 10) for c, f, t in wl.arrivals]
    flags = (capi.F_BIND | capi.F_DELAY | capi.F_BATCH | capi.F_ADMIT | capi.F_GRAPH
             if policy == "urgency" else capi.F_GRAPH)
    dw, comps, trace, est, stats, metrics = run_workload(wl, policy, arrivals=arr, flags=flags)
    assert len(comps) == len(arr) and stats["trace_dropped"] == 0
    check_cfg0_outputs(wl, dw, 0)
    check_cfg0_outputs(wl, dw, 1)
    inst = T.instants_from_trace(trace)
    chains = T.oracle_chains(wl, est)
    cfg = oracle_cfg(policy, graph=True)
    assert des.replay(chains, cfg, inst) is None
    # one start event per task: no batches inside a task
    n_start = sum(1 for i in inst for d in i[3] if d[0] == "EVREC" and d[4] == 0)
    assert n_start == len(arr) * 3


# ----------------------------------------------------------------------------
def _last_writers(ch):
    """slot name -> last block writing it, per task."""
    last = {}
    for b in ch.blocks:
        for role, name in b.outputs.items():
            last[name] = (b, role)
    return last


def check_cfg1_outputs(wl, dw, k=0, samples=6, seed=0):
    """Sampled outputs of every chain whose frame k ran (frame k writes output
    copy k); returns the number of chains checked."""
    r = np.random.default_rng(seed)
    checked = 0
    for c, ch in enumerate(wl.chains):
        if not any(cc == c and f == k for cc, f, _ in wl.arrivals):
            continue
        checked += 1
        slot = {b.name: i for i, b in enumerate(ch.buffers)}
        inp = {}

        def host(name):
            if name not in inp:
                inp[name] = dw.host_input(c, slot[name])
            return inp[name]

        for name, (blk, role) in _last_writers(ch).items():
            j = blk.task
            got = dw.output(c, slot[name], k)
            bf16 = f"t{j}.in_a16" in slot or f"t{j}.in_x16" in slot
            if blk.kind == "dense":
                M, N, K = blk.shape
                if bf16:
                    # bfloat16 operands (B transposed), exact in float64
                    A = OK.bf16_decode(host(f"t{j}.in_a16")[: M * K].view(np.uint16)).reshape(M, K)
                    B = OK.bf16_decode(host(f"t{j}.in_bt16")[: N * K].view(np.uint16)).reshape(N, K).T
                else:
                    A = host(f"t{j}.in_a")[: M * K].reshape(M, K)
                    B = host(f"t{j}.in_b")[: K * N].reshape(K, N)
                bias = host(f"t{j}.bias_col")[:N]
                rows = r.integers(0, M, samples)
                for m in rows:
                    row = A[m].astype(np.float64) @ B.astype(np.float64)
                    sc = np.abs(A[m]).astype(np.float64) @ np.abs(B).astype(np.float64) + np.abs(bias)
                    y = OK.bias_relu_f32(row.astype(np.float32)[None, :], bias, 0)[0]
                    if role == "C":
                        g = got[m * N:(m + 1) * N]
                        assert np.all(np.abs(g - y) <= TOL * sc), (ch.name, name)
                    elif role == "SM":
                        ref = OK.softmax_f64(y[None, :])[0]
                        g = got[m * N:(m + 1) * N]
                        # softmax of a row known to 1e-5 * scale: allow that
                        # input error through the (1-Lipschitz in log) map
                        tol = TOL * ref + 2 * ref * TOL * sc.max()
                        assert np.all(np.abs(g - ref) <= tol + 1e-37), (ch.name, name)
                    elif role == "RS":
                        ref = float(np.sum(y.astype(np.float64)))
                        assert abs(got[m] - ref) <= TOL * float(np.sum(np.abs(y))) + TOL * sc.sum(), \
                            (ch.name, name)
            elif blk.kind == "conv":
                _, Cc, H, W = blk.shape
                if bf16:
                    # NHWC activations and OHWI weights, as NCHW / OIHW values
                    X = OK.bf16_decode(host(f"t{j}.in_x16")[: Cc * H * W].view(np.uint16)).reshape(
                        H, W, Cc).transpose(2, 0, 1)[None]
                    Wt = OK.bf16_decode(host(f"t{j}.in_w16")[: Cc * Cc * 9].view(np.uint16)).reshape(
                        Cc, 3, 3, Cc).transpose(0, 3, 1, 2)
                else:
                    X = host(f"t{j}.in_x")[: Cc * H * W].reshape(1, Cc, H, W)
                    Wt = host(f"t{j}.in_w")[: Cc * Cc * 9].reshape(Cc, Cc, 3, 3)
                bias = host(f"t{j}.bias_row")[:Cc]
                if role == "Y":
                    for o, y, x in zip(r.integers(0, Cc, samples), r.integers(0, H, samples),
                                       r.integers(0, W, samples)):
                        v, s = OK.conv3x3_entry_f64(X, Wt, 0, o, y, x)
                        want = max(np.float32(v) + bias[o], 0)
                        assert abs(got[(o * H + y) * W + x] - want) <= TOL * (s + abs(bias[o])), \
                            (ch.name, name)
                elif role == "RS":
                    for o in r.integers(0, Cc, 2):
                        full = OK.conv3x3_f64(X, Wt[o:o + 1])[0, 0]
                        plane = np.maximum(full + bias[o], 0).reshape(-1)
                        sc = (OK.conv3x3_abs_f64(X, Wt[o:o + 1])[0, 0] + abs(bias[o])).reshape(-1)
                        assert abs(got[o] - plane.sum()) <= TOL * sc.sum(), (ch.name, name)
            else:
                n = blk.shape[0]
                P = host(f"t{j}.pts")[: 4 * n].reshape(n, 4)
                want = OK.voxel_scatter(P)
                idx = {"VI": 0, "VC": 1, "VZ": 2, "VF": 3}[role]
                w = np.asarray(want[idx])
                g = got[: len(w)]
                assert np.array_equal(g.view(np.uint32), w.view(np.uint32)), (ch.name, name)
    return checked


def _no_set_overlap(comps, n_sets):
    by = {}
    for c in comps:
        by.setdefault((int(c["chain"]), int(c["frame"]) % n_sets), []).append(
            (int(c["t_arr_ns"]), int(c["t_done_ns"])))
    for iv in by.values():
        iv.sort()
        for (a0, d0), (a1, d1) in zip(iv, iv[1:]):
            if a1 < d0:
                return False
    return True


def _frames_per_chain(wl):
    return max(sum(1 for c, _, _ in wl.arrivals if c == ci) for ci in range(len(wl.chains)))


def test_cfg1_window_replay_and_sampled_outputs():
    wl = synth.config1(seed=0, window_s=0.3)
    n_sets = _frames_per_chain(wl)        # every frame writes its own outputs
    dw, comps, trace, est, stats, metrics = run_workload(wl, "urgency", n_sets=n_sets, th=3 * MS)
    assert len(comps) == len(wl.arrivals) and stats["trace_dropped"] == 0
    assert stats["launches"] > 10_000
    inst = T.instants_from_trace(trace)
    chains = T.oracle_chains(wl, est)
    assert des.replay(chains, oracle_cfg("urgency", th=3 * MS), inst) is None
    assert _no_set_overlap(comps, n_sets)
    assert check_cfg1_outputs(wl, dw, 0, samples=4, seed=0) >= 8


def test_cfg1_window_task_graphs_replay_and_sampled_outputs():
    wl = synth.config1(seed=2, window_s=0.3)
    n_sets = _frames_per_chain(wl)
    flags = capi.F_BIND | capi.F_DELAY | capi.F_BATCH | capi.F_ADMIT | capi.F_GRAPH
    dw, comps, trace, est, stats, metrics = run_workload(wl, "urgency", n_sets=n_sets, th=3 * MS,
                                                         flags=flags)
    assert len(comps) == len(wl.arrivals) and stats["trace_dropped"] == 0
    inst = T.instants_from_trace(trace)
    chains = T.oracle_chains(wl, est)
    assert des.replay(chains, oracle_cfg("urgency", th=3 * MS, graph=True), inst) is None
    assert check_cfg1_outputs(wl, dw, 0, samples=3, seed=1) >= 8


def test_alone_and_in_the_mix_bit_identical():
    """One frame of every cfg1 chain alone on the GPU, then the whole window
    together: every output buffer is bit-identical."""
    wl = synth.config1(seed=0, window_s=0.2)
    alone = {}
    est = None
    for c in range(len(wl.chains)):
        arr = [(c, 0, 0)]
        dw, comps, _, e, _, _ = run_workload(wl, "urgency", n_sets=1, arrivals=arr,
                                             profile=est is None, est_from=est)
        est = est or e
        alone[c] = {s: dw.output(c, s, 0).copy() for s, b in enumerate(wl.chains[c].buffers)
                    if b.role == "out"}
        del dw
        torch.cuda.empty_cache()
    n_sets = _frames_per_chain(wl)
    dw, comps, _, _, _, _ = run_workload(wl, "urgency", n_sets=n_sets, est_from=est)
    assert _no_set_overlap(comps, n_sets)
    for c in range(len(wl.chains)):
        for s, ref in alone[c].items():
            for k in range(n_sets):
                if any(cc == c and f == k for cc, f, _ in wl.arrivals):
                    assert np.array_equal(dw.output(c, s, k).view(np.uint32), ref.view(np.uint32)), \
                        (wl.chains[c].name, wl.chains[c].buffers[s].name, k)
