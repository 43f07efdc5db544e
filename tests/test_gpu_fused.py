"""Fused tails on the GPU, through the C-ABI.

* The tail executor alone (ug_tails_*): bias+ReLU bit-exact, softmax and row
  sum within 1e-5 of the oracle, on ragged tiles, long rows, per-row and
  per-column bias, in place and not, -0 / NaN inputs.
* Its service order with one worker: tiles in the oracle's order
  (oracle.fused.service_order), also after keys are rewritten.
* A tail behind a contraction that counts its wavefronts
  (ug_kernel_launch_signal): the tail reads the finished product and the
  counter is reset for the next launch.
* The gate with UG_F_FUSE on configuration 2 (BF16 contractions, private
  block outputs): every frame completes, the decision log replays through
  the oracle gate model, sampled outputs match the oracle.
"""

import time

import numpy as np
import pytest
import torch

from oracle import des
from oracle import fused as OF
from oracle import kernels as OK
from paper_2509_12207_amd import capi, runner, synth

import _trace as T
from test_gpu_gate import _frames_per_chain, check_cfg1_outputs, oracle_cfg, run_workload

pytestmark = pytest.mark.gpu
MS = 1_000_000
TOL = 1e-5


def wait_finished(q, items, timeout_s=20.0):
    t0 = time.time()
    left = list(items)
    while left:
        q.kick()
        left = [(s, p) for s, p in left if not q.finished(s, p)]
        if left and time.time() - t0 > timeout_s:
            raise AssertionError(f"{len(left)} tail items unfinished after {timeout_s} s")
        if left:
            time.sleep(0.0005)


def check_tail(x, bias, axis, y, sm, rs):
    yy, ref_sm, ref_rs = OF.tail_outputs(x, bias, axis, sm is not None, rs is not None)
    assert np.array_equal(y.view(np.uint32), yy.view(np.uint32))
    if sm is not None:
        big = ref_sm >= 1e-30
        assert np.all(np.abs(sm - ref_sm)[big] <= TOL * ref_sm[big])
        assert np.all(np.abs(sm - ref_sm)[~big] <= 1e-37)
    if rs is not None:
        r64, ra = ref_rs
        assert np.all(np.abs(rs - r64) <= TOL * ra + 1e-30)


SHAPES = [  # rows, cols, axis, softmax, rowsum, in place
    (1, 4, 0, True, True, True),
    (7, 32, 0, True, False, False),
    (300, 256, 0, True, True, True),        # several tiles, ragged last
    (64, 4096, 0, True, True, False),       # the longest fused softmax row
    (5, 65536, 1, False, True, True),       # conv planes of 256 x 256
    (130, 8192, 0, False, True, False),     # long rows, bias from global memory, row pairs
    (513, 1024, 1, False, True, False),
    (2049, 64, 1, False, False, True),
]


@pytest.mark.parametrize("R,Cn,axis,do_sm,do_rs,inplace", SHAPES)
def test_tail_executor_outputs(R, Cn, axis, do_sm, do_rs, inplace):
    r = np.random.default_rng(R * 7 + Cn)
    x = r.uniform(-1, 1, (R, Cn)).astype(np.float32)
    x.reshape(-1)[:3] = [-0.0, np.nan, 0.0]
    bias = r.uniform(-0.5, 0.5, Cn if axis == 0 else R).astype(np.float32)
    dx = torch.from_numpy(x).cuda()
    dy = dx if inplace else torch.empty_like(dx)
    db = torch.from_numpy(bias).cuda()
    dsm = torch.empty_like(dx) if do_sm else None
    drs = torch.empty(R, device="cuda") if do_rs else None
    torch.cuda.synchronize()
    q = capi.TailQueue(workers=16)
    item = q.publish(dx.data_ptr(), dy.data_ptr(), db.data_ptr(), R, Cn, axis, key=1,
                     sm=dsm.data_ptr() if do_sm else 0, rs=drs.data_ptr() if do_rs else 0)
    wait_finished(q, [item])
    q.close()
    check_tail(x, bias, axis, dy.cpu().numpy(), dsm.cpu().numpy() if do_sm else None,
               drs.cpu().numpy() if do_rs else None)


def test_tail_executor_many_items_and_slot_reuse():
    # more items than slots over time; each checked
    r = np.random.default_rng(3)
    q = capi.TailQueue(workers=64)
    for rnd in range(3):
        xs, items = [], []
        for i in range(200):
            R, Cn = int(r.integers(1, 40)), 4 * int(r.integers(1, 80))
            x = r.uniform(-1, 1, (R, Cn)).astype(np.float32)
            b = r.uniform(-1, 1, Cn).astype(np.float32)
            dx, db = torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda()
            dy, drs = torch.empty_like(dx), torch.empty(R, device="cuda")
            xs.append((x, b, dy, drs, dx, db))
            torch.cuda.synchronize()
            items.append(q.publish(dx.data_ptr(), dy.data_ptr(), db.data_ptr(), R, Cn, 0,
                                   key=int(r.integers(0, 1 << 40)), rs=drs.data_ptr()))
        wait_finished(q, items)
        for x, b, dy, drs, _, _ in xs:
            check_tail(x, b, 0, dy.cpu().numpy(), None, drs.cpu().numpy())
    # the executor leaves 0.5 ms after its last item: its statistics count
    # every item once, and at least a tile each
    time.sleep(0.2)
    st = q.stats()
    assert st["items"] == 600 and st["tiles"] >= 600 and st["rounds"] > 0
    assert st["serve_ticks"] > 0 and st["round_ticks"] > 0
    q.close()


def _order_items(q, specs):
    """Publish items (key, rows) of 8192-float rows (one worker: 16 rows per
    tile, the most a 512 KiB tile of 32 KiB rows takes); returns
    publications and tensors."""
    out = []
    for key, rows in specs:
        x = torch.rand(rows, 8192, device="cuda")
        b = torch.zeros(8192, device="cuda")
        torch.cuda.synchronize()
        slot, pub = q.publish(x.data_ptr(), x.data_ptr(), b.data_ptr(), rows, 8192, 0, key=key)
        out.append((slot, pub, x, b))
    return out


def test_tail_executor_serves_smallest_key_first():
    # one worker: the tiles come in the oracle's service order, all items
    # ready before the worker starts (paused while they are taken in)
    q = capi.TailQueue(workers=1, idle_ns=2_000_000_000, log_cap=4096)
    q.pause(True)
    specs = [(5 << 32 | 1, 40), (2 << 32 | 2, 20), (9 << 32 | 3, 60), (2 << 32 | 4, 25), (7, 36)]
    items = _order_items(q, specs)
    q.kick()
    time.sleep(0.2)
    # the gate re-ranks: the last-but-one item becomes the most urgent
    q.set_key(items[3][0], 1 << 32 | 4)
    time.sleep(0.1)
    q.pause(False)
    wait_finished(q, [(s, p) for s, p, _, _ in items])
    log = q.log()
    q.close()
    rpt = 16                               # rows per tile at 8192 floats
    keys = [k for k, _ in specs]
    keys[3] = 1 << 32 | 4
    oracle_items = [{"key": k, "tiles": -(-rows // rpt), "ready": 0}
                    for k, (_, rows) in zip(keys, specs)]
    want = OF.service_order(oracle_items)
    pub_of = {p: i for i, (_, p, _, _) in enumerate(items)}
    got = [(pub_of[e >> 24], e & 0xFFFFFF) for e in log]
    assert got == want


def test_tail_behind_a_counted_contraction():
    # FP32 GEMM 1024^3 (about 0.1 ms) then its tail: the executor may start
    # before the product is done, and must wait for the counter
    M = N = K = 1024
    r = np.random.default_rng(11)
    A = r.uniform(-1, 1, (M, K)).astype(np.float32)
    B = r.uniform(-1, 1, (K, N)).astype(np.float32)
    bias = r.uniform(-1, 1, N).astype(np.float32)
    dA, dB, db = (torch.from_numpy(v).cuda() for v in (A, B, bias))
    dC = torch.zeros(M, N, device="cuda")
    dY, dS = torch.empty_like(dC), torch.empty_like(dC)
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    q = capi.TailQueue(workers=32)
    for rep in range(3):
        waves = capi.kernel_launch_signal(
            {"op": "gemm", "shape": (M, N, K), "in": (0, 1), "out": (2,)},
            [dA.data_ptr(), dB.data_ptr(), dC.data_ptr()], cnt.data_ptr(), s.cuda_stream)
        item = q.publish(dC.data_ptr(), dY.data_ptr(), db.data_ptr(), M, N, 0, key=rep,
                         sm=dS.data_ptr(), counter=cnt.data_ptr(), target=waves)
        wait_finished(q, [item])
        s.synchronize()
        assert int(cnt.item()) == 0                       # reset for the next launch
        C = dC.cpu().numpy()
        check_tail(C, bias, 0, dY.cpu().numpy(), dS.cpu().numpy(), None)
        assert np.all(np.abs(C - OK.gemm_f64(A, B)) <= TOL * OK.gemm_abs_f64(A, B))
    q.close()


def test_tail_behind_a_counted_bf16_convolution():
    Cc, H, W = 64, 48, 40
    r = np.random.default_rng(5)
    X16 = (r.uniform(-1, 1, (H, W, Cc)).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    W16 = (r.uniform(-1, 1, (Cc, 3, 3, Cc)).astype(np.float32).view(np.uint32) >> 16).astype(
        np.uint16)
    bias = r.uniform(-1, 1, Cc).astype(np.float32)
    dx = torch.from_numpy(X16.view(np.int16)).cuda()
    dw = torch.from_numpy(W16.view(np.int16)).cuda()
    db = torch.from_numpy(bias).cuda()
    dY = torch.zeros(Cc, H * W, device="cuda")
    drs = torch.empty(Cc, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    q = capi.TailQueue(workers=8)
    waves = capi.kernel_launch_signal(
        {"op": "conv3x3_bf16", "shape": (1, Cc, H, W), "in": (0, 1), "out": (2,)},
        [dx.data_ptr(), dw.data_ptr(), dY.data_ptr()], cnt.data_ptr(), s.cuda_stream)
    item = q.publish(dY.data_ptr(), dY.data_ptr(), db.data_ptr(), Cc, H * W, 1, key=0,
                     rs=drs.data_ptr(), counter=cnt.data_ptr(), target=waves)
    wait_finished(q, [item])
    s.synchronize()
    q.close()
    ref = OK.conv3x3_bf16_f64(X16, W16)[0].reshape(Cc, H * W)
    sc = OK.conv3x3_bf16_abs_f64(X16, W16)[0].reshape(Cc, H * W)
    Yc = dY.cpu().numpy()
    want = np.maximum(ref + bias[:, None], 0)
    assert np.all(np.abs(Yc - want) <= TOL * (sc + np.abs(bias)[:, None]))
    assert np.all(np.abs(drs.cpu().numpy() - Yc.astype(np.float64).sum(1))
                  <= TOL * np.abs(Yc).astype(np.float64).sum(1))


def _signal_buffers(op, shape, r):
    if op == "gemm":
        M, N, K = shape
        return [r.uniform(-1, 1, M * K).astype(np.float32),
                r.uniform(-1, 1, K * N).astype(np.float32), np.zeros(M * N, np.float32)]
    if op == "conv3x3":
        n, Cc, H, W = shape
        return [r.uniform(-1, 1, n * Cc * H * W).astype(np.float32),
                r.uniform(-1, 1, Cc * Cc * 9).astype(np.float32),
                np.zeros(n * Cc * H * W, np.float32)]
    bf = lambda n: (r.uniform(-1, 1, n).astype(np.float32).view(np.uint32) >> 16).astype(
        np.uint16).view(np.int16)
    if op == "gemm_bf16":
        M, N, K = shape
        return [bf(M * K), bf(N * K), np.zeros(M * N, np.float32)]
    _, Cc, H, W = shape
    return [bf(H * W * Cc), bf(Cc * 9 * Cc), np.zeros(Cc * H * W, np.float32)]


@pytest.mark.parametrize("op,shape,variant", [
    ("gemm", (1024, 1024, 1024), -1),
    ("gemm", (96, 160, 2048), 2),          # K split in four: slices 1-3 leave early
    ("gemm", (200, 136, 264), 1),
    ("conv3x3", (1, 64, 24, 40), 3),       # K split in four
    ("conv3x3", (1, 32, 20, 16), 4),       # K split in four
    ("conv3x3", (1, 64, 32, 32), 0),
    ("gemm_bf16", (512, 384, 256), -1),
    ("conv3x3_bf16", (1, 64, 24, 40), -1),
])
def test_launch_signal_counts_every_wavefront(op, shape, variant):
    """The completion counter ends at exactly the wavefront count the launch
    reports, and a counted launch stores what an uncounted one does."""
    r = np.random.default_rng(hash((op, shape)) % (1 << 32))
    host = _signal_buffers(op, shape, r)
    dev = [torch.from_numpy(h).cuda() for h in host]
    out2 = torch.zeros_like(dev[2])
    cnt = torch.zeros(2, dtype=torch.int32, device="cuda")
    k = {"op": op, "shape": shape, "in": (0, 1), "out": (2,)}
    s = torch.cuda.Stream()
    if variant >= 0:
        capi.tile_set(op, shape, variant)
        assert capi.tile_get(k) == variant
    try:
        torch.cuda.synchronize()
        capi.kernel_launch(k, [dev[0].data_ptr(), dev[1].data_ptr(), out2.data_ptr()],
                           s.cuda_stream)
        for rep in range(2):
            waves = capi.kernel_launch_signal(k, [d.data_ptr() for d in dev],
                                              cnt[1:].data_ptr(), s.cuda_stream)
            s.synchronize()
            assert waves > 0 and int(cnt[1].item()) == (rep + 1) * waves
        assert int(cnt[0].item()) == 0      # the word before the counter is untouched
    finally:
        if variant >= 0:
            capi.tile_set(op, shape, -1)
    a, b = dev[2].cpu().numpy(), out2.cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_launch_signal_refuses_other_ops():
    with pytest.raises(capi.UgError):
        x = torch.zeros(16, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        capi.kernel_launch_signal({"op": "bias_relu", "shape": (4, 4, 0), "in": (0, 1),
                                   "out": (0,)}, [x.data_ptr(), x.data_ptr()], cnt.data_ptr())


FUSED = capi.F_BIND | capi.F_DELAY | capi.F_BATCH | capi.F_ADMIT | capi.F_FUSE


@pytest.mark.parametrize("policy,graph", [("urgency", False), ("fifo", False), ("urgency", True)])
def test_cfg2_window_fused_replay_and_sampled_outputs(policy, graph):
    wl = synth.config2(seed=1, window_s=0.25)
    n_sets = _frames_per_chain(wl)
    flags = (FUSED if policy == "urgency" else capi.F_FUSE) | (capi.F_GRAPH if graph else 0)
    dw, comps, trace, est, stats, metrics = run_workload(wl, policy, n_sets=n_sets, th=3 * MS,
                                                         flags=flags)
    assert len(comps) == len(wl.arrivals) and stats["trace_dropped"] == 0
    assert stats["tails_fused"] > 100 and stats["executor_launches"] >= 1
    inst = T.instants_from_trace(trace)
    chains = T.oracle_chains(wl, est)
    assert des.replay(chains, oracle_cfg(policy, th=3 * MS, graph=graph), inst) is None
    assert check_cfg1_outputs(wl, dw, 0, samples=3, seed=2) >= 8


def test_fused_task_graphs_prepared_and_run_twice():
    # graphs captured before the run (ug_graph_prepare) hold the producers'
    # counters; the same gate runs the window twice (stop, start): every
    # frame completes both times and the outputs match the oracle
    wl = synth.config2(seed=4, window_s=0.15)
    n_sets = _frames_per_chain(wl)
    dw = runner.DeviceWorkload(wl, n_sets=n_sets)
    g = runner.make_gate(wl, "urgency", trace_capacity=1 << 22, th_slack_ns=3 * MS,
                         flags=FUSED | capi.F_GRAPH)
    runner.profile(g, dw, warmup=1, reps=2)
    runner.prepare_graphs(g, dw)
    for _ in range(2):
        g.start()
        comps, _ = runner.run(g, dw, wl.arrivals)
        g.drain(60.0)
        g.stop()
        assert len(comps) == len(wl.arrivals)
        assert g.stats()["tails_fused"] > 50
    g.close()
    assert check_cfg1_outputs(wl, dw, 0, samples=2, seed=5) >= 8
