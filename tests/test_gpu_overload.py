"""The overload case: a best-effort chain of FP8 products split into row
bands (each band a kernel of its own, a separate gated launch) beside the
deadline chains, through the gate on the GPU."""

import numpy as np
import pytest
import torch

from oracle import des
from oracle import kernels as OK
from paper_2509_12207_amd import capi, runner, synth

import _trace as T
from test_gpu_gate import oracle_cfg
from test_gpu_kernels import _fp8_codes, fp8_bound

pytestmark = pytest.mark.gpu
MS = 1_000_000


def test_fp8_row_bands_equal_the_whole_product():
    # rows m0 .. m0 + M of C from the same rows of A: four bands of 256 rows
    # give exactly the whole product (every element is computed by the same
    # instructions in the same order), on the ring path (K % 64 == 0) and on
    # the other one
    r = np.random.default_rng(5)
    for K in (512, 528):
        A8, B8 = _fp8_codes(r, (1024, K)), _fp8_codes(r, (384, K))
        a = torch.from_numpy(A8).cuda()
        b = torch.from_numpy(B8).cuda()
        whole = torch.full((1024, 384), float("nan"), device="cuda")
        bands = torch.full((1024, 384), float("nan"), device="cuda")
        capi.kernel_launch({"op": "gemm_fp8", "shape": (1024, 384, K), "in": (0, 1), "out": (2,)},
                           [a.data_ptr(), b.data_ptr(), whole.data_ptr()])
        for i in range(4):
            capi.kernel_launch({"op": "gemm_fp8", "shape": (256, 384, K, 256 * i), "in": (0, 1),
                                "out": (2,)}, [a.data_ptr(), b.data_ptr(), bands.data_ptr()])
        torch.cuda.synchronize()
        assert torch.equal(whole, bands)
        rows = [0, 255, 256, 700, 1023]
        C = bands.cpu().numpy()[rows]
        ref = OK.gemm_fp8_f64(A8[rows], B8)
        assert np.all(np.abs(C - ref) <= fp8_bound(A8[rows], B8))


def test_cfg4_window_best_effort_bands_through_the_gate():
    # the eleven deadline chains plus the closed-loop best-effort chain of
    # 8192^3 FP8 products, each split into four row bands, for a short
    # window: every frame completes, the log replays through the oracle gate
    # model (best-effort kernels are batches of their own and always
    # delayable), and the best-effort product is within the FP8 bound
    wl = synth.config4(seed=0, window_s=0.3, be_chunks=4)
    c_be = wl.meta["be_chain"]
    n_sets = 2
    dw = runner.DeviceWorkload(wl, n_sets=n_sets)
    g = runner.make_gate(wl, "urgency", trace_capacity=1 << 22, th_slack_ns=3 * MS,
                         queue_capacity=1 << 14)
    runner.profile(g, dw, warmup=1, reps=3)
    est = runner.estimates(g, wl)
    g.start()
    comps, _ = runner.run(g, dw, wl.arrivals, be=(c_be, wl.meta["be_depth"], 200 * MS))
    g.drain(60.0)
    g.stop()
    trace = g.trace()
    st = g.stats()
    g.close()
    n_be = int(np.count_nonzero(comps["chain"] == c_be))
    assert len(comps) == len(wl.arrivals) + n_be and n_be >= 2
    assert st["trace_dropped"] == 0
    assert not np.any(comps["missed"][comps["chain"] == c_be])
    inst = T.instants_from_trace(trace)
    chains = T.oracle_chains(wl, est)
    cfg = oracle_cfg("urgency", th=3 * MS)
    assert des.replay(chains, cfg, inst) is None
    des.check_log(chains, cfg, inst)
    # each best-effort band is a batch of its own (its own start event)
    starts = sum(1 for i in inst for d in i[3] if d[0] == "EVREC" and d[1] == c_be and d[4] == 0)
    bands = sum(1 for i in inst for d in i[3] if d[0] == "LAUNCH" and d[1] == c_be)
    assert starts == bands > 0
    # sampled entries of the product, every band represented
    ch = wl.chains[c_be]
    slot = {b.name: i for i, b in enumerate(ch.buffers)}
    d = wl.meta["be_dim"]
    A8 = dw.host_input(c_be, slot["A8"]).reshape(d, d)
    B8 = dw.host_input(c_be, slot["Bt8"]).reshape(d, d)
    C = dw.outputs[c_be][0][slot["C"]].view(d, d)
    r = np.random.default_rng(3)
    rows = np.sort(np.concatenate([r.integers(i * d // 4, (i + 1) * d // 4, 2) for i in range(4)]))
    cols = np.sort(r.integers(0, d, 24))
    got = C[torch.as_tensor(rows, device=C.device)][:, torch.as_tensor(cols, device=C.device)]
    got = got.cpu().numpy()
    ref = OK.gemm_fp8_f64(A8[rows], B8[cols])
    assert np.all(np.abs(got - ref) <= fp8_bound(A8[rows], B8[cols]))
