"""C-ABI semantics on the GPU: state errors, queue capacity, drain timeout,
profiling results, calibration threshold and Eq. (3) metrics against the
oracle, and run-to-run bit identity of the outputs."""

from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import policy as OP
from paper_2509_12207_amd import capi, runner, synth

pytestmark = pytest.mark.gpu
MS = 1_000_000


def small_gate(wl, **kw):
    g = runner.make_gate(wl, "urgency", **kw)
    return g


def test_state_errors_and_queue_capacity():
    wl = synth.config0(frames=1)
    dw = runner.DeviceWorkload(wl, n_sets=1)
    g = small_gate(wl, queue_capacity=2)
    with pytest.raises(capi.UgError) as e:
        g.submit(0, -1, dw.ptrs[0][0])
    assert e.value.status == capi.ESTATE                      # not started
    g.start()
    with pytest.raises(capi.UgError) as e:
        g.start()
    assert e.value.status == capi.ESTATE
    with pytest.raises(capi.UgError) as e:
        g.register_chain(MS, MS, wl.chains[0].tasks, len(wl.chains[0].buffers))
    assert e.value.status == capi.ESTATE
    with pytest.raises(capi.UgError) as e:
        g.submit(0, -1, dw.ptrs[0][0][:-1])                   # wrong buffer count
    assert e.value.status == capi.EINVAL
    far = capi.now_ns() + 30 * 1000 * MS                      # arrives in 30 s
    assert g.submit(0, far, dw.ptrs[0][0]) == 0
    assert g.submit(1, far, dw.ptrs[1][0]) == 0
    assert g.submit(0, far, dw.ptrs[0][0]) is None            # UG_EAGAIN: capacity 2
    with pytest.raises(capi.UgError) as e:
        g.drain(0.05)
    assert e.value.status == capi.ETIMEDOUT
    g.stop()
    g.close()


def test_profile_estimates_and_utilisation():
    wl = synth.config0(frames=1)
    dw = runner.DeviceWorkload(wl, n_sets=1)
    g = small_gate(wl)
    runner.profile(g, dw, warmup=1, reps=5)
    est = runner.estimates(g, wl)
    for (c, k), (e, u) in est.items():
        assert 0 < e < 10 * MS
        assert 0.0 < u <= 1.0
    # equal (op, shape) kernels share one measurement
    assert est[(0, 0)][0] == est[(0, 4)][0] == est[(0, 8)][0]
    g.close()


def test_calibration_threshold_and_metrics_match_oracle():
    wl = synth.config1(seed=3, window_s=0.4)
    dw = runner.DeviceWorkload(wl, n_sets=4)
    g = small_gate(wl, flags=capi.F_BIND | capi.F_BATCH | capi.F_CALIBRATE, th_slack_ns=0,
                   queue_capacity=1 << 14)
    runner.profile(g, dw, warmup=1, reps=3)
    g.start()
    comps, _ = runner.run(g, dw, wl.arrivals)
    g.drain(60.0)
    g.stop()
    samples = g.calibration_samples()
    assert len(samples) > 50
    assert g.calibration_threshold(95) == OP.threshold_from_samples(samples)
    assert g.calibration_threshold(50) == OP.threshold_from_samples(samples, 50)
    m = g.metrics()
    per = {}
    for c in comps:
        m_, n_ = per.get(int(c["chain"]), (0, 0))
        per[int(c["chain"])] = (m_ + int(c["missed"]), n_ + 1)
    assert abs(m["miss_ratio"] - float(OP.overall_miss_ratio(per))) < 1e-12
    lat = [int(x) for x in comps["latency_ns"]]
    assert m["p50_ns"] == OP.percentile_nearest_rank(lat, 50)
    assert m["p99_ns"] == OP.percentile_nearest_rank(lat, 99)
    assert m["frames"] == len(lat) == len(wl.arrivals)
    g.close()


def test_two_runs_bit_identical():
    wl = synth.config0(frames=2)
    outs = []
    for _ in range(2):
        dw = runner.DeviceWorkload(wl, n_sets=2)
        g = small_gate(wl)
        runner.profile(g, dw, warmup=1, reps=2)
        g.start()
        arr = [(c, f, t // 20) for c, f, t in wl.arrivals]
        runner.run(g, dw, arr)
        g.drain(30.0)
        g.stop()
        g.close()
        outs.append({(c, s, k): dw.output(c, s, k).copy() for c, ch in enumerate(wl.chains)
                     for s, b in enumerate(ch.buffers) if b.role == "out" for k in range(2)})
        del dw
        torch.cuda.empty_cache()
    for key in outs[0]:
        assert np.array_equal(outs[0][key].view(np.uint32), outs[1][key].view(np.uint32)), key


def test_early_exit_frames_complete_as_missed():
    # deadlines of 1 us, far below the chains' profiled work: with early
    # exit every frame leaves its chain at its first task start (negative
    # urgency) and completes as missed and exited, outside the latencies
    wl = synth.config0(frames=2)
    dw = runner.DeviceWorkload(wl, n_sets=1)
    g = capi.Gate("urgency", flags=capi.F_BIND | capi.F_DELAY | capi.F_BATCH | capi.F_EXIT,
                  queue_capacity=64)
    for ch in wl.chains:
        g.register_chain(ch.period_ns, 1000, ch.tasks, len(ch.buffers))
    runner.profile(g, dw, warmup=1, reps=2)
    g.start()
    comps, _ = runner.run(g, dw, [(c, f, t // 20) for c, f, t in wl.arrivals])
    g.drain(30.0)
    g.stop()
    assert len(comps) == len(wl.arrivals)
    assert np.all(comps["exited"] == 1) and np.all(comps["missed"] == 1)
    m = g.metrics()
    assert m["miss_ratio"] == 1.0 and m["frames"] == 0
    g.close()
