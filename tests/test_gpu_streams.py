"""The stream pool comes from the caller: torch streams attached through
ug_attach_streams (the lanes of the gate, or FIFO launch's task streams), the
library-owned fallback, and the errors of the attach call."""

import ctypes as C

import pytest
import torch

from oracle import des
from paper_2509_12207_amd import capi, runner, synth

import _trace as T
from test_gpu_gate import check_cfg0_outputs, oracle_cfg

pytestmark = pytest.mark.gpu
MS = 1_000_000


def _run_cfg0(g, wl, dw, arr):
    runner.profile(g, dw, warmup=1, reps=3)
    est = runner.estimates(g, wl)
    g.start()
    comps, _ = runner.run(g, dw, arr)
    g.drain(60.0)
    g.stop()
    return comps, g.trace(), est


@pytest.mark.parametrize("policy,flags", [("urgency", None), ("fifo", 0),
                                          ("fifo", capi.F_PLACE)])
def test_cfg0_on_attached_torch_streams(policy, flags):
    wl = synth.config0(frames=6)
    arr = [(c, f, t // 10) for c, f, t in wl.arrivals]
    dw = runner.DeviceWorkload(wl, n_sets=2)
    kw = {"trace_capacity": 1 << 20, "th_slack_ns": 5 * MS}
    if flags is not None:
        kw["flags"] = flags
    g = runner.make_gate(wl, policy, **kw)
    n = g.streams_needed()
    assert n == (8 if policy == "urgency" else 6)        # lanes {2, 6}; 2 chains x 3 tasks
    streams = [torch.cuda.Stream() for _ in range(n)]
    assert all(s.priority == 0 for s in streams)
    g.attach_streams(streams)
    comps, trace, est = _run_cfg0(g, wl, dw, arr)
    assert len(comps) == len(arr)
    check_cfg0_outputs(wl, dw, 0)
    check_cfg0_outputs(wl, dw, 1)
    inst = T.instants_from_trace(trace)
    assert des.replay(T.oracle_chains(wl, est), oracle_cfg(policy), inst) is None
    g.close()
    # the streams stay the caller's: usable after the context is gone
    x = torch.ones(1024, device="cuda")
    with torch.cuda.stream(streams[0]):
        y = x * 2
    streams[0].synchronize()
    assert float(y.sum()) == 2048.0


def test_library_owned_streams_on_request():
    wl = synth.config0(frames=2)
    arr = [(c, f, t // 10) for c, f, t in wl.arrivals]
    dw = runner.DeviceWorkload(wl, n_sets=2)
    g = runner.make_gate(wl, "urgency", trace_capacity=1 << 20, th_slack_ns=5 * MS,
                         own_streams=1)
    comps, trace, est = _run_cfg0(g, wl, dw, arr)
    assert len(comps) == len(arr) and g._streams is None
    check_cfg0_outputs(wl, dw, 0)
    g.close()


def test_attach_errors():
    L = capi.lib()
    wl = synth.config0(frames=1)
    g = runner.make_gate(wl, "urgency")
    s = [torch.cuda.Stream() for _ in range(9)]
    ptr = lambda xs: capi.pointer_array([x.cuda_stream for x in xs])  # noqa: E731
    assert L.ug_attach_streams(g.h, ptr(s[:7]), 7) == capi.EINVAL      # wrong count
    assert L.ug_attach_streams(g.h, ptr(s[:7] + s[:1]), 8) == capi.EINVAL  # repeated
    assert L.ug_attach_streams(g.h, capi.pointer_array([0] * 8), 8) == capi.EINVAL
    # no streams and own_streams 0: the raw start call refuses
    assert L.ug_start(g.h) == capi.ESTATE
    assert L.ug_attach_streams(g.h, ptr(s[:8]), 8) == capi.OK
    assert L.ug_attach_streams(g.h, ptr(s[:8]), 8) == capi.ESTATE      # once per context
    g._streams = s[:8]
    g.close()
    # FIFO: the chains come first
    f = capi.Gate("fifo")
    assert L.ug_attach_streams(f.h, ptr(s[:1]), 1) == capi.ESTATE
    n = C.c_uint32()
    assert L.ug_streams_needed(f.h, C.byref(n)) == capi.OK and n.value == 0
    f.close()
