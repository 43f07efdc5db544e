"""Serving form on the GPU, through the C-ABI: per-frame kernel sizes
(ug_frame_submit_dims) against the oracle, admission against an HBM budget
(UG_EAGAIN, deferral and peak counters), and a short window of the serving
workload (20 chains, Poisson arrivals, per-frame point counts, a tight
budget) whose decision log replays through the oracle gate model."""

import numpy as np
import pytest
import torch

from oracle import des
from oracle import kernels as OK
from paper_2509_12207_amd import capi, runner, synth

import _trace as T

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
MS = 1_000_000


def _voxel_chain(nmax):
    k = {"op": "voxel", "shape": (nmax, 512, 512), "in": (0,), "out": (1, 2, 3, 4),
         "fparam": (-51.2, -51.2, 5.0), "frame_dim": 1}
    return [{"cpu_ns": 0, "kernels": [k]}]


def test_per_frame_point_counts_match_the_oracle():
    nmax = 5000
    r = np.random.default_rng(41)
    P = np.concatenate([r.normal(0, 20, (nmax, 3)), r.uniform(0, 1, (nmax, 1))], 1).astype(np.float32)
    pts = torch.from_numpy(P.reshape(-1)).to(DEV)
    G = 512 * 512
    g = capi.Gate("urgency", queue_capacity=64)
    c = g.register_chain(10 * MS, 10 * MS, _voxel_chain(nmax), 5)
    g.set_estimate(c, 0, 50_000, 1.0)
    sizes = [0, 1, 777, nmax]
    outs = [[torch.full((nmax,), 7, dtype=torch.int32, device=DEV),
             torch.full((G,), 7, dtype=torch.int32, device=DEV), torch.full((G,), 7.0, device=DEV),
             torch.full((G,), 7, dtype=torch.int32, device=DEV)] for _ in sizes]
    g.start()
    ptrs = [[int(pts.data_ptr())] + [int(t.data_ptr()) for t in o] for o in outs]
    with pytest.raises(capi.UgError) as e:
        g.submit(c, -1, ptrs[0], [nmax + 1])
    assert e.value.status == capi.EINVAL
    with pytest.raises(capi.UgError) as e:
        g.submit(c, -1, ptrs[0])                       # the chain needs per-frame sizes
    assert e.value.status == capi.EINVAL
    for n, p in zip(sizes, ptrs):
        assert g.submit(c, -1, p, [n]) is not None
    g.drain(30.0)
    comps = g.poll()
    g.stop()
    g.close()
    assert len(comps) == len(sizes)
    for n, o in zip(sizes, outs):
        vi, vc, vz, vf = (t.cpu().numpy() for t in o)
        wi, wc, wz, wf = OK.voxel_scatter(P[:n])
        assert np.array_equal(vi[:n], wi) and np.all(vi[n:] == 7)     # only n points touched
        assert np.array_equal(vc, wc) and np.array_equal(vf, wf)
        assert np.array_equal(vz.view(np.uint32), np.asarray(wz, np.float32).view(np.uint32))


def test_hbm_budget_admission():
    # footprint 100 bytes a frame, budget 150: one frame in flight at a time
    nmax = 1000
    P = np.zeros((nmax, 4), np.float32)
    pts = torch.from_numpy(P.reshape(-1)).to(DEV)
    G = 512 * 512
    bufs = [pts, torch.empty(nmax, dtype=torch.int32, device=DEV),
            torch.empty(G, dtype=torch.int32, device=DEV), torch.empty(G, device=DEV),
            torch.empty(G, dtype=torch.int32, device=DEV)]
    ptrs = [int(t.data_ptr()) for t in bufs]
    g = capi.Gate("urgency", queue_capacity=64, hbm_budget_bytes=150)
    c = g.register_chain(10 * MS, 100 * MS, _voxel_chain(nmax), 5)
    g.set_estimate(c, 0, 50_000, 1.0)
    g.set_footprint(c, 100)
    g.start()
    later = capi.now_ns() + 300 * MS           # keeps the first frame in flight meanwhile
    assert g.submit(c, later, ptrs, [nmax]) == 0
    assert g.submit(c, -1, ptrs, [nmax]) is None          # over the budget: UG_EAGAIN
    st = g.stats()
    assert st["frames_deferred"] == 1 and st["hbm_peak_bytes"] == 100
    g.drain(30.0)
    assert len(g.poll()) == 1
    assert g.submit(c, -1, ptrs, [nmax]) == 1             # admitted once the first is done
    g.drain(30.0)
    assert len(g.poll()) == 1
    st = g.stats()
    assert st["frames_deferred"] == 1 and st["hbm_peak_bytes"] == 100
    g.stop()
    with pytest.raises(capi.UgError):
        g.set_footprint(c, 10)                 # only before the first start
    g.close()


def test_serving_window_tight_budget_and_replay():
    wl = synth.config3(seed=1, window_s=0.6)
    dw = runner.DeviceWorkload(wl, n_sets=3)
    fps = [synth.footprint_bytes(ch) for ch in wl.chains]
    budget = 3 * max(fps)                      # a few frames in flight at most
    g = runner.make_gate(wl, "urgency", trace_capacity=1 << 22, th_slack_ns=3 * MS,
                         queue_capacity=1 << 14, hbm_budget_bytes=budget)
    for c, fp in enumerate(fps):
        g.set_footprint(c, fp)
    runner.profile(g, dw, warmup=1, reps=2)
    est = runner.estimates(g, wl)
    g.start()
    comps, _, deferred = runner.serve(g, dw, wl.arrivals, wl.meta["dims"], timeout_s=120.0)
    g.drain(60.0)
    g.stop()
    st = g.stats()
    trace = g.trace()
    g.close()
    assert len(comps) == len(wl.arrivals) and st["trace_dropped"] == 0
    assert st["hbm_peak_bytes"] <= budget
    assert deferred > 0 and st["frames_deferred"] >= deferred
    inst = T.instants_from_trace(trace)
    chains = T.oracle_chains(wl, est)
    cfg = {"policy": "urgency", "th_slack_ns": 3 * MS}
    assert des.replay(chains, cfg, inst) is None
