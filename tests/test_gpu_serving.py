"""Serving form on the GPU, through the C-ABI: per-frame kernel sizes
(ug_frame_submit_dims) against the oracle, admission against an HBM budget
(UG_EAGAIN, deferral and peak counters), and windows of the serving workload
(20 chains, Poisson arrivals, per-frame point counts and image sizes, gated
uploads of each frame's points from pinned host memory, device-resident
chain state): decision logs replay through the oracle gate model, every
frame's outputs match the oracle, the state is the sum over the frames, and
frames give bit-identical outputs alone and in the mix."""

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
    profs = runner.profiles(g, wl)
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
    chains = T.oracle_chains(wl, est, profs)
    cfg = {"policy": "urgency", "th_slack_ns": 3 * MS}
    assert des.replay(chains, cfg, inst) is None


# ----------------------------------------------------------------------------
def _last_writers(ch):
    last = {}
    for b in ch.blocks:
        for role, name in b.outputs.items():
            last[name] = (b, role)
    return last


def _frame_outputs(wl, dw, c, f):
    """Every output buffer of frame f of chain c (its buffer set), copied."""
    k = f % dw.n_sets
    return {s: dw.output(c, s, k).copy() for s, b in enumerate(wl.chains[c].buffers)
            if b.role == "out"}


def check_cfg3_frame(wl, dw, c, f, dims, samples=4, seed=0):
    """Outputs of frame f of chain c at its own sizes against the oracle:
    voxel outputs bit-exact on the frame's uploaded points, sampled conv
    outputs at the frame's image size (and the plane row sums), sampled
    dense outputs.  Returns the kinds of blocks checked."""
    ch = wl.chains[c]
    r = np.random.default_rng([seed, c, f])
    slot = {b.name: i for i, b in enumerate(ch.buffers)}
    k = f % dw.n_sets
    kinds = set()
    for name, (blk, role) in _last_writers(ch).items():
        j = blk.task
        if role == "STATE":
            continue
        got = dw.output(c, slot[name], k)
        if blk.kind == "voxel":
            n = dims[0]
            P = dw.frame_host_input(c, f, slot[f"t{j}.pts_host"], n)[: 4 * n].reshape(n, 4)
            want = OK.voxel_scatter(P)
            w = np.asarray(want[{"VI": 0, "VC": 1, "VZ": 2, "VF": 3}[role]])
            assert np.array_equal(got[: len(w)].view(np.uint32), w.view(np.uint32)), (ch.name, f, name)
            kinds.add("voxel")
        elif blk.kind == "conv":
            shift = next(kk.get("frame_shift", 0) for kk in
                         (ch.tasks[j]["kernels"][i] for i in blk.kernels))
            _, Cc, H, _ = blk.shape
            s = dims[1] >> shift if shift else H
            X = dw.host_input(c, slot[f"t{j}.in_x"])[: Cc * s * s].reshape(1, Cc, s, s)
            Wt = dw.host_input(c, slot[f"t{j}.in_w"])[: Cc * Cc * 9].reshape(Cc, Cc, 3, 3)
            bias = dw.host_input(c, slot[f"t{j}.bias_row"])[:Cc]
            if role == "Y":
                for o, y, x in zip(r.integers(0, Cc, samples), r.integers(0, s, samples),
                                   r.integers(0, s, samples)):
                    v, sc = OK.conv3x3_entry_f64(X, Wt, 0, o, y, x)
                    want = max(np.float32(v) + bias[o], 0)
                    assert abs(got[(o * s + y) * s + x] - want) <= 1e-5 * (sc + abs(bias[o])), \
                        (ch.name, f, name, s)
            elif role == "RS":
                o = int(r.integers(0, Cc))
                full = OK.conv3x3_f64(X, Wt[o:o + 1])[0, 0]
                plane = np.maximum(full + bias[o], 0).reshape(-1)
                sc = (OK.conv3x3_abs_f64(X, Wt[o:o + 1])[0, 0] + abs(bias[o])).reshape(-1)
                assert abs(got[o] - plane.sum()) <= 1e-5 * sc.sum(), (ch.name, f, name, s)
            kinds.add("conv")
        elif blk.kind == "dense" and role == "C":
            M, N, K = blk.shape
            A = dw.host_input(c, slot[f"t{j}.in_a"])[: M * K].reshape(M, K)
            B = dw.host_input(c, slot[f"t{j}.in_b"])[: K * N].reshape(K, N)
            bias = dw.host_input(c, slot[f"t{j}.bias_col"])[:N]
            m = int(r.integers(0, M))
            row = A[m].astype(np.float64) @ B.astype(np.float64)
            sc = np.abs(A[m]).astype(np.float64) @ np.abs(B).astype(np.float64) + np.abs(bias)
            want = OK.bias_relu_f32(row.astype(np.float32)[None, :], bias, 0)[0]
            assert np.all(np.abs(got[m * N:(m + 1) * N] - want) <= 1e-5 * sc), (ch.name, f, name)
            kinds.add("dense")
    return kinds


def _frames_per_chain(wl):
    return max(sum(1 for c, _, _ in wl.arrivals if c == ci) for ci in range(len(wl.chains)))


def _serve(wl, dw, arrivals, est=None, profs=None, **cfg):
    g = runner.make_gate(wl, "urgency", trace_capacity=1 << 22, th_slack_ns=3 * MS,
                         queue_capacity=1 << 14, **cfg)
    if est is None:
        runner.profile(g, dw, warmup=1, reps=2)
    else:
        for (c, k), (e, u) in est.items():
            g.set_estimate(c, k, e, u)
        for (c, k), pts in profs.items():
            g.set_profile(c, k, pts)
    est, profs = runner.estimates(g, wl), runner.profiles(g, wl)
    dw.reset_state()
    g.start()
    comps, _, _ = runner.serve(g, dw, arrivals, wl.meta["dims"], timeout_s=120.0)
    g.drain(60.0)
    g.stop()
    trace = g.trace()
    g.close()
    return comps, trace, est, profs


def test_cfg3_window_every_frame_state_and_replay():
    # each frame its own buffer set: every frame's outputs are checked at
    # its own point count / image size; the device-resident state of every
    # chain with a point cloud is the sum of its frames' cell counts; the
    # log (with the frames' sizes) replays through the oracle gate model,
    # whose estimates follow each frame's size
    wl = synth.config3(seed=2, window_s=0.25)
    dims = wl.meta["dims"]
    dw = runner.DeviceWorkload(wl, n_sets=_frames_per_chain(wl))
    comps, trace, est, profs = _serve(wl, dw, wl.arrivals)
    assert len(comps) == len(wl.arrivals)
    assert any(p for p in profs.values())
    kinds = set()
    for c, f, _ in wl.arrivals:
        kinds |= check_cfg3_frame(wl, dw, c, f, dims.get((c, f), [0, 0]), samples=2)
    assert kinds == {"voxel", "conv", "dense"}
    n_state = 0
    for c, ch in enumerate(wl.chains):
        for s, b in enumerate(ch.buffers):
            if b.role != "state":
                continue
            vc = ch.slot(b.name.replace("VSTATE", "VC"))
            want = np.zeros(b.n, np.int64)
            for cc, f, _ in wl.arrivals:
                if cc == c:
                    want += dw.output(c, vc, f % dw.n_sets)
            assert np.array_equal(dw.state(c, s).astype(np.int64), want), ch.name
            n_state += 1
    assert n_state >= 2
    inst = T.instants_from_trace(trace)
    assert any(len(a) > 3 for i in inst for a in i[1])       # sizes are in the log
    chains = T.oracle_chains(wl, est, profs)
    assert des.replay(chains, {"policy": "urgency", "th_slack_ns": 3 * MS}, inst) is None


def test_cfg3_frames_alone_and_in_the_mix_bit_identical():
    # a frame of each of a few chains (point clouds and camera images, of
    # their own sizes) alone on the GPU, then the whole window together:
    # every output of those frames is bit-identical
    wl = synth.config3(seed=3, window_s=0.2)
    dw = runner.DeviceWorkload(wl, n_sets=_frames_per_chain(wl))
    # chains whose frame 0 arrives in the window
    have = [c for c in wl.meta["frame_dims"] if (c, 0) in wl.meta["dims"]]
    lidar = [c for c in have if wl.meta["dims"][(c, 0)][0] > 0][:2]
    cams = [c for c in have if wl.meta["dims"][(c, 0)][1] > 0][:2]
    picks = [(c, 0) for c in lidar + cams]
    assert len(picks) == 4
    def zero_outputs():
        # a frame smaller than the registered size writes only its own part
        # of a buffer; the rest must hold the same (zero) in both runs
        for s in dw.outputs:
            for outs in s:
                for t in outs.values():
                    t.zero_()
        torch.cuda.synchronize()

    # profile first (it runs every kernel at its registered size)
    _, _, est, profs = _serve(wl, dw, [], None, None)
    alone = {}
    for c, f in picks:
        zero_outputs()
        _serve(wl, dw, [(c, f, 0)], est, profs)
        alone[(c, f)] = _frame_outputs(wl, dw, c, f)
    zero_outputs()
    comps, _, _, _ = _serve(wl, dw, wl.arrivals, est, profs)
    assert len(comps) == len(wl.arrivals)
    for (c, f), ref in alone.items():
        mix = _frame_outputs(wl, dw, c, f)
        for s, a in ref.items():
            assert np.array_equal(a.view(np.uint8), mix[s].view(np.uint8)), \
                (wl.chains[c].name, wl.chains[c].buffers[s].name)
