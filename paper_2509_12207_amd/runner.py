"""Drive a synthetic workload through libug on torch-allocated device memory.

Torch provides device memory (and pinned host memory for per-frame
inputs) only; every kernel, copy and scheduling decision runs in libug.
Read-only inputs are uploaded once per chain; outputs and per-frame host
inputs come in ``n_sets`` copies and frame f of a chain uses copy
f % n_sets; device-resident chain state is one buffer per chain.
"""

import os
import time

import numpy as np

from . import capi, synth


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the HIP path cannot run")
    return torch


class DeviceWorkload:
    def __init__(self, wl, device="cuda:0", n_sets=2):
        torch = _torch()
        self.wl = wl
        self.device = torch.device(device)
        self.n_sets = n_sets
        self.inputs = []          # per chain: {slot: tensor} (read-only and state)
        self.outputs = []         # per chain: [ {slot: tensor} per set ] (outputs, host inputs)
        self.ptrs = []            # per chain: [ [ptr per slot] per set ]
        dts = {"f32": torch.float32, "i32": torch.int32, "u8": torch.uint8, "bf16": torch.int16}
        for c, ch in enumerate(wl.chains):
            ins = {}
            for s, b in enumerate(ch.buffers):
                if b.role == "in":
                    host = synth.input_array(wl.seed, c, s, b)
                    ins[s] = torch.from_numpy(host).to(self.device)
                elif b.role == "state":
                    ins[s] = torch.zeros(b.n, dtype=dts[b.kind], device=self.device)
            sets = []
            for _ in range(n_sets):
                outs = {}
                for s, b in enumerate(ch.buffers):
                    if b.role == "out":
                        outs[s] = torch.zeros(b.n, dtype=dts[b.kind], device=self.device)
                    elif b.role == "host":
                        outs[s] = torch.zeros(b.n, dtype=dts[b.kind], pin_memory=True)
                sets.append(outs)
            self.inputs.append(ins)
            self.outputs.append(sets)
            self.ptrs.append([[int((ins.get(s) if s in ins else sets[k][s]).data_ptr())
                               for s in range(len(ch.buffers))] for k in range(n_sets)])
        torch.cuda.synchronize(self.device)

    def load_frame(self, c, f, dims=None):
        """Write frame f's own host inputs into its buffer set (before it is
        submitted; the set must not hold an unfinished frame)."""
        ch = self.wl.chains[c]
        k = f % self.n_sets
        for s, b in enumerate(ch.buffers):
            if b.role == "host":
                n = dims[0] if dims else None
                self.outputs[c][k][s].numpy()[:] = synth.frame_input(self.wl.seed, c, f, s, b, n)

    def frame_host_input(self, c, f, slot, n=None):
        return synth.frame_input(self.wl.seed, c, f, slot, self.wl.chains[c].buffers[slot], n)

    def state(self, c, slot):
        return self.inputs[c][slot].cpu().numpy()

    def reset_state(self):
        """Zero every chain's device-resident state."""
        for c, ch in enumerate(self.wl.chains):
            for s, b in enumerate(ch.buffers):
                if b.role == "state":
                    self.inputs[c][s].zero_()
        import torch
        torch.cuda.synchronize(self.device)

    def host_input(self, c, slot):
        return synth.input_array(self.wl.seed, c, slot, self.wl.chains[c].buffers[slot])

    def output(self, c, slot, k=0):
        return self.outputs[c][k][slot].cpu().numpy()

    def nbytes(self):
        """Device bytes (pinned host inputs are not counted)."""
        tot = 0
        for ins, sets in zip(self.inputs, self.outputs):
            tot += sum(t.numel() * t.element_size() for t in ins.values())
            tot += sum(t.numel() * t.element_size() for s in sets for t in s.values() if t.is_cuda)
        return tot


# the tile-variant table the autotuner measured for the FP32 GEMM and
# convolution shapes of configuration 1 (three seeds) on gfx950
TILE_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles_gfx950.txt")


def make_gate(wl, policy="urgency", device=0, **cfg):
    """A gate with ``wl``'s chains registered; the package's tile table
    unless ``tile_table`` is given (None: the launchers' rules)."""
    if "tile_table" not in cfg and os.path.exists(TILE_TABLE):
        cfg["tile_table"] = TILE_TABLE
    if cfg.get("tile_table") is None:
        cfg.pop("tile_table", None)
        capi.tile_clear()   # the table is process-wide
    g = capi.Gate(policy=policy, device=device, **cfg)
    for ch in wl.chains:
        g.register_chain(ch.period_ns, ch.deadline_ns, ch.tasks, len(ch.buffers))
    return g


def prepare_graphs(g, dw):
    """Capture every task graph of every chain for every buffer set before
    the run (UG_F_GRAPH), so no capture lands inside a frame's latency
    (workloads without per-frame sizes)."""
    for c in range(len(dw.wl.chains)):
        for k in range(dw.n_sets):
            g.prepare_graphs(c, dw.ptrs[c][k])


def profile(g, dw, warmup=3, reps=10):
    for c in range(len(dw.wl.chains)):
        g.profile(c, dw.ptrs[c][0], warmup=warmup, reps=reps)


def copy_estimates(src, dst, wl):
    """Give ``dst`` the estimates (and per-frame profile points) profiled on
    ``src`` (same chains)."""
    for c, ch in enumerate(wl.chains):
        ks = [k for t in ch.tasks for k in t["kernels"]]
        for i, k in enumerate(ks):
            e, u = src.get_estimate(c, i)
            dst.set_estimate(c, i, e, u)
            if k.get("frame_dim", 0):
                dst.set_profile(c, i, src.get_profile(c, i))


def estimates(g, wl):
    out = {}
    for c, ch in enumerate(wl.chains):
        n = sum(len(t["kernels"]) for t in ch.tasks)
        for k in range(n):
            out[(c, k)] = g.get_estimate(c, k)
    return out


def profiles(g, wl):
    """Profile points of every kernel with a per-frame size."""
    out = {}
    for c, ch in enumerate(wl.chains):
        ks = [k for t in ch.tasks for k in t["kernels"]]
        for i, k in enumerate(ks):
            if k.get("frame_dim", 0):
                out[(c, i)] = g.get_profile(c, i)
    return out


def serve(g, dw, arrivals, dims=None, lead_ns=20_000_000, timeout_s=120.0):
    """Serving driver: every frame is submitted when its arrival time comes
    (not ahead), with its chain's buffer sets taken round robin (frame f
    uses set f % n_sets; the gate numbers the frames it is given in its own
    order).  A frame whose buffer set still holds an earlier
    frame, or that the gate refuses with UG_EAGAIN (HBM budget, queue), waits
    in a FIFO queue and is retried whenever completions come back; frames of
    one chain are submitted in arrival order.  The submitted t_arr stays the
    arrival time, so the wait counts in the frame's latency.  ``dims`` maps
    (chain, frame) to the frame's per-frame sizes.  Returns (completions,
    t0, deferrals), deferrals = submissions refused at least once."""
    from collections import deque
    t0 = capi.now_ns() + lead_ns
    todo = deque(sorted(arrivals, key=lambda a: (a[2], a[0], a[1])))
    waitq = []
    busy = set()
    deferred = set()
    ours = {}            # (chain, frame index given by the gate) -> workload frame
    done, n_done = [], 0
    deadline = time.time() + timeout_s + (max(t for _, _, t in arrivals) / 1e9 if arrivals else 0)
    while n_done < len(arrivals):
        now = capi.now_ns()
        while todo and t0 + todo[0][2] <= now:
            waitq.append(todo.popleft())
        blocked = set()
        keep = []
        for c, f, t in waitq:
            key = (c, f % dw.n_sets)
            if c in blocked or key in busy:
                blocked.add(c)
                keep.append((c, f, t))
                continue
            d = None if dims is None else dims.get((c, f))
            dw.load_frame(c, f, d)
            fid = g.submit(c, t0 + t, dw.ptrs[c][f % dw.n_sets], d)
            if fid is None:                  # over the HBM budget: retry later
                deferred.add((c, f))
                blocked.add(c)
                keep.append((c, f, t))
                continue
            ours[(c, fid)] = f
            busy.add(key)
        waitq = keep
        got = g.poll()
        if len(got):
            done.append(got)
            n_done += len(got)
            for r in got:
                c = int(r["chain"])
                busy.discard((c, ours.pop((c, int(r["frame"]))) % dw.n_sets))
        elif time.time() > deadline:
            raise TimeoutError(f"{n_done} of {len(arrivals)} frames completed")
        elif not todo or t0 + todo[0][2] > capi.now_ns() + 200_000:
            time.sleep(0.0002)
    out = np.concatenate(done) if done else np.zeros(0, capi.COMPLETION_DTYPE)
    return out, t0, len(deferred)


def run(g, dw, arrivals, lead_ns=20_000_000, timeout_s=120.0, progress=None, be=None):
    """Submit every arrival (offsets relative to a start time ``lead_ns``
    from now), wait for all completions and return them.  The gate must be
    started; it is left running.

    ``be = (chain, depth, window_ns)`` adds a closed-loop best-effort source:
    ``depth`` frames of ``chain`` are submitted at the start time and each of
    their completions submits the next frame at once, until ``window_ns``
    after the start time."""
    t0 = capi.now_ns() + lead_ns
    for c, f, t in arrivals:
        fid = g.submit(c, t0 + t, dw.ptrs[c][f % dw.n_sets])
        if fid is None:
            raise RuntimeError("submission queue full")
    n_be = 0
    if be is not None:
        c_be, depth, win = be
        for _ in range(depth):
            if g.submit(c_be, t0, dw.ptrs[c_be][n_be % dw.n_sets]) is None:
                raise RuntimeError("submission queue full")
            n_be += 1
    done = []
    n_done = 0
    deadline = time.time() + timeout_s + (max(t for _, _, t in arrivals) / 1e9 if arrivals else 0)
    while n_done < len(arrivals) + n_be:
        got = g.poll()
        if len(got):
            done.append(got)
            n_done += len(got)
            if be is not None:
                for _ in range(int(np.count_nonzero(got["chain"] == c_be))):
                    if capi.now_ns() < t0 + win:
                        if g.submit(c_be, -1, dw.ptrs[c_be][n_be % dw.n_sets]) is None:
                            raise RuntimeError("submission queue full")
                        n_be += 1
        elif time.time() > deadline:
            raise TimeoutError(f"{n_done} of {len(arrivals) + n_be} frames completed")
        else:
            time.sleep(0.002)
    out = np.concatenate(done) if done else np.zeros(0, capi.COMPLETION_DTYPE)
    return out, t0
