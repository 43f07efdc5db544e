"""Discrete-event drivers for the oracle gate: prediction on a device model, and replay.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``simulate`` runs ``oracle.gate.GateModel`` against a serial, non-preemptive
  device: one kernel executes at a time; every stream is a FIFO; when the
  device is free it starts the head kernel that was enqueued first (all
  streams at one hardware priority), or, with ``device_priority``, the one on
  the lowest level first.  An event recorded on a stream completes when every
  item before it on that stream has completed; the gate observes it as soon as
  it is both complete and at the head of the events its instance waits for
  (zero-latency gate).  Every decision instant is recorded, so
  the run can be replayed.
* ``replay`` re-runs a recorded sequence of instants (time, arrivals,
  observed events) through a fresh ``GateModel`` and compares its decisions
  with the recorded ones.
* ``check_log`` tests the invariants every urgency-gated log must satisfy.
"""

from collections import deque

from . import policy as P
from .gate import END, START, GateModel


class SerialDevice:
    def __init__(self, device_priority=False):
        self.streams = {}
        self.seq = 0
        self.busy = None            # (t_end, stream key, item)
        self.done_events = set()    # events completed on the device, not yet observed
        self.device_priority = device_priority
        self.trace = []             # (t_start, t_end, c, f, g)

    def enqueue(self, key, item):
        self.seq += 1
        self.streams.setdefault(key, deque()).append((self.seq, item))

    def settle(self, t):
        progressed = True
        while progressed:
            progressed = False
            for key in sorted(self.streams):
                q = self.streams[key]
                while q and q[0][1][0] == "E" and not (self.busy and self.busy[1] == key):
                    _, item = q.popleft()
                    self.done_events.add(item[1])
                    progressed = True
        if self.busy is None:
            heads = []
            for key, q in self.streams.items():
                if q and q[0][1][0] == "K":
                    prio = key[0] if self.device_priority else 0
                    heads.append((prio, q[0][0], key))
            if heads:
                _, _, key = min(heads)
                _, item = self.streams[key][0]
                _, c, f, g, dur = item
                self.busy = (t + dur, key, item)
                self.trace.append((t, t + dur, c, f, g))

    def complete(self, t):
        t_end, key, item = self.busy
        assert t_end == t
        self.streams[key].popleft()
        self.busy = None



def observable(gate, done_events):
    """Events the gate observes now: for every instance, the completed prefix
    of the events it is waiting for (the gate polls only the event at the head
    of each instance's wait list, so an event recorded at the start of a batch
    that is still open is not observed until the batch closes)."""
    obs = []
    for key in sorted(gate.inst):
        inst = gate.inst[key]
        for kind, seq in inst.waits:
            ev = (inst.c, inst.f, inst.task, kind, seq)
            if ev not in done_events:
                break
            obs.append(ev)
    return obs


def simulate(chains, cfg, arrivals, duration_of, device_priority=False,
             max_instants=2_000_000):
    """Run the gate on the serial device model.

    ``arrivals``: (c, f, t_arr) for every frame (frame indices 0, 1, ... per
    chain in arrival order), or (c, f, t_arr, dims) with per-frame sizes.  ``duration_of(c, f, g)``: the actual device time
    of kernel g of frame f of chain c (the gate itself only sees estimates).

    Returns a dict with ``instants`` (t, arrivals, evdones, decisions),
    ``completed`` (c, f, t_arr, t_done), ``trace`` (device start/end of every
    kernel) and the ``gate`` object.
    """
    gate = GateModel(chains, cfg)
    dev = SerialDevice(device_priority)
    pending = deque(sorted(arrivals, key=lambda a: (a[2], a[0], a[1])))
    bound = {}
    instants = []
    now = 0
    while len(instants) < max_instants:
        cand = []
        if pending:
            cand.append(pending[0][2])
        if dev.busy:
            cand.append(dev.busy[0])
        nt = gate.timers()
        if nt is not None:
            cand.append(nt)
        if observable(gate, dev.done_events):
            cand.append(now)
        if not cand:
            break
        t = min(cand)
        assert t >= now
        now = t
        if dev.busy and dev.busy[0] == t:
            dev.complete(t)
            dev.settle(t)
        arr = []
        while pending and pending[0][2] <= t:
            arr.append(pending.popleft())
        evs = observable(gate, dev.done_events)
        dev.done_events.difference_update(evs)
        if not (arr or evs or gate.due(t)):
            continue
        dec = gate.instant(t, arr, evs)
        instants.append((t, arr, evs, dec))
        for d in dec:
            if d[0] == "BIND":
                bound[(d[1], d[2], d[3])] = (d[4], d[5])
            elif d[0] == "EVREC":
                _, c, f, j, kind, seq = d
                dev.enqueue(bound[(c, f, j)], ("E", (c, f, j, kind, seq)))
            elif d[0] == "LAUNCH":
                _, c, f, g, level, lane = d
                dev.enqueue((level, lane), ("K", c, f, g, int(duration_of(c, f, g))))
        dev.settle(t)
    return {"instants": instants, "completed": list(gate.completed),
            "trace": dev.trace, "gate": gate}


def replay(chains, cfg, instants):
    """Re-run recorded instants; return None if every decision matches, else
    (index, expected_decisions, recorded_decisions)."""
    gate = GateModel(chains, cfg)
    for idx, (t, arr, evs, dec) in enumerate(instants):
        got = gate.instant(t, arr, evs)
        if list(got) != list(dec):
            return idx, got, list(dec)
    return None


def check_log(chains, cfg, instants):
    """Invariants of an urgency-gated decision log (raises AssertionError).

    1. Within an instant, instances are served in order of decreasing urgency:
       the sequence of instances as they first launch or are held never
       places a less urgent instance before a more urgent one.
    2. The reserved top level is bound only to truly urgent instances.
    3. Each task's launches form consecutive kernel indices, split into
       batches exactly as the Delta_eval rule partitions them.
    4. Every frame's kernels are launched in chain order.
    """
    model = GateModel(chains, cfg)
    cfg = model.cfg
    launched = {}
    batches = {}
    for t, arr, evs, dec in instants:
        got = model.instant(t, arr, evs)
        assert got == list(dec)
        snap = model.last_snapshot
        order = []
        for d in dec:
            if d[0] in ("LAUNCH", "HOLD"):
                k = (d[1], d[2])
                if k not in order:
                    order.append(k)
            if d[0] == "BIND" and d[4] == 0 and cfg["bind"] and len(cfg["lanes"]) > 1:
                assert P.is_truly_urgent(snap[(d[1], d[2])], cfg["th_slack_ns"]), d
            if d[0] == "LAUNCH":
                _, c, f, g, _, _ = d
                prev = launched.get((c, f), -1)
                assert g == prev + 1, ("out of order", d)
                launched[(c, f)] = g
                batches.setdefault((c, f), [[]])[-1].append(g)
            if d[0] == "EVREC" and d[4] == START:
                bl = batches.setdefault((d[1], d[2]), [[]])
                if bl[-1]:
                    bl.append([])
        for a, b in zip(order, order[1:]):
            assert not P.more_urgent(snap[b], b, snap[a], a), ("release order", t, a, b)
    # batch partition per task
    for (c, f), bl in batches.items():
        ch = model.chains[c]
        est = model.inst[(c, f)].est or ch.est     # the frame's own estimates, if any
        bl = [b for b in bl if b]
        for j in range(ch.n_tasks):
            lo, hi = ch.task_first[j], ch.task_end[j]
            got = [[g - lo for g in b] for b in bl if b and lo <= b[0] < hi]
            if not got:
                continue
            delta = cfg["delta_eval_ns"] if cfg["batch"] else None
            if delta is not None and ch.best_effort:
                want = [[i] for i in range(hi - lo)]   # one kernel per batch
            else:
                want = P.batch_partition(est[lo:hi], delta)
            assert got == want[:len(got)], ("batches", c, f, j, got, want)
    return True
