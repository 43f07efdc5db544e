"""Oracle model of the urgency-ordered launch gate, one decision instant at a time.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

This is the paper's GPU prioritisation (Sec. 4.4) written as a state machine
over *decision instants*.  At an instant ``t`` the gate receives inputs (frame
arrivals and observed completions of events it recorded), updates the urgency
of every active chain instance (Eq. (2), Sec. 4.2) and decides, in order of
decreasing urgency, which kernels to launch, on which stream, and which to
hold back:

* task-level stream binding with a reserved top level (Sec. 4.4.3);
* delayed launching while a more urgent, truly urgent kernel of another chain
  is active (Sec. 4.4.4), with the low-utilisation exemption;
* batched launching with batch overlap (Sec. 4.4.5): an event marks the start
  of each batch; once a batch is closed the task waits until the *previous*
  batch has finished before it launches more, and each such observation
  advances the executing-kernel index used by Eq. (2);
* the Active Kernel Buffer (Sec. 4.4.2) as the per-instance range of launched
  kernels not yet confirmed complete.

Readings where the paper is silent (each listed in the design notes):
executing-kernel index = kernels confirmed complete by an observed event;
exact rational comparison of urgencies with ties to the lower (chain, frame);
a task binds when its first kernel is actually released; the delay rule holds
a kernel only for a *more urgent* truly urgent instance of another chain;
frames of one chain run each task in arrival order, one frame per task at a
time; a CPU segment is a host-side delay before the task's kernels.  A chain
registered with deadline 0 is best-effort (the overload load): it has no
urgency (ranked below every deadline instance), is never truly urgent, its
kernels are delayable whatever their utilisation, and it is not sampled for
TH_urgent.

Decision records (tuples):
    ("COMPLETE", c, f, t_done)
    ("TSTART",   c, f, j)
    ("BIND",     c, f, j, level, lane)
    ("HOLD",     c, f, g, why)            why 0 = delayed launching, 1 = task admission
    ("EVREC",    c, f, j, kind, seq)      kind 0 = batch start, 1 = task end
    ("EXIT",     c, f, j)                 early chain exit instead of starting task j
    ("LAUNCH",   c, f, g, level, lane)
where c = chain, f = frame index within the chain, j = task, g = kernel index
within the chain (kernels of all tasks numbered in order).  For a batch-start
event ``seq`` is the batch index; for the end event it is the number of
batches of the task.
"""

from collections import deque

from fractions import Fraction

import numpy as np

from . import policy as P

START = 0
END = 1
HOLD_DELAY = 0      # held by delayed launching (Sec. 4.4.4)
HOLD_ADMIT = 1      # held by task admission (no free place among admit_tasks)


class ChainSpec:
    """A chain: deadline and ordered tasks, each a CPU segment then kernels."""

    def __init__(self, spec):
        self.deadline = int(spec["deadline_ns"])
        self.period = int(spec.get("period_ns", 0))
        # deadline 0: a best-effort chain (never urgent, always delayable,
        # ranked below every deadline instance, outside the miss ratio)
        self.best_effort = self.deadline == 0
        self.task_first = []      # first global kernel index of each task
        self.task_end = []        # one past the last global kernel index
        self.cpu = []             # CPU-segment estimate of each task (ns)
        self.est = []             # estimated time of each kernel (ns)
        self.util = []            # utilisation of each kernel (float32)
        self.fdim = []            # per-frame size index + 1 of each kernel (0: fixed)
        self.prof = []            # profile points [(v, E), ...] of each kernel, or None
        for task in spec["tasks"]:
            self.task_first.append(len(self.est))
            self.est.extend(int(e) for e in task["est_ns"])
            self.util.extend(np.float32(u) for u in task["util"])
            nk = len(task["est_ns"])
            self.fdim.extend(int(d) for d in task.get("frame_dim", [0] * nk))
            self.prof.extend(task.get("prof", [None] * nk))
            self.task_end.append(len(self.est))
            self.cpu.append(int(task.get("cpu_ns", 0)))
            assert self.task_end[-1] > self.task_first[-1], "a task needs kernels"
        self.n_tasks = len(self.task_first)
        n = len(self.est)
        # Remaining-work sums of Eq. (2): gpu_rem[g] = sum_{k >= g} E_k,
        # cpu_rem[j] = sum_{j' >= j} E^cpu_j'.
        self.gpu_rem = [0] * (n + 1)
        for g in range(n - 1, -1, -1):
            self.gpu_rem[g] = self.gpu_rem[g + 1] + self.est[g]
        self.cpu_rem = [0] * (self.n_tasks + 1)
        for j in range(self.n_tasks - 1, -1, -1):
            self.cpu_rem[j] = self.cpu_rem[j + 1] + self.cpu[j]
        # a kernel with a per-frame size and profile points is estimated per
        # frame, at that frame's size
        self.per_frame = any(d > 0 and p for d, p in zip(self.fdim, self.prof))

    def frame_estimates(self, dims):
        """E of every kernel for a frame with sizes ``dims``."""
        est = list(self.est)
        for g, (d, pts) in enumerate(zip(self.fdim, self.prof)):
            if d > 0 and pts:
                est[g] = P.profile_estimate(pts, dims[d - 1])
        return est


class Instance:
    """One chain instance (one data frame travelling through the chain)."""

    def __init__(self, c, f, t_arr, chain):
        self.c, self.f, self.t_arr = c, f, t_arr
        self.chain = chain
        self.phase = "wait"       # wait | cpu | launch | done
        self.task = -1
        self.task_t0 = None       # when the current task started (its CPU segment)
        self.cpu_ready = None
        self.i_gpu = 0            # kernels confirmed complete (executing index)
        self.i_cpu = 0            # index of the first unfinished CPU segment
        self.g_next = 0           # next kernel to release
        self.released_hi = 0      # one past the last released kernel
        self.batch = 0            # index of the open (or next) batch
        self.batch_open = False
        self.batch_sum = 0
        self.batch_first = []     # first kernel of each batch of the task
        self.waits = deque()      # events to observe, in order: (kind, seq)
        self.seen = set()         # events of the current task already observed
        self.bound = False
        self.level = None
        self.lane = None
        self.wake = None          # re-check time of a held launch (sleep loop)
        self.est = None           # this frame's estimates (per-frame sizes), else None
        self.gpu_rem = None       # their suffix sums
        self.cpu_left = 0         # CPU work of the current segment still to run (cores > 0)
        self.cpu_req = None       # when the segment asked for a core
        self.cpu_run = False      # holds a core
        self.cpu_since = None     # last time its work was credited
        self.cpu_prio = None      # CPU priority rank (1 = most urgent), Sec. 4.3
        self.held_since = None    # first hold of the current task (hold-age bound)
        self.expire = None        # while held: when the hold age reaches its bound

    @property
    def key(self):
        return (self.c, self.f)

    def in_flight(self):
        """Has Active-Kernel-Buffer entries: launched, not yet confirmed complete."""
        return self.released_hi > self.i_gpu


DEFAULT_CFG = {
    "policy": "urgency",        # "urgency" or "fifo"
    "bind": True,
    "delay": True,
    "batch": True,
    "delta_eval_ns": 500_000,   # Delta_eval = 0.5 ms (Sec. 4.4.5)
    "delay_poll_ns": 1_000_000, # 1 ms sleep loop (Sec. 4.4.4); 0 = re-check every instant
    "util_exempt": 0.1,         # kernels below this utilisation are never delayed
    "th_slack_ns": 0,           # TH_urgent as a slack; <= 0 means +infinity
    "lanes": [2, 6],            # streams per level; len = number of levels
    "calibrate": False,
    "calib_period_ns": 1_000_000,  # sample the highest urgency at most once per period
    "admit": True,              # urgency-ordered task admission (no stream priorities)
    "admit_tasks": 4,           # instances with kernels in flight before new tasks wait
    "exit": False,              # early chain exit (Sec. 4.3)
    "no_overlap": False,        # wait for a closed batch to finish (launch-sync variants)
    "key": "urgency",           # ranking order: urgency | edf | sjf | hrrn | lcuf | saedf | eqdf
    "graph": False,             # tasks launch as one graph each (configuration 2)
    "est_noise_permille": 0,    # estimate noise n: per task instance, E * (1000 + k) / 1000
    "noise_seed": 0,            #   with k uniform in [-n, n] (Sec. 6.6)
    "max_hold_ns": 0,           # hold-age bound: a task first held at t0 is not held
                                #   again from t0 + max_hold_ns on; 0 = no bound;
                                #   best-effort tasks are not bounded
    "cpu_cores": 0,             # CPU cores the CPU segments share; 0 = one each
    "cpu_prio": False,          # urgency-centric CPU scheduling (Sec. 4.3)
}


class GateModel:
    def __init__(self, chains, cfg=None):
        self.cfg = dict(DEFAULT_CFG)
        if cfg:
            self.cfg.update(cfg)
        self.chains = [c if isinstance(c, ChainSpec) else ChainSpec(c) for c in chains]
        self.urgency_policy = self.cfg["policy"] == "urgency"
        self.now = 0
        self.u_exempt = np.float32(self.cfg["util_exempt"])
        self.lanes = list(self.cfg["lanes"])
        self.n_levels = len(self.lanes)
        # FIFO launch: one stream per task of every chain.
        self.fifo_lane = []
        k = 0
        for ch in self.chains:
            self.fifo_lane.append(list(range(k, k + ch.n_tasks)))
            k += ch.n_tasks
        self.inst = {}                                 # (c, f) -> Instance
        self.slot = {}                                 # (c, j) -> frame running task j
        self.queue = {}                                # (c, j) -> frames waiting for task j
        for c, ch in enumerate(self.chains):
            for j in range(ch.n_tasks):
                self.slot[(c, j)] = None
                self.queue[(c, j)] = deque()
        self.lane_load = {(lv, ln): 0 for lv in range(self.n_levels)
                          for ln in range(self.lanes[lv])}
        self.samples = []                              # slacks for TH_urgent
        self.next_sample = None                        # earliest time of the next sample
        self.completed = []                            # (c, f, t_arr, t_done)
        self.exited = set()                            # (c, f) that left their chain
        self.last_snapshot = {}

    # ------------------------------------------------------------------
    def slack(self, inst, t):
        ch = inst.chain
        if ch.best_effort:
            return None
        gpu, cpu = self.remaining(inst)
        return P.slack_ns(t, inst.t_arr, ch.deadline, gpu, cpu)

    def remaining(self, inst):
        """Remaining GPU and CPU work of Eq. (2): the suffix sums, or, with
        estimate noise, the same sums with every task's part scaled by that
        task instance's factor (1000 + k) / 1000 (floor per task)."""
        ch = inst.chain
        rem = ch.gpu_rem if inst.gpu_rem is None else inst.gpu_rem
        n = self.cfg["est_noise_permille"]
        if n <= 0:
            return rem[inst.i_gpu], ch.cpu_rem[inst.i_cpu]
        gpu = cpu = 0
        for j in range(ch.n_tasks):
            fac = 1000 + P.noise_permille(self.cfg["noise_seed"], inst.c, inst.f, j, n)
            lo = max(inst.i_gpu, ch.task_first[j])
            if lo < ch.task_end[j]:
                gpu += (rem[lo] - rem[ch.task_end[j]]) * fac // 1000
            if j >= inst.i_cpu:
                cpu += ch.cpu[j] * fac // 1000
        return gpu, cpu

    def _start_task(self, inst, j, t, out):
        ch = inst.chain
        inst.task = j
        inst.task_t0 = t
        inst.phase = "cpu"
        inst.cpu_ready = t + ch.cpu[j]
        inst.cpu_left = ch.cpu[j]
        inst.cpu_req = t
        inst.cpu_run = False
        inst.cpu_since = None
        inst.g_next = ch.task_first[j]
        inst.released_hi = ch.task_first[j]
        inst.batch = 0
        inst.batch_open = False
        inst.batch_sum = 0
        inst.batch_first = []
        inst.seen = set()
        inst.waits = deque()
        inst.bound = False
        inst.level = inst.lane = None
        inst.wake = None
        inst.held_since = None
        inst.expire = None
        self.slot[(inst.c, j)] = inst.f
        out.append(("TSTART", inst.c, inst.f, j))

    # ------------------------------------------------------------------
    def instant(self, t, arrivals=(), evdones=()):
        """Process one decision instant.  Returns the list of decisions.

        ``arrivals``: (c, f, t_arr) of frames first seen at this instant, or
        (c, f, t_arr, dims) for a frame with per-frame sizes.
        ``evdones``: (c, f, j, kind, seq) of events observed complete.
        """
        self.now = t
        out = []
        finished = []
        # 1. inputs, in canonical order
        for a in sorted(arrivals):
            c, f, t_arr = a[:3]
            assert (c, f) not in self.inst, "frame arrives twice"
            inst = Instance(c, f, t_arr, self.chains[c])
            if inst.chain.per_frame:
                inst.est = inst.chain.frame_estimates(a[3])
                n = len(inst.est)
                inst.gpu_rem = [0] * (n + 1)
                for g in range(n - 1, -1, -1):
                    inst.gpu_rem[g] = inst.gpu_rem[g + 1] + inst.est[g]
            self.inst[(c, f)] = inst
            self.queue[(c, 0)].append(f)
        for c, f, j, kind, seq in sorted(evdones, key=lambda e: (e[0], e[1], e[2], e[4], e[3])):
            inst = self.inst[(c, f)]
            assert inst.task == j and inst.waits and inst.waits[0] == (kind, seq), \
                ("unexpected event", (c, f, j, kind, seq), list(inst.waits))
            inst.waits.popleft()
            inst.seen.add((kind, seq))
            ch = inst.chain
            if kind == START:
                # Batch `seq` has begun, so every earlier batch of the task is
                # done: the executing kernel is the first kernel of `seq`.
                inst.i_gpu = inst.batch_first[seq]
            else:
                inst.i_gpu = ch.task_end[j]
                if inst.bound and self.urgency_policy:
                    self.lane_load[(inst.level, inst.lane)] -= 1
                self.slot[(c, j)] = None
                if j == ch.n_tasks - 1:
                    inst.phase = "done"
                    finished.append(inst)
                else:
                    inst.phase = "wait"
                    self.queue[(c, j + 1)].append(f)
        for inst in sorted(finished, key=lambda i: i.key):
            out.append(("COMPLETE", inst.c, inst.f, t))
            self.completed.append((inst.c, inst.f, inst.t_arr, t))
        # 2. tasks whose predecessor (in the chain and in the frame order) is
        #    done.  With early exit, a frame whose urgency is negative when
        #    its task would start leaves the chain instead (Sec. 4.3)
        for c, ch in enumerate(self.chains):
            for j in range(ch.n_tasks):
                while self.slot[(c, j)] is None and self.queue[(c, j)]:
                    f = self.queue[(c, j)].popleft()
                    inst = self.inst[(c, f)]
                    if self._exits(inst, t):
                        out.append(("EXIT", c, f, j))
                        inst.phase = "done"
                        self.completed.append((c, f, inst.t_arr, t))
                        self.exited.add((c, f))
                        continue
                    self._start_task(inst, j, t, out)
        # 3. CPU segments that have finished
        active = sorted((i for i in self.inst.values() if i.phase != "done"),
                        key=lambda i: i.key)
        if self.cfg["cpu_cores"] > 0:
            self._cpu(t, active, any(d[0] == "TSTART" for d in out), out)
        else:
            for inst in active:
                if inst.phase == "cpu" and inst.cpu_ready <= t:
                    inst.phase = "launch"
                    inst.i_cpu = inst.task + 1
        # 4. one urgency snapshot for the whole instant (Eq. (2))
        slack = {inst.key: self.slack(inst, t) for inst in active}
        self.last_snapshot = dict(slack)
        # 5. sample the highest urgency among active kernels, periodically
        #    (Sec. 4.4.3): at the first instant at or after each sampling time
        if self.cfg["calibrate"] and (self.next_sample is None or t >= self.next_sample):
            fl = [(slack[i.key], i.key, None) for i in active
                  if i.in_flight() and not i.chain.best_effort]
            if fl:
                self.samples.append(P.rank_sort(fl)[0][0])
                self.next_sample = t + self.cfg["calib_period_ns"]
        # 6. launch requests, most urgent first
        ready = [i for i in active
                 if i.phase == "launch" and i.g_next < i.chain.task_end[i.task]
                 and not i.waits
                 and (i.wake is None or i.wake <= t or (i.expire is not None and i.expire <= t))]
        if self.urgency_policy:
            ready = self._order(ready, slack, t)
        self.n_active = sum(1 for i in active if i.in_flight())
        for inst in ready:
            self._release(inst, t, slack, active, out)
        return out

    # ------------------------------------------------------------------
    def _cpu(self, t, active, started, out):
        """CPU segments on ``cpu_cores`` cores.  Segments that held a core
        since the last instant are credited the time in between; those with
        no work left finish (the task may launch).  Without urgency-centric
        scheduling the cores serve segments first come, first served, each
        to its end.  With it (Sec. 4.3), whenever a chain starts a new CPU
        segment every active instance is ranked by urgency at that instant
        (rank 1 the most urgent), and the cores run the segments of the best
        ranks, preempting worse-ranked ones (fixed-priority FIFO scheduling:
        ties in chain, frame order).  A CPU record marks a segment taking a
        core (1) or losing it (0)."""
        cpu = [i for i in active if i.phase == "cpu"]
        for inst in cpu:
            if inst.cpu_run:
                inst.cpu_left = max(0, inst.cpu_left - (t - inst.cpu_since))
                inst.cpu_since = t
        for inst in cpu:
            if inst.cpu_left == 0:
                inst.phase = "launch"
                inst.i_cpu = inst.task + 1
                inst.cpu_run = False
        waiting = [i for i in cpu if i.phase == "cpu"]
        prio = self.urgency_policy and self.cfg["cpu_prio"]
        if prio and started:
            slack = {i.key: self.slack(i, t) for i in active}
            for r, inst in enumerate(self._order(active, slack, t)):
                inst.cpu_prio = r + 1
        k = self.cfg["cpu_cores"]
        if prio:
            want = sorted(waiting, key=lambda i: (i.cpu_prio, i.key))[:k]
        else:
            running = [i for i in waiting if i.cpu_run]
            queued = sorted((i for i in waiting if not i.cpu_run), key=lambda i: (i.cpu_req, i.key))
            want = running + queued[:max(0, k - len(running))]
        chosen = {i.key for i in want}
        for inst in waiting:
            if inst.cpu_run and inst.key not in chosen:
                inst.cpu_run = False
                out.append(("CPU", inst.c, inst.f, inst.task, 0))
        for inst in sorted(want, key=lambda i: i.key):
            if not inst.cpu_run:
                inst.cpu_run = True
                inst.cpu_since = t
                out.append(("CPU", inst.c, inst.f, inst.task, 1))

    def _exits(self, inst, t):
        """Early chain exit: UL < 0 (the slack is negative) at a task start."""
        if not (self.urgency_policy and self.cfg["exit"]) or inst.chain.best_effort:
            return False
        return self.slack(inst, t) < 0

    def _urgent(self, s):
        return P.is_truly_urgent(s, self.cfg["th_slack_ns"])

    def _before(self, a, b, slack, t):
        """True iff instance a ranks before b.  Urgency (Eq. 2) by default;
        the alternatives of the policy comparison (Sec. 6.4) otherwise, each
        with best-effort instances last and ties broken by (chain, frame):
        EDF (earliest t_arr + D), SJF (least remaining work R, the two sums
        of Eq. 2), HRRN (highest (t - t_arr + R) / R; R = 0 first), LCUF
        (lowest estimated work per frame / period; period 0 last), SAEDF and
        EQDF (earliest deadline of the current task, the chain's slack split
        equally or by work over its remaining tasks)."""
        k = self.cfg["key"]
        if k == "urgency":
            return P.more_urgent(slack[a.key], a.key, slack[b.key], b.key)
        ca, cb = a.chain, b.chain
        if ca.best_effort != cb.best_effort:
            return cb.best_effort
        if not ca.best_effort:
            ra, rb = sum(self.remaining(a)), sum(self.remaining(b))
            if k == "edf":
                va, vb = a.t_arr + ca.deadline, b.t_arr + cb.deadline
            elif k == "sjf":
                va, vb = ra, rb
            elif k == "hrrn":
                # larger ratio first: compare the negated ratios, R = 0 first
                va = (0, 0) if ra == 0 else (1, -Fraction(t - a.t_arr + ra, ra))
                vb = (0, 0) if rb == 0 else (1, -Fraction(t - b.t_arr + rb, rb))
            elif k in ("saedf", "eqdf"):
                va, vb = self._subtask_deadline(a, t), self._subtask_deadline(b, t)
            elif k == "lcuf":
                va = (1, 0) if ca.period <= 0 else (0, Fraction(ca.gpu_rem[0] + ca.cpu_rem[0], ca.period))
                vb = (1, 0) if cb.period <= 0 else (0, Fraction(cb.gpu_rem[0] + cb.cpu_rem[0], cb.period))
            else:
                raise ValueError(k)
            if va != vb:
                return va < vb
        return a.key < b.key

    def _subtask_deadline(self, inst, t):
        """Deadline of the instance's current task under the SAEDF / EQDF
        slack split (policy.subtask_deadline), from the profiled estimates
        (the frame's own with per-frame sizes): the task that has started,
        else the next one, taken as starting now."""
        ch = inst.chain
        rem = ch.gpu_rem if inst.gpu_rem is None else inst.gpu_rem
        if inst.phase in ("cpu", "launch"):
            j, t_ref = inst.task, inst.task_t0
        else:
            j, t_ref = inst.task + 1, t
        lo, hi = ch.task_first[j], ch.task_end[j]
        w_task = ch.cpu[j] + rem[lo] - rem[hi]
        w_rem = ch.cpu_rem[j] + rem[lo]
        return P.subtask_deadline(self.cfg["key"], t_ref, inst.t_arr, ch.deadline, w_task,
                                  w_rem, ch.n_tasks - j)

    def _order(self, insts, slack, t):
        from functools import cmp_to_key
        return sorted(insts, key=cmp_to_key(
            lambda a, b: -1 if self._before(a, b, slack, t) else (1 if self._before(b, a, slack, t) else 0)))

    def _blocked(self, inst, slack, active):
        """Sec. 4.4.4: another chain's truly urgent, more urgent instance is active."""
        si = slack[inst.key]
        for o in active:
            if o.c == inst.c or not o.in_flight():
                continue
            so = slack[o.key]
            if self._urgent(so) and self._before(o, inst, slack, self.now):
                return True
        return False

    def _bind(self, inst, slack, active, out):
        """Sec. 4.4.3: choose the stream of the whole task at its first launch."""
        if not self.urgency_policy:
            inst.level, inst.lane = 0, self.fifo_lane[inst.c][inst.task]
        else:
            si = slack[inst.key]
            if not self.cfg["bind"]:
                # binding switched off: every task shares the first unreserved level
                level = min(1, self.n_levels - 1)
            elif self.n_levels <= 1:
                level = 0
            elif self._urgent(si):
                level = 0
            else:
                group = [o for o in active
                         if o is not inst and o.in_flight() and not self._urgent(slack[o.key])]
                group.append(inst)
                order = self._order(group, slack, self.now)
                rank = order.index(inst) + 1
                level = P.binding_level(rank, len(order), self.n_levels)
            loads = [(self.lane_load[(level, ln)], ln) for ln in range(self.lanes[level])]
            lane = min(loads)[1]
            self.lane_load[(level, lane)] += 1
            inst.level, inst.lane = level, lane
        inst.bound = True
        out.append(("BIND", inst.c, inst.f, inst.task, inst.level, inst.lane))

    @staticmethod
    def _wait(inst, ev):
        """Wait for event ``ev`` of the instance's current task.  Every
        recorded event is observed exactly once (the runtime releases it
        when it has been seen), so waiting on one already consumed would
        never end."""
        assert ev not in inst.seen, ("wait on an event already observed", inst.key, ev)
        inst.waits.append(ev)

    def _release(self, inst, t, slack, active, out):
        ch = inst.chain
        end = ch.task_end[inst.task]
        graph = self.urgency_policy and self.cfg["graph"]
        delta = (self.cfg["delta_eval_ns"]
                 if (self.urgency_policy and self.cfg["batch"] and not graph) else None)
        max_hold = self.cfg["max_hold_ns"]
        while inst.g_next < end and not inst.waits:
            g = inst.g_next
            # hold-age bound: once the task has waited max_hold since its
            # first hold, neither delayed launching nor admission holds it
            # (best-effort tasks have no deadline to protect: never aged)
            aged = (max_hold > 0 and not ch.best_effort and inst.held_since is not None
                    and t >= inst.held_since + max_hold)
            # task graphs: the task is one launch, gated at its first kernel
            # with the largest utilisation of its kernels, never inside
            gate_here = not graph or g == ch.task_first[inst.task]
            u = max(ch.util[g:end]) if graph and gate_here else ch.util[g]
            if (self.urgency_policy and self.cfg["delay"] and gate_here and not aged
                    and (ch.best_effort or u >= self.u_exempt)
                    and self._blocked(inst, slack, active)):
                out.append(("HOLD", inst.c, inst.f, g, HOLD_DELAY))
                poll = self.cfg["delay_poll_ns"]
                inst.wake = t + poll if poll > 0 else None
                self._held(inst, t)
                return
            # task admission: a task that is not truly urgent starts only
            # while fewer than admit_tasks instances have kernels in flight
            if (self.urgency_policy and self.cfg["admit"] and not inst.bound and not aged
                    and self.n_active >= self.cfg["admit_tasks"]
                    and not self._urgent(slack[inst.key])):
                out.append(("HOLD", inst.c, inst.f, g, HOLD_ADMIT))
                inst.wake = None
                self._held(inst, t)
                return
            if not inst.bound and not inst.in_flight():
                self.n_active += 1
            inst.wake = None
            inst.expire = None
            if not inst.bound:
                self._bind(inst, slack, active, out)
            if not inst.batch_open:
                inst.batch_open = True
                inst.batch_first.append(g)
                out.append(("EVREC", inst.c, inst.f, inst.task, START, inst.batch))
            out.append(("LAUNCH", inst.c, inst.f, g, inst.level, inst.lane))
            inst.released_hi = g + 1
            inst.g_next = g + 1
            inst.batch_sum += ch.est[g] if inst.est is None else inst.est[g]
            last = g == end - 1
            # a best-effort kernel is a batch of its own: the gate decides
            # again before each of them (each is a point where deadline work
            # can overtake the background load)
            if last or (delta is not None and (ch.best_effort or inst.batch_sum > delta)):
                # the start event of a batch opened ahead (no overlap) has
                # already been waited for, before its first kernel was released
                if not (self.urgency_policy and self.cfg["no_overlap"] and inst.batch > 0):
                    self._wait(inst, (START, inst.batch))
                if last:
                    out.append(("EVREC", inst.c, inst.f, inst.task, END, inst.batch + 1))
                    self._wait(inst, (END, inst.batch + 1))
                inst.batch += 1
                inst.batch_open = False
                inst.batch_sum = 0
                if not last and self.urgency_policy and self.cfg["no_overlap"]:
                    # Launch-synchronisation variants (Sec. 6.4): the next
                    # batch's start event is recorded right behind this
                    # batch's last kernel and waited for too, so the next
                    # batch is launched only once this one has finished.
                    inst.batch_open = True
                    inst.batch_first.append(g + 1)
                    out.append(("EVREC", inst.c, inst.f, inst.task, START, inst.batch))
                    self._wait(inst, (START, inst.batch))

    def _held(self, inst, t):
        """A hold of the task at t: its first hold starts the hold age, and
        while it waits a timer fires when the age reaches its bound."""
        max_hold = self.cfg["max_hold_ns"]
        if max_hold <= 0 or inst.chain.best_effort:
            return
        if inst.held_since is None:
            inst.held_since = t
        inst.expire = inst.held_since + max_hold

    # ------------------------------------------------------------------
    def timers(self):
        """Earliest future time at which the gate must run without an input."""
        ts = []
        cores = self.cfg["cpu_cores"]
        for inst in self.inst.values():
            if inst.phase == "cpu" and cores <= 0:
                ts.append(inst.cpu_ready)
            if inst.phase == "cpu" and cores > 0 and inst.cpu_run:
                ts.append(inst.cpu_since + inst.cpu_left)
            if inst.phase == "launch" and inst.wake is not None:
                ts.append(inst.wake)
            if inst.phase == "launch" and inst.expire is not None:
                ts.append(inst.expire)
        return min(ts) if ts else None

    def due(self, t):
        """True if some timer has expired by ``t`` (a timer-only instant)."""
        nt = self.timers()
        return nt is not None and nt <= t
