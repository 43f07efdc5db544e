"""Pins of the oracle gate model and its discrete-event drivers.

Hand timelines (closed forms), brute force over every execution order on
tiny instances, the Jackson special case, a pinned counterexample that keeps
the policy least-laxity rather than earliest-deadline, and invariants on
randomised runs.
"""

import itertools

import numpy as np
import pytest

from oracle import brute, des
from oracle import policy as P
from oracle.gate import END, HOLD_ADMIT, START, GateModel

MS = 1_000_000
US = 1_000


def chain(deadline, tasks):
    """tasks: list of (cpu_ns, [(est_ns, util), ...])."""
    return {"deadline_ns": deadline,
            "tasks": [{"cpu_ns": cpu, "est_ns": [e for e, _ in ks], "util": [u for _, u in ks]}
                      for cpu, ks in tasks]}


def by_est(chains):
    """Device durations equal to the estimates."""
    def d(c, f, g):
        est = [e for t in chains[c]["tasks"] for e in t["est_ns"]]
        return est[g]
    return d


# ------------------------------------------------------------------ T1
def test_T1_slack_after_first_batch_is_confirmed():
    ch = [chain(10 * MS, [(0, [(2 * MS, 1.0), (3 * MS, 1.0), (1 * MS, 1.0)])])]
    actual = [int(2.5 * MS), 3 * MS, 1 * MS]
    cfg = {"policy": "urgency", "delta_eval_ns": 500 * US}
    res = des.simulate(ch, cfg, [(0, 0, 0)], lambda c, f, g: actual[g])
    # instant at 2.5 ms observes the start of batch 1 (kernel 1): kernel 0 is done
    snaps = {}
    model = GateModel(ch, cfg)
    for t, arr, evs, dec in res["instants"]:
        model.instant(t, arr, evs)
        snaps[t] = model.last_snapshot.get((0, 0))
    assert snaps[0] == 4 * MS
    assert snaps[int(2.5 * MS)] == int(3.5 * MS)
    # frame completes when the last kernel does: 2.5 + 3 + 1 ms
    assert res["completed"] == [(0, 0, 0, int(6.5 * MS))]


# ------------------------------------------------------------------ T2 on the gate
def test_T2_batches_and_overlap_on_gate():
    est = [200 * US, 200 * US, 200 * US, 100 * US, 600 * US, 50 * US]
    ch = [chain(100 * MS, [(0, [(e, 1.0) for e in est])])]
    cfg = {"policy": "urgency", "delta_eval_ns": 500 * US}
    res = des.simulate(ch, cfg, [(0, 0, 0)], by_est(ch))
    dec = [d for _, _, _, ds in res["instants"] for d in ds]
    seq = [(d[0], d[5] if d[0] == "EVREC" else d[3]) for d in dec if d[0] in ("EVREC", "LAUNCH")]
    assert seq == [("EVREC", 0), ("LAUNCH", 0), ("LAUNCH", 1), ("LAUNCH", 2),
                   ("EVREC", 1), ("LAUNCH", 3), ("LAUNCH", 4),
                   ("EVREC", 2), ("LAUNCH", 5), ("EVREC", 3)]
    # batch 2 is launched when batch 0 is done (start event of batch 1 observed)
    t_b2 = [t for t, _, _, ds in res["instants"] if any(d[0] == "LAUNCH" and d[3] == 5 for d in ds)]
    assert t_b2 == [600 * US]
    des.check_log(ch, cfg, res["instants"])


# ------------------------------------------------------------------ launch-synchronisation modes
def _launch_times(res):
    return {d[3]: t for t, _, _, ds in res["instants"] for d in ds if d[0] == "LAUNCH"}


@pytest.mark.parametrize("mode", ["overlap", "sync_batched", "sync", "async"])
def test_launch_synchronisation_modes(mode):
    # the T2 chain: kernels of 200, 200, 200, 100, 600, 50 us on an idle
    # device, Delta_eval = 0.5 ms.  Batches {0,1,2}, {3,4}, {5}.
    #   overlap (the paper's):   batch b+1 goes out when batch b starts
    #   synchronous batched:     ... when batch b has finished
    #   synchronous:             every kernel is a batch, each waits for the last
    #   asynchronous:            the whole task at once, one end event
    est = [200 * US, 200 * US, 200 * US, 100 * US, 600 * US, 50 * US]
    ch = [chain(100 * MS, [(0, [(e, 1.0) for e in est])])]
    cfg = {"policy": "urgency", "delta_eval_ns": 500 * US,
           "overlap": {}, "sync_batched": {"no_overlap": True},
           "sync": {"no_overlap": True, "delta_eval_ns": 0}, "async": {"batch": False}}[mode]
    cfg = dict({"policy": "urgency", "delta_eval_ns": 500 * US}, **cfg)
    res = des.simulate(ch, cfg, [(0, 0, 0)], by_est(ch))
    want = {"overlap": [0, 0, 0, 0, 0, 600],
            "sync_batched": [0, 0, 0, 600, 600, 1300],
            "sync": [0, 200, 400, 600, 700, 1300],
            "async": [0, 0, 0, 0, 0, 0]}[mode]
    got = _launch_times(res)
    assert [got[g] for g in range(6)] == [w * US for w in want]
    # the serial device finishes the frame at the same time in every mode
    assert res["completed"] == [(0, 0, 0, 1350 * US)]
    dec = [d for _, _, _, ds in res["instants"] for d in ds]
    n_start = sum(1 for d in dec if d[0] == "EVREC" and d[4] == START)
    assert n_start == {"overlap": 3, "sync_batched": 3, "sync": 6, "async": 1}[mode]
    des.check_log(ch, cfg, res["instants"])


def test_every_event_is_waited_for_once():
    # a wait on an event that was already observed would never end on the
    # device (the runtime releases an event once seen): the model refuses it
    model = GateModel([chain(10 * MS, [(0, [(100 * US, 1.0)])])], {"policy": "urgency"})
    model.instant(0, [(0, 0, 0)], [])
    inst = model.inst[(0, 0)]
    inst.seen.add((START, 5))
    with pytest.raises(AssertionError):
        GateModel._wait(inst, (START, 5))


# ------------------------------------------------------------------ alternative orders
@pytest.mark.parametrize("key,want", [
    # three chains, one one-kernel task each, all arriving at t = 0 on an idle
    # device (nobody truly urgent, so every request launches at once in rank
    # order):   A: D 10 ms, E 6 ms, P 100 ms  -> slack 4, deadline 10, util 0.06
    #           B: D  8 ms, E 1 ms, P  10 ms  -> slack 7, deadline  8, util 0.1
    #           C: D 20 ms, E 15 ms, P 500 ms -> slack 5, deadline 20, util 0.03
    ("urgency", [0, 2, 1]),   # least slack first (highest 1/slack)
    ("edf", [1, 0, 2]),       # earliest t_arr + D
    ("sjf", [1, 0, 2]),       # least remaining work
    ("lcuf", [2, 0, 1]),      # lowest E / P
    ("hrrn", [0, 1, 2]),      # no waiting yet: every ratio is 1, ties by chain
])
def test_alternative_orders_rank_as_defined(key, want):
    ch = [dict(chain(10 * MS, [(0, [(6 * MS, 1.0)])]), period_ns=100 * MS),
          dict(chain(8 * MS, [(0, [(1 * MS, 1.0)])]), period_ns=10 * MS),
          dict(chain(20 * MS, [(0, [(15 * MS, 1.0)])]), period_ns=500 * MS)]
    model = GateModel(ch, {"policy": "urgency", "key": key, "admit": False})
    dec = model.instant(0, [(0, 0, 0), (1, 0, 0), (2, 0, 0)], [])
    assert [d[1] for d in dec if d[0] == "LAUNCH"] == want


@pytest.mark.parametrize("key,want", [
    # four chains arriving at t = 0, CPU segments 0, one kernel per task,
    # estimates in ms; every first task launches at once in rank order.
    #   A: D 100, tasks [10, 10]  S = 80: SAEDF 10 + 80/2 = 50,  EQDF 10 + 80*10/20 = 50
    #   B: D 100, tasks [40, 10]  S = 50: SAEDF 40 + 50/2 = 65,  EQDF 40 + 50*40/50 = 80
    #   C: D 110, tasks [10, 50]  S = 50: SAEDF 10 + 50/2 = 35,  EQDF 10 + 50*10/60 = 18.3
    #   D: D  70, tasks [30]      S = 40: SAEDF 30 + 40 = 70,    EQDF 30 + 40 = 70
    ("saedf", [2, 0, 1, 3]),
    ("eqdf", [2, 0, 3, 1]),
    ("edf", [3, 0, 1, 2]),        # 70, 100, 100, 110 (tie A, B by chain)
    ("urgency", [3, 1, 2, 0]),    # slack 40, 50, 50, 80 (tie B, C by chain)
])
def test_subtask_deadline_orders(key, want):
    ch = [chain(100 * MS, [(0, [(10 * MS, 1.0)]), (0, [(10 * MS, 1.0)])]),
          chain(100 * MS, [(0, [(40 * MS, 1.0)]), (0, [(10 * MS, 1.0)])]),
          chain(110 * MS, [(0, [(10 * MS, 1.0)]), (0, [(50 * MS, 1.0)])]),
          chain(70 * MS, [(0, [(30 * MS, 1.0)])])]
    model = GateModel(ch, {"policy": "urgency", "key": key, "admit": False})
    dec = model.instant(0, [(c, 0, 0) for c in range(4)], [])
    assert [d[1] for d in dec if d[0] == "LAUNCH"] == want


@pytest.mark.parametrize("rule", ["saedf", "eqdf"])
def test_subtask_deadlines_split_the_slack_as_defined(rule):
    # a chain whose every task starts exactly at its predecessor's deadline:
    # the slack S0 = D - sum(w) is split into equal shares S0 / n (equal
    # slack) or shares S0 * w_j / sum(w) (equal flexibility), and the last
    # task's deadline is the chain's end-to-end deadline under both rules
    from fractions import Fraction
    w = [3 * MS, 11 * MS, 5 * MS, 7 * MS]
    t_arr, D = 17 * MS, 61 * MS
    s0 = D - sum(w)
    t = Fraction(t_arr)
    for j in range(len(w)):
        d = P.subtask_deadline(rule, t, t_arr, D, w[j], sum(w[j:]), len(w) - j)
        share = Fraction(s0, len(w)) if rule == "saedf" else Fraction(s0 * w[j], sum(w))
        assert d - t - w[j] == share
        t = d
    assert t == t_arr + D
    # a late task (negative slack) gets a deadline before its own work ends
    assert P.subtask_deadline(rule, 50 * MS, 0, 40 * MS, 5 * MS, 10 * MS, 2) < 55 * MS
    # no work left: the whole slack
    assert P.subtask_deadline("eqdf", 5, 0, 20, 0, 0, 1) == 20


def test_subtask_deadline_uses_the_current_task_and_its_start():
    # chain A of the order test after its first task: task 1 started at 12 ms
    # (task 0 ran 2 ms over its estimate), so S = 100 - 12 - 10 = 78 and both
    # rules give task 1 (the last) the chain deadline, 100 ms; chain C's
    # first task is still running: SAEDF 35 ms, EQDF 18.3 ms
    from fractions import Fraction
    ch = [chain(100 * MS, [(0, [(10 * MS, 1.0)]), (0, [(10 * MS, 1.0)])]),
          chain(110 * MS, [(0, [(10 * MS, 1.0)]), (0, [(50 * MS, 1.0)])])]
    for rule, want_c in (("saedf", Fraction(35 * MS)), ("eqdf", 10 * MS + Fraction(50 * MS, 6))):
        model = GateModel(ch, {"policy": "urgency", "key": rule, "admit": False})
        model.instant(0, [(0, 0, 0), (1, 0, 0)], [])
        model.instant(12 * MS, [], [(0, 0, 0, START, 0), (0, 0, 0, END, 1)])
        a, c = model.inst[(0, 0)], model.inst[(1, 0)]
        assert a.task == 1 and a.task_t0 == 12 * MS
        assert model._subtask_deadline(a, 12 * MS) == 100 * MS
        assert model._subtask_deadline(c, 12 * MS) == want_c


def test_hrrn_prefers_the_longer_wait():
    # HRRN at t = 4 ms: A (arrived at 0, R = 6 ms) has (4 + 6) / 6 = 1.67;
    # B (arrived at 3 ms, R = 1 ms) has (1 + 1) / 1 = 2: B first; SJF agrees
    # here, EDF (A's 10 ms before B's 11 ms) does not
    ch = [chain(10 * MS, [(0, [(6 * MS, 1.0)])]), chain(8 * MS, [(0, [(1 * MS, 1.0)])])]
    for key, first in (("hrrn", 1), ("edf", 0)):
        model = GateModel(ch, {"policy": "urgency", "key": key})
        model.instant(4 * MS, [(0, 0, 0), (1, 0, 3 * MS)], [])
        a, b = model.inst[(0, 0)], model.inst[(1, 0)]
        slack = {i.key: model.slack(i, 4 * MS) for i in (a, b)}
        order = model._order([a, b], slack, 4 * MS)
        assert order[0].c == first, key


# ------------------------------------------------------------------ estimate noise
def test_splitmix64_published_outputs():
    # the first outputs of SplitMix64 from the state 0, as published with the
    # generator (each state advances by 0x9E3779B97F4A7C15)
    x, got = 0, []
    for _ in range(4):
        got.append(P.splitmix64(x))
        x = (x + 0x9E3779B97F4A7C15) % (1 << 64)
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                   0xF88BB8A8724C81EC]


def test_noise_draws_are_uniform_and_keyed():
    ks = [P.noise_permille(3, c, f, j, 2) for c in range(5) for f in range(200) for j in range(3)]
    assert set(ks) == {-2, -1, 0, 1, 2}
    counts = np.bincount(np.array(ks) + 2)
    assert counts.min() > 0.8 * len(ks) / 5 and counts.max() < 1.2 * len(ks) / 5
    # a pure function of (seed, chain, frame, task), different when any changes
    base = P.noise_permille(3, 1, 2, 0, 300)
    assert base == P.noise_permille(3, 1, 2, 0, 300)
    assert len({base, P.noise_permille(4, 1, 2, 0, 300), P.noise_permille(3, 2, 2, 0, 300),
                P.noise_permille(3, 1, 3, 0, 300), P.noise_permille(3, 1, 2, 1, 300)}) > 1
    assert all(P.noise_permille(9, c, 0, 0, 0) == 0 for c in range(20))


def test_noisy_slack_is_the_slack_of_scaled_estimates():
    # the noisy remaining work of a frame equals the plain suffix sums of a
    # chain whose task estimates are scaled by that frame's factors
    tasks = [(300 * US, [(2 * MS, 1.0), (1 * MS, 1.0)]), (0, [(5 * MS, 1.0)]),
             (100 * US, [(700 * US, 1.0), (300 * US, 1.0), (1 * MS, 1.0)])]
    n, seed, f = 400, 77, 3
    cfg = {"policy": "urgency", "est_noise_permille": n, "noise_seed": seed}
    noisy = GateModel([chain(50 * MS, tasks)], cfg)
    noisy.instant(0, [(0, f, 0)], [])
    fac = [1000 + P.noise_permille(seed, 0, f, j, n) for j in range(3)]
    # one task at a time, so per-task floors match: compare the first task
    # alone (before any kernel is confirmed) with its scaled plain chain
    scaled = [(cpu * fac[j] // 1000, [(e * fac[j] // 1000, u) for e, u in ks])
              for j, (cpu, ks) in enumerate(tasks)]
    plain = GateModel([chain(50 * MS, scaled)], {"policy": "urgency"})
    plain.instant(0, [(0, f, 0)], [])
    inst_n, inst_p = noisy.inst[(0, f)], plain.inst[(0, f)]
    gpu_n, cpu_n = noisy.remaining(inst_n)
    gpu_p = sum((e * fac[j] // 1000) for j, (_, ks) in enumerate(tasks) for e, _ in ks)
    cpu_p = sum(cpu * fac[j] // 1000 for j, (cpu, _) in enumerate(tasks) if j >= inst_n.i_cpu)
    # per-task floor of the scaled sum vs the sum of per-kernel floors differ
    # by less than one nanosecond per kernel
    assert abs(gpu_n - gpu_p) <= 6 and cpu_n == cpu_p
    assert noisy.slack(inst_n, 0) == 50 * MS - gpu_n - cpu_n
    assert abs(plain.slack(inst_p, 0) - noisy.slack(inst_n, 0)) <= 6


# ------------------------------------------------------------------ delay timelines
def _delay_case(poll, deadline_a=3 * MS):
    # A: truly urgent (slack 1.5 ms < TH 2 ms at t = 0, 0.5 ms at 1 ms);
    # B: lax, high utilisation
    ch = [chain(deadline_a, [(0, [(int(1.5 * MS), 1.0)])]),
          chain(100 * MS, [(0, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "th_slack_ns": 2 * MS, "delay_poll_ns": poll}
    return ch, cfg, des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 0)], by_est(ch))


def test_delay_sleep_loop_timeline():
    ch, cfg, res = _delay_case(1 * MS)
    holds = [t for t, _, _, ds in res["instants"] for d in ds if d[0] == "HOLD"]
    rel = [t for t, _, _, ds in res["instants"] for d in ds if d[0] == "LAUNCH" and d[1] == 1]
    # held at 0 and again at the 1 ms wake (A still active until 1.5 ms);
    # released at the next wake, 2 ms, not when A retires
    assert holds == [0, 1 * MS]
    assert rel == [2 * MS]
    assert sorted(res["completed"]) == [(0, 0, 0, int(1.5 * MS)), (1, 0, 0, 3 * MS)]
    binds = [d for _, _, _, ds in res["instants"] for d in ds if d[0] == "BIND"]
    assert binds[0][4] == 0            # A bound to the reserved level
    des.check_log(ch, cfg, res["instants"])


def test_delay_event_driven_timeline():
    ch, cfg, res = _delay_case(0)
    rel = [t for t, _, _, ds in res["instants"] for d in ds if d[0] == "LAUNCH" and d[1] == 1]
    assert rel == [int(1.5 * MS)]      # released as soon as A's completion is observed


def test_lost_deadline_is_no_longer_urgent():
    """With D_A = 2 ms, A's slack is 0.5 ms at t = 0 but -0.5 ms at the 1 ms
    wake (its estimate says the deadline is lost), so A stops blocking and B
    is released at that wake although A is still running."""
    ch, cfg, res = _delay_case(1 * MS, deadline_a=2 * MS)
    holds = [t for t, _, _, ds in res["instants"] for d in ds if d[0] == "HOLD"]
    rel = [t for t, _, _, ds in res["instants"] for d in ds if d[0] == "LAUNCH" and d[1] == 1]
    assert holds == [0] and rel == [1 * MS]


def test_low_utilisation_kernels_are_exempt():
    ch = [chain(3 * MS, [(0, [(int(1.5 * MS), 1.0)])]),
          chain(100 * MS, [(0, [(1 * MS, 0.09)])])]
    cfg = {"policy": "urgency", "th_slack_ns": 2 * MS}
    res = des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 0)], by_est(ch))
    assert not any(d[0] == "HOLD" for _, _, _, ds in res["instants"] for d in ds)


@pytest.mark.parametrize("graph", [False, True])
def test_task_graphs_gate_the_whole_task_at_its_first_kernel(graph):
    # A truly urgent and running; B's task = a 0.09-utilisation kernel then a
    # full one.  Per kernel: B's first kernel passes (exempt), the second is
    # held.  As one graph: the task's largest utilisation (1.0) decides, so
    # the whole task is held at its first kernel and then released at once
    ch = [chain(3 * MS, [(0, [(int(1.5 * MS), 1.0)])]),
          chain(100 * MS, [(0, [(200 * US, 0.09), (1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "th_slack_ns": 2 * MS, "graph": graph}
    res = des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 0)], by_est(ch))
    holds = [(t, d[3]) for t, _, _, ds in res["instants"] for d in ds if d[0] == "HOLD"]
    rel = {d[3]: t for t, _, _, ds in res["instants"] for d in ds if d[0] == "LAUNCH" and d[1] == 1}
    if graph:
        assert holds == [(0, 0), (1 * MS, 0)] and rel == {0: 2 * MS, 1: 2 * MS}
        # one batch for the task: a start and an end event only
        evs = [d for _, _, _, ds in res["instants"] for d in ds if d[0] == "EVREC" and d[1] == 1]
        assert [(e[4], e[5]) for e in evs] == [(START, 0), (END, 1)]
    else:
        assert holds[0] == (0, 1) and rel[0] == 0 and rel[1] == 2 * MS
    des.check_log(ch, cfg, res["instants"])


def test_best_effort_kernels_are_always_delayable():
    # the same case as the exemption test, with the low-utilisation kernel in
    # a best-effort chain: it is held while the urgent chain runs, released
    # at the first wake after A's completion, and takes the unreserved level
    ch = [chain(3 * MS, [(0, [(int(1.5 * MS), 1.0)])]),
          chain(0, [(0, [(1 * MS, 0.09)])])]
    cfg = {"policy": "urgency", "th_slack_ns": 2 * MS}
    res = des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 0)], by_est(ch))
    holds = [(t, d[1]) for t, _, _, ds in res["instants"] for d in ds if d[0] == "HOLD"]
    rel = [(t, d[4]) for t, _, _, ds in res["instants"] for d in ds
           if d[0] == "LAUNCH" and d[1] == 1]
    assert holds == [(0, 1), (1 * MS, 1)]
    assert rel == [(2 * MS, 1)]
    des.check_log(ch, cfg, res["instants"])


def test_best_effort_ranks_last_and_is_not_sampled():
    # a best-effort instance ranks below a deadline instance that is already
    # late, and calibration samples ignore it even when it is the only one
    # in flight
    assert P.more_urgent(-5 * MS, (1, 0), None, (0, 0))
    assert not P.more_urgent(None, (0, 0), -5 * MS, (1, 0))
    assert not P.is_truly_urgent(None, 10 * MS)
    ch = [chain(0, [(0, [(1 * MS, 1.0), (1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "th_slack_ns": 0, "calibrate": True}
    res = des.simulate(ch, cfg, [(0, 0, 0)], by_est(ch))
    assert res["gate"].samples == []
    assert res["completed"] == [(0, 0, 0, 2 * MS)]


def test_early_chain_exit():
    # two tasks of 2 ms each, D = 5 ms; the first frame runs alone and makes
    # it.  The second frame arrives at 0.5 ms and waits for task 0 until
    # 2 ms, where its slack is 0.5 + 5 - 4 - 2 = -0.5 ms: it leaves the chain
    # instead of starting task 0.  A best-effort chain (D = 0) never exits,
    # and FIFO launch never exits.
    ch = [chain(5 * MS, [(0, [(2 * MS, 1.0)]), (0, [(2 * MS, 1.0)])]),
          chain(0, [(0, [(1 * MS, 1.0)])])]
    arr = [(0, 0, 0), (0, 1, 500 * US), (1, 0, 0)]
    res = des.simulate(ch, {"policy": "urgency", "exit": True}, arr, by_est(ch))
    exits = [(t, d) for t, _, _, ds in res["instants"] for d in ds if d[0] == "EXIT"]
    assert exits == [(2 * MS, ("EXIT", 0, 1, 0))]
    assert res["gate"].exited == {(0, 1)}
    done = {(c, f): td for c, f, _, td in res["completed"]}
    assert done[(0, 1)] == 2 * MS and (1, 0) in done and (0, 0) in done
    res = des.simulate(ch, {"policy": "fifo", "exit": True}, arr, by_est(ch))
    assert not any(d[0] == "EXIT" for _, _, _, ds in res["instants"] for d in ds)


def test_same_chain_never_blocks_itself():
    # two frames of one chain, pipelined over two tasks; the urgent older
    # frame must not hold the newer one back
    ch = [chain(2 * MS, [(0, [(1 * MS, 1.0)]), (0, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "th_slack_ns": 5 * MS}
    res = des.simulate(ch, cfg, [(0, 0, 0), (0, 1, 500 * US)], by_est(ch))
    assert not any(d[0] == "HOLD" for _, _, _, ds in res["instants"] for d in ds)


# ------------------------------------------------------------------ CPU segments
def test_cpu_segment_delays_and_counts_in_slack():
    ch = [chain(20 * MS, [(3 * MS, [(1 * MS, 1.0)]), (2 * MS, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency"}
    res = des.simulate(ch, cfg, [(0, 0, 0)], by_est(ch))
    launches = [(t, d[3]) for t, _, _, ds in res["instants"] for d in ds if d[0] == "LAUNCH"]
    assert launches == [(3 * MS, 0), (6 * MS, 1)]
    assert res["completed"] == [(0, 0, 0, 7 * MS)]
    model = GateModel(ch, cfg)
    model.instant(0, [(0, 0, 0)], [])
    assert model.last_snapshot[(0, 0)] == 20 * MS - 2 * MS - 5 * MS


# ------------------------------------------------------------------ FIFO
def test_fifo_launches_everything_on_task_streams():
    ch = [chain(50 * MS, [(0, [(1 * MS, 1.0)] * 3)]),
          chain(50 * MS, [(0, [(1 * MS, 1.0)] * 2), (0, [(1 * MS, 1.0)])])]
    cfg = {"policy": "fifo"}
    res = des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 0)], by_est(ch))
    first = res["instants"][0][3]
    kinds = [d[0] for d in first]
    assert kinds.count("LAUNCH") == 5 and "HOLD" not in kinds
    lanes = {(d[1], d[3]): d[5] for d in first if d[0] == "BIND"}
    assert lanes == {(0, 0): 0, (1, 0): 1}
    t_task1 = [t for t, _, _, ds in res["instants"] if ("TSTART", 1, 0, 1) in ds]
    assert lanes and t_task1 == [5 * MS]    # served in launch order: 3 + 2 ms


# ------------------------------------------------------------------ brute force
def _random_tiny(r, n_chains, max_kernels=6, unit=US):
    chains, arrivals = [], []
    budget = max_kernels
    for c in range(n_chains):
        k_left = budget - (n_chains - c - 1)
        n_k = int(r.integers(1, min(3, k_left) + 1))
        budget -= n_k
        split = int(r.integers(0, n_k)) if n_k > 1 else 0
        ks = [(int(r.integers(1, 8)) * 100 * unit, 1.0) for _ in range(n_k)]
        tasks = [(0, ks)] if split == 0 else [(0, ks[:split]), (int(r.integers(0, 3)) * 100 * unit, ks[split:])]
        chains.append(chain(int(r.integers(3, 25)) * 100 * unit, tasks))
        arrivals.append((c, 0, int(r.integers(0, 6)) * 100 * unit))
    return chains, arrivals


def _exec_order(trace):
    return [(c, g) for _, _, c, _, g in sorted(trace)]


def test_bruteforce_accounting_identity_and_optimality():
    r = np.random.default_rng(0)
    for it in range(150):
        chains, arrivals = _random_tiny(r, int(r.integers(2, 4)))
        dur = by_est(chains)
        cfg = {"policy": "urgency", "delay": False, "th_slack_ns": 0,
               "delta_eval_ns": int(r.integers(1, 10)) * 100 * US}
        res = des.simulate(chains, cfg, arrivals, dur)
        done = {c: td for c, f, ta, td in res["completed"]}
        forced = brute.forced_order(chains, arrivals, dur, _exec_order(res["trace"]))
        assert done == forced, it
        m, lmax, _ = brute.objectives(chains, arrivals, done)
        bm, bl, _ = brute.best(chains, arrivals, dur)
        assert m >= bm and lmax >= bl
        des.check_log(chains, cfg, res["instants"])


def test_jackson_subclass_is_optimal_for_lateness():
    """Common arrival, one kernel per chain, equal durations, no deadline
    already lost (D >= e, so every slack at t = 0 is >= 0): slack order is
    deadline order (Jackson's rule), which minimises the maximum lateness and
    so meets every deadline whenever some order does.  (A chain whose slack is
    negative would rank last under Eq. (2), which is not EDF.)"""
    r = np.random.default_rng(1)
    for it in range(60):
        n = int(r.integers(2, 7))
        e = 300 * US
        chains = [chain(int(r.integers(2, 13)) * 150 * US, [(0, [(e, 1.0)])]) for _ in range(n)]
        arrivals = [(c, 0, 0) for c in range(n)]
        cfg = {"policy": "urgency", "delay": False}
        res = des.simulate(chains, cfg, arrivals, by_est(chains))
        done = {c: td for c, f, ta, td in res["completed"]}
        m, lmax, _ = brute.objectives(chains, arrivals, done)
        bm, bl, _ = brute.best(chains, arrivals, by_est(chains))
        assert lmax == bl, it
        assert (m == 0) == (bm == 0)


def test_T3_least_laxity_is_not_edf():
    """A (e = 5, D = 6) and B (e = 1, D = 3) at t = 0 with no truly urgent
    level: A has the smaller slack (1 < 2) and runs first, so B misses, while
    running B first meets both deadlines: regret 1."""
    chains = [chain(6 * MS, [(0, [(5 * MS, 1.0)])]), chain(3 * MS, [(0, [(1 * MS, 1.0)])])]
    arrivals = [(0, 0, 0), (1, 0, 0)]
    cfg = {"policy": "urgency", "th_slack_ns": 0}
    res = des.simulate(chains, cfg, arrivals, by_est(chains))
    done = {c: td for c, f, ta, td in res["completed"]}
    assert done == {0: 5 * MS, 1: 6 * MS}
    m, _, _ = brute.objectives(chains, arrivals, done)
    bm, _, _ = brute.best(chains, arrivals, by_est(chains))
    assert (m, bm) == (1, 0)


def test_brute_force_enumerates_every_interleaving():
    chains = [chain(MS, [(0, [(1, 1.0)] * 2)]), chain(MS, [(0, [(1, 1.0)] * 2)]),
              chain(MS, [(0, [(1, 1.0)] * 1)])]
    orders = list(brute.all_orders(chains))
    assert len(orders) == 30                  # 5! / (2! 2! 1!)
    assert len(set(map(tuple, orders))) == 30


# ------------------------------------------------------------------ randomised invariants
def _random_workload(r, n_chains=4, n_frames=4):
    chains, arrivals = [], []
    for c in range(n_chains):
        tasks = []
        for j in range(int(r.integers(1, 4))):
            ks = [(int(r.integers(20, 400)) * US, float(r.choice([0.05, 0.5, 1.0])))
                  for _ in range(int(r.integers(1, 8)))]
            tasks.append((int(r.integers(0, 3)) * 200 * US, ks))
        period = int(r.integers(4, 12)) * MS
        chains.append(chain(int(period * r.choice([0.5, 1.0])), tasks))
        phase = int(r.integers(0, period))
        for f in range(n_frames):
            arrivals.append((c, f, phase + f * period + int(r.integers(0, 300)) * US))
    return chains, arrivals


@pytest.mark.parametrize("seed", range(6))
def test_random_runs_satisfy_invariants_and_replay(seed):
    r = np.random.default_rng(100 + seed)
    chains, arrivals = _random_workload(r)
    noise = {}

    def dur(c, f, g):
        key = (c, f, g)
        if key not in noise:
            est = [e for t in chains[c]["tasks"] for e in t["est_ns"]]
            noise[key] = max(1, int(est[g] * r.uniform(0.7, 1.4)))
        return noise[key]

    for cfg in ({"policy": "urgency", "th_slack_ns": 3 * MS},
                {"policy": "urgency", "th_slack_ns": 3 * MS, "delay_poll_ns": 0},
                {"policy": "urgency", "th_slack_ns": 0, "lanes": [1, 1]},
                {"policy": "urgency", "batch": False, "bind": False, "th_slack_ns": 2 * MS}):
        res = des.simulate(chains, cfg, arrivals, dur)
        assert len(res["completed"]) == len(arrivals)
        des.check_log(chains, cfg, res["instants"])
        assert des.replay(chains, cfg, res["instants"]) is None
    res = des.simulate(chains, {"policy": "fifo"}, arrivals, dur)
    assert len(res["completed"]) == len(arrivals)


def test_replay_detects_a_changed_decision():
    r = np.random.default_rng(7)
    chains, arrivals = _random_workload(r, 3, 3)
    cfg = {"policy": "urgency", "th_slack_ns": 2 * MS}
    res = des.simulate(chains, cfg, arrivals, by_est(chains))
    inst = list(res["instants"])
    k = next(i for i, x in enumerate(inst) if any(d[0] == "LAUNCH" for d in x[3]))
    t, a, e, d = inst[k]
    d = list(d)
    li = next(i for i, x in enumerate(d) if x[0] == "LAUNCH")
    d[li] = d[li][:5] + (d[li][5] + 1,)
    inst[k] = (t, a, e, d)
    assert des.replay(chains, cfg, inst)[0] == k


def test_calibration_samples_and_threshold():
    r = np.random.default_rng(3)
    chains, arrivals = _random_workload(r, 4, 6)
    cfg = {"policy": "urgency", "delay": False, "th_slack_ns": 0, "calibrate": True}
    res = des.simulate(chains, cfg, arrivals, by_est(chains))
    s = res["gate"].samples
    assert len(s) > 10
    th = P.threshold_from_samples(s)
    pos = sorted(v for v in s if v > 0)
    assert th == 0 or th in s
    if th > 0:
        # at most 5 % of the samples are more urgent than the threshold
        more = sum(1 for v in s if P.ul_greater(v, th))
        assert more <= 0.05 * len(s) + 1


# ------------------------------------------------------------------ task admission
def _holds(res):
    return [(t, d[1], d[4]) for t, _, _, ds in res["instants"] for d in ds if d[0] == "HOLD"]


def _first_launch(res):
    out = {}
    for t, _, _, ds in res["instants"]:
        for d in ds:
            if d[0] == "LAUNCH":
                out.setdefault(d[1], t)
    return out


@pytest.mark.parametrize("admit_tasks", [1, 2])
def test_admission_holds_a_task_until_the_in_flight_count_drops(admit_tasks):
    # admit_tasks - 1 long fillers (chains 2..) and chain 0 occupy every place;
    # chain 1 arrives at 0.5 ms, is not truly urgent (TH = +inf) and waits
    # (HOLD, reason admission) until the first task end of another chain is
    # observed, where the count of instances with kernels in flight drops
    # below the cap
    ch = [chain(100 * MS, [(0, [(2 * MS, 1.0)])]),
          chain(50 * MS, [(0, [(1 * MS, 1.0)])])]
    ch += [chain(100 * MS, [(0, [(5 * MS, 1.0)])]) for _ in range(admit_tasks - 1)]
    arr = [(0, 0, 0), (1, 0, 500 * US)] + [(c, 0, 0) for c in range(2, len(ch))]
    cfg = {"policy": "urgency", "th_slack_ns": 0, "admit_tasks": admit_tasks}
    res = des.simulate(ch, cfg, arr, by_est(ch))
    holds = _holds(res)
    assert holds and all(h[1] == 1 and h[2] == HOLD_ADMIT for h in holds)
    assert holds[0][0] == 500 * US
    # while the others run the cap is full; chain 1 is admitted at the
    # first task end observed (the count drops below the cap), not earlier
    first_end = min(td for c, f, _, td in res["completed"] if c != 1)
    assert _first_launch(res)[1] == first_end
    assert all(t < first_end for t, _, _ in holds)
    assert len(res["completed"]) == len(arr)
    des.check_log(ch, cfg, res["instants"])
    # without admission, chain 1 launches on arrival
    res = des.simulate(ch, dict(cfg, admit=False), arr, by_est(ch))
    assert _first_launch(res)[1] == 500 * US and not _holds(res)


def test_admission_timeline_one_place():
    # admit_tasks = 1, nobody truly urgent.  A (2 ms kernel) starts at 0; B
    # arrives at 0.5 ms and is held; A's end is observed at 2 ms, B launches
    # then and ends at 3 ms.
    ch = [chain(100 * MS, [(0, [(2 * MS, 1.0)])]), chain(50 * MS, [(0, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "th_slack_ns": 0, "admit_tasks": 1}
    res = des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 500 * US)], by_est(ch))
    assert _holds(res) == [(500 * US, 1, HOLD_ADMIT)]
    assert _first_launch(res) == {0: 0, 1: 2 * MS}
    assert sorted(res["completed"]) == [(0, 0, 0, 2 * MS), (1, 0, 500 * US, 3 * MS)]


@pytest.mark.parametrize("th_ms,urgent", [(5, True), (0, False)])
def test_truly_urgent_task_bypasses_admission(th_ms, urgent):
    # admit_tasks = 1 and A (lax, slack 98 ms) holds the only place.  B
    # arrives at 0.5 ms with D = 4 ms: slack 0.5 + 4 - 1 - 0.5 = 3 ms.  With
    # TH_urgent at a 5 ms slack B is truly urgent: it starts at once on the
    # reserved level; with TH = +inf it waits for A like any other task.
    ch = [chain(100 * MS, [(0, [(2 * MS, 1.0)])]), chain(4 * MS, [(0, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "th_slack_ns": th_ms * MS, "admit_tasks": 1}
    res = des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 500 * US)], by_est(ch))
    binds = {d[1]: d[4] for _, _, _, ds in res["instants"] for d in ds if d[0] == "BIND"}
    if urgent:
        assert _holds(res) == [] and _first_launch(res)[1] == 500 * US and binds[1] == 0
    else:
        assert _holds(res) == [(500 * US, 1, HOLD_ADMIT)] and _first_launch(res)[1] == 2 * MS
        assert binds[1] == 1
    des.check_log(ch, cfg, res["instants"])


def test_admission_releases_the_most_urgent_waiting_task_first():
    # admit_tasks = 1, nobody truly urgent.  A runs 0..2 ms.  B (D 60 ms)
    # arrives at 0.5 ms, C (D 20 ms) at 0.6 ms; both wait.  When A's end is
    # observed at 2 ms the place goes to C, the more urgent (slack 17.6 ms
    # against B's 57.5 ms), and B waits again until C ends at 3 ms.
    ch = [chain(100 * MS, [(0, [(2 * MS, 1.0)])]),
          chain(60 * MS, [(0, [(1 * MS, 1.0)])]),
          chain(20 * MS, [(0, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "th_slack_ns": 0, "admit_tasks": 1}
    res = des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 500 * US), (2, 0, 600 * US)], by_est(ch))
    # (the second hold at 2 ms is the re-check at the instant that observes
    # C's batch start: a waiting task is re-checked at every instant)
    assert _holds(res) == [(500 * US, 1, HOLD_ADMIT),
                           (600 * US, 2, HOLD_ADMIT), (600 * US, 1, HOLD_ADMIT),
                           (2 * MS, 1, HOLD_ADMIT), (2 * MS, 1, HOLD_ADMIT)]
    assert _first_launch(res) == {0: 0, 2: 2 * MS, 1: 3 * MS}
    assert sorted(res["completed"]) == [(0, 0, 0, 2 * MS), (1, 0, 500 * US, 4 * MS),
                                        (2, 0, 600 * US, 3 * MS)]
    des.check_log(ch, cfg, res["instants"])


def test_admission_of_pipelined_frames_of_one_chain():
    # one place, two frames of a two-task chain: frame 1 waits for task 0's
    # slot, then for the place; no deadlock, every frame completes in order
    ch = [chain(20 * MS, [(0, [(1 * MS, 1.0)]), (0, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "th_slack_ns": 0, "admit_tasks": 1}
    res = des.simulate(ch, cfg, [(0, 0, 0), (0, 1, 500 * US)], by_est(ch))
    # at 1 ms frame 0 may start task 1 and frame 1 task 0.  Frame 1 is the
    # more urgent (slack 0.5 + 20 - 2 - 1 = 17.5 ms against frame 0's
    # 20 - 1 - 1 = 18 ms: all its work is still ahead) and takes the place;
    # frame 0 waits until 2 ms, and frame 1's task 1 waits for frame 0 to
    # leave that task's slot at 3 ms
    holds = [(t, d[2], d[3], d[4]) for t, _, _, ds in res["instants"] for d in ds if d[0] == "HOLD"]
    assert holds and set(holds) == {(1 * MS, 0, 1, HOLD_ADMIT)}
    launch = {(d[2], d[3]): t for t, _, _, ds in res["instants"] for d in ds if d[0] == "LAUNCH"}
    assert launch == {(0, 0): 0, (1, 0): 1 * MS, (0, 1): 2 * MS, (1, 1): 3 * MS}
    assert sorted(res["completed"]) == [(0, 0, 0, 3 * MS), (0, 1, 500 * US, 4 * MS)]


@pytest.mark.parametrize("admit_tasks", [1, 2, 3])
@pytest.mark.parametrize("seed", range(3))
def test_admission_never_deadlocks_on_random_workloads(admit_tasks, seed):
    r = np.random.default_rng(200 + seed)
    chains, arrivals = _random_workload(r)
    for th in (0, 3 * MS):
        cfg = {"policy": "urgency", "th_slack_ns": th, "admit_tasks": admit_tasks}
        res = des.simulate(chains, cfg, arrivals, by_est(chains))
        assert len(res["completed"]) == len(arrivals)
        # the cap holds: with nobody truly urgent, no instant ends with more
        # than admit_tasks instances holding launched, unconfirmed kernels
        g = GateModel(chains, cfg)
        peak = 0
        for t, arr, evs, dec in res["instants"]:
            assert g.instant(t, arr, evs) == list(dec)
            n = sum(1 for i in g.inst.values() if i.phase != "done" and i.in_flight())
            peak = max(peak, n)
            if th == 0:
                assert n <= admit_tasks, (t, n)
        if th == 0:
            assert peak == admit_tasks
        des.check_log(chains, cfg, res["instants"])


# ------------------------------------------------------------------ calibration sampling
def test_calibration_samples_at_the_first_instant_of_each_period():
    # A (D 20 ms, one 10 ms kernel) runs from t = 0; best-effort frames of
    # chain 1 arrive at chosen times to create instants; C (D 8 ms, 1 ms)
    # arrives at 2.25 ms and is then the most urgent.  With a 1 ms period the
    # highest urgency is sampled at the first instant at or after each
    # sampling time: 0.3 (first sample: nothing was in flight at 0), 1.3
    # (exactly one period later), 2.3 and 3.35 ms.
    ch = [chain(20 * MS, [(0, [(10 * MS, 1.0)])]), chain(0, [(0, [(100 * US, 1.0)])]),
          chain(8 * MS, [(0, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "delay": False, "admit": False, "th_slack_ns": 0,
           "calibrate": True, "calib_period_ns": 1 * MS}
    g = GateModel(ch, cfg)
    g.instant(0, [(0, 0, 0)], [])
    times = [300, 900, 1300, 1500, 2200, 2250, 2300, 2400, 3350]
    f = 0
    for t_us in times:
        t = t_us * US
        if t_us == 2250:
            g.instant(t, [(2, 0, t)], [])
        else:
            g.instant(t, [(1, f, t)], [])
            f += 1
    # slack of A: 20 - 10 - t; of C: 2.25 + 8 - 1 - t (ms)
    assert g.samples == [int(9.7 * MS), int(8.7 * MS), int(6.95 * MS), int(5.9 * MS)]
    # a zero period samples at every instant with something in flight
    g = GateModel(ch, dict(cfg, calib_period_ns=0))
    g.instant(0, [(0, 0, 0)], [])
    f = 0
    for t_us in times:
        t = t_us * US
        g.instant(t, [(2, 0, t)] if t_us == 2250 else [(1, f, t)], [])
        f += t_us != 2250
    assert len(g.samples) == len(times)


# ------------------------------------------------------------------ hold-age bound
def _long_urgent_case(poll, max_hold, b_kernels=((1 * MS, 1.0),)):
    # A: D 10 ms, one 4.5 ms kernel, truly urgent for its whole run (slack
    # 5.5 - t ms, between 1 and 5.5 ms, under TH 6 ms); B: lax (D 100 ms),
    # high utilisation, arrives at 0
    ch = [chain(10 * MS, [(0, [(int(4.5 * MS), 1.0)])]),
          chain(100 * MS, [(0, list(b_kernels))])]
    cfg = {"policy": "urgency", "th_slack_ns": 6 * MS, "delay_poll_ns": poll,
           "max_hold_ns": max_hold}
    return ch, cfg, des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 0)], by_est(ch))


@pytest.mark.parametrize("poll", [1 * MS, 0])
def test_hold_age_bounds_delayed_launching(poll):
    # unbounded: B is held while A runs and released at the 5 ms wake (sleep
    # loop) or when A's end is observed at 4.5 ms (event-driven).  With a
    # 2.5 ms bound, B is released at 2.5 ms by the bound's own timer, A still
    # running: a timer, not an input, makes that instant
    ch, cfg, res = _long_urgent_case(poll, 0)
    assert _first_launch(res)[1] == (5 * MS if poll else int(4.5 * MS))
    ch, cfg, res = _long_urgent_case(poll, int(2.5 * MS))
    holds = [t for t, _, _, ds in res["instants"] for d in ds if d[0] == "HOLD"]
    # (event-driven: re-checked at the instant that observes A's batch start)
    assert holds == ([0, 1 * MS, 2 * MS] if poll else [0, 0])
    assert _first_launch(res)[1] == int(2.5 * MS)
    t_rel = [t for t, arr, evs, ds in res["instants"]
             if any(d[0] == "LAUNCH" and d[1] == 1 for d in ds)]
    assert t_rel == [int(2.5 * MS)]
    assert not next(i for i in res["instants"] if i[0] == int(2.5 * MS))[2]   # no input
    des.check_log(ch, cfg, res["instants"])
    assert des.replay(ch, cfg, res["instants"]) is None


def test_hold_age_exemption_lasts_for_the_rest_of_the_task():
    # B has two kernels; once its first is released by the bound, its second
    # is not held either, although A is still truly urgent and running
    ch, cfg, res = _long_urgent_case(1 * MS, int(2.5 * MS),
                                     b_kernels=((1 * MS, 1.0), (1 * MS, 1.0)))
    holds = [(t, d[3]) for t, _, _, ds in res["instants"] for d in ds if d[0] == "HOLD"]
    assert holds == [(0, 0), (1 * MS, 0), (2 * MS, 0)]
    rel = {d[3]: t for t, _, _, ds in res["instants"] for d in ds if d[0] == "LAUNCH" and d[1] == 1}
    assert rel[0] == int(2.5 * MS) and rel[1] < int(4.5 * MS)


@pytest.mark.parametrize("poll", [1 * MS, 0])
def test_hold_age_bound_leaves_best_effort_tasks_held(poll):
    # the case above with B best-effort (no deadline): the 2.5 ms bound does
    # not release it, so it waits for A exactly as without a bound (5 ms
    # wake of the sleep loop, or A's end observed at 4.5 ms), and no timer
    # instant is made for it
    ch = [chain(10 * MS, [(0, [(int(4.5 * MS), 1.0)])]), chain(0, [(0, [(1 * MS, 1.0)])])]
    arr = [(0, 0, 0), (1, 0, 0)]
    free = {"policy": "urgency", "th_slack_ns": 6 * MS, "delay_poll_ns": poll}
    bounded = dict(free, max_hold_ns=int(2.5 * MS))
    r0 = des.simulate(ch, free, arr, by_est(ch))
    r1 = des.simulate(ch, bounded, arr, by_est(ch))
    assert _first_launch(r1)[1] == _first_launch(r0)[1] == (5 * MS if poll else int(4.5 * MS))
    assert [i[0] for i in r1["instants"]] == [i[0] for i in r0["instants"]]
    assert int(2.5 * MS) not in [i[0] for i in r1["instants"]]
    des.check_log(ch, bounded, r1["instants"])
    assert des.replay(ch, bounded, r1["instants"]) is None


def test_hold_age_bounds_admission():
    # one place; A runs 10 ms; B arrives at 0.5 ms and waits for the place.
    # With a 3 ms bound it starts at 3.5 ms, beside A; unbounded at 10 ms
    ch = [chain(100 * MS, [(0, [(10 * MS, 1.0)])]), chain(50 * MS, [(0, [(1 * MS, 1.0)])])]
    base = {"policy": "urgency", "th_slack_ns": 0, "admit_tasks": 1}
    arr = [(0, 0, 0), (1, 0, 500 * US)]
    res = des.simulate(ch, base, arr, by_est(ch))
    assert _first_launch(res)[1] == 10 * MS
    cfg = dict(base, max_hold_ns=3 * MS)
    res = des.simulate(ch, cfg, arr, by_est(ch))
    assert _holds(res) == [(500 * US, 1, HOLD_ADMIT)]
    assert _first_launch(res)[1] == int(3.5 * MS)
    des.check_log(ch, cfg, res["instants"])


def test_hold_age_restarts_with_every_task():
    # driven by hand.  A (D 20 ms, one 10 ms kernel) is truly urgent until
    # 10 ms (slack 10 - t ms, TH 20 ms).  B (two one-kernel tasks) is held
    # from 0 and released by the 2.5 ms bound; its first task ends at 2.6 ms;
    # its second task is held afresh (a new hold age) and released by the
    # bound at 5.1 ms, not at once
    ch = [chain(20 * MS, [(0, [(10 * MS, 1.0)])]),
          chain(100 * MS, [(0, [(1 * MS, 1.0)]), (0, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "th_slack_ns": 20 * MS, "delay_poll_ns": 1 * MS,
           "max_hold_ns": int(2.5 * MS)}
    g = GateModel(ch, cfg)
    log = []

    def step(t, arr=(), evs=()):
        log.extend((t, d) for d in g.instant(t, list(arr), list(evs)))

    step(0, [(0, 0, 0), (1, 0, 0)])
    step(50 * US, evs=[(0, 0, 0, START, 0)])
    while True:
        nt = g.timers()
        if nt is None or nt > 2 * MS + 600 * US:
            break
        step(nt)
    step(2 * MS + 600 * US, evs=[(1, 0, 0, START, 0), (1, 0, 0, END, 1)])
    while True:
        nt = g.timers()
        if nt is None or nt > 8 * MS:
            break
        step(nt)
    holds = [(t, d[3]) for t, d in log if d[0] == "HOLD"]
    launch = {d[3]: t for t, d in log if d[0] == "LAUNCH" and d[1] == 1}
    assert holds == [(0, 0), (1 * MS, 0), (2 * MS, 0),
                     (2 * MS + 600 * US, 1), (3 * MS + 600 * US, 1), (4 * MS + 600 * US, 1)]
    assert launch == {0: int(2.5 * MS), 1: 5 * MS + 100 * US}


# ------------------------------------------------------------------ split best-effort work
@pytest.mark.parametrize("chunks", [1, 4])
def test_split_best_effort_product_gives_way_between_chunks(chunks):
    # a best-effort task of 1.2 ms of work, as one kernel or as four 0.3 ms
    # row bands; each best-effort kernel is a batch of its own.  A (D 4 ms,
    # one 1 ms kernel) arrives at 0.45 ms truly urgent.  Split: bands 0-2
    # are out (band b + 1 goes when band b starts), band 3 is held at 0.6 ms
    # and released at the 2.6 ms wake, so A runs 0.9-1.9 ms.  Whole: A waits
    # for the whole product, 1.2-2.2 ms.
    be = chain(0, [(0, [(1200 * US // chunks, 1.0)] * chunks)])
    ch = [chain(4 * MS, [(0, [(1 * MS, 1.0)])]), be]
    cfg = {"policy": "urgency", "th_slack_ns": 4 * MS}
    res = des.simulate(ch, cfg, [(1, 0, 0), (0, 0, 450 * US)], by_est(ch))
    done = {c: td for c, f, _, td in res["completed"]}
    holds = [(t, d[1], d[3]) for t, _, _, ds in res["instants"] for d in ds if d[0] == "HOLD"]
    if chunks == 4:
        assert holds == [(600 * US, 1, 3), (1600 * US, 1, 3)]
        assert done == {0: 1900 * US, 1: 2900 * US}
        evs = [d for _, _, _, ds in res["instants"] for d in ds if d[0] == "EVREC" and d[1] == 1]
        assert [e[5] for e in evs if e[4] == START] == [0, 1, 2, 3]
    else:
        assert holds == [] and done == {0: 2200 * US, 1: 1200 * US}
    des.check_log(ch, cfg, res["instants"])


# ------------------------------------------------------------------ per-frame estimates
def test_profile_estimate_is_the_piecewise_linear_lookup():
    # against numpy's piecewise-linear interpolation (which also clamps to
    # the end values), rounded down; and exactly linear data stays linear
    import math
    pts = [(1000, 100_000), (2000, 300_000), (4000, 500_000), (8000, 2_000_000)]
    vs, es = [p[0] for p in pts], [p[1] for p in pts]
    for v in [0, 1, 999, 1000, 1001, 1500, 1999, 2000, 2001, 3333, 4000, 7999, 8000, 10 ** 6]:
        want = math.floor(float(np.interp(v, vs, es)) + 1e-6)
        assert P.profile_estimate(pts, v) == want, v
    lin = [(v, 7 * v + 1000) for v in (16, 48, 256)]
    for v in range(16, 257, 5):
        assert P.profile_estimate(lin, v) == 7 * v + 1000
    # a falling segment (noisy profiles) rounds down too
    assert P.profile_estimate([(10, 50), (30, 40)], 13) == 48
    assert P.profile_estimate([(5, 9)], 1) == P.profile_estimate([(5, 9)], 99) == 9


def _sized_chain(deadline, pts):
    return {"deadline_ns": deadline,
            "tasks": [{"cpu_ns": 0, "est_ns": [pts[-1][1]], "util": [1.0],
                       "frame_dim": [1], "prof": [pts]}]}


def test_frames_of_different_size_rank_by_their_own_estimates():
    # two chains, same deadline (10 ms), one sized kernel each, profiled at
    # 1000 -> 1 ms and 4000 -> 4 ms.  Chain 0's frame has 1000 points (slack
    # 9 ms), chain 1's 4000 (slack 6 ms): chain 1 is the more urgent and is
    # served first.  With the fixed (largest) estimate both slacks are 6 ms
    # and the tie goes to chain 0.
    pts = [(1000, 1 * MS), (4000, 4 * MS)]
    ch = [_sized_chain(10 * MS, pts), _sized_chain(10 * MS, pts)]
    cfg = {"policy": "urgency", "th_slack_ns": 0, "admit": False}
    g = GateModel(ch, cfg)
    dec = g.instant(0, [(0, 0, 0, (1000,)), (1, 0, 0, (4000,))], [])
    assert g.last_snapshot == {(0, 0): 9 * MS, (1, 0): 6 * MS}
    assert [d[1] for d in dec if d[0] == "LAUNCH"] == [1, 0]
    fixed = [dict(c, tasks=[dict(c["tasks"][0], prof=[None])]) for c in ch]
    g = GateModel(fixed, cfg)
    dec = g.instant(0, [(0, 0, 0, (1000,)), (1, 0, 0, (4000,))], [])
    assert g.last_snapshot == {(0, 0): 6 * MS, (1, 0): 6 * MS}
    assert [d[1] for d in dec if d[0] == "LAUNCH"] == [0, 1]
    # a frame between profile points: 2500 -> 2.5 ms, slack 7.5 ms
    g = GateModel(ch, cfg)
    g.instant(0, [(0, 0, 0, (2500,))], [])
    assert g.last_snapshot == {(0, 0): int(7.5 * MS)}


def test_frame_estimates_set_the_batches():
    # a task of a sized kernel then a fixed 300 us one, Delta_eval 0.5 ms: a
    # small frame (100 us) batches both together, a large one (800 us)
    # closes the first batch at the sized kernel
    pts = [(100, 100 * US), (800, 800 * US)]
    ch = [{"deadline_ns": 50 * MS,
           "tasks": [{"cpu_ns": 0, "est_ns": [800 * US, 300 * US], "util": [1.0, 1.0],
                      "frame_dim": [1, 0], "prof": [pts, None]}]}]
    cfg = {"policy": "urgency", "delta_eval_ns": 500 * US}
    for size, n_batches in ((100, 1), (800, 2)):
        res = des.simulate(ch, cfg, [(0, 0, 0, (size,))],
                           lambda c, f, g: (size * US if g == 0 else 300 * US))
        starts = [d for _, _, _, ds in res["instants"] for d in ds if d[0] == "EVREC" and d[4] == START]
        assert len(starts) == n_batches
        des.check_log(ch, cfg, res["instants"])
        assert des.replay(ch, cfg, res["instants"]) is None


# ------------------------------------------------------------------ CPU scheduling (Sec. 4.3)
def _cpu_records(res):
    return [(t, d[1], d[4]) for t, _, _, ds in res["instants"] for d in ds if d[0] == "CPU"]


@pytest.mark.parametrize("prio", [False, True])
def test_cpu_segments_share_one_core(prio):
    # A: D 100 ms, CPU 5 ms, then a 1 ms kernel; B: D 10 ms, CPU 3 ms, then a
    # 1 ms kernel; both arrive at 0 and there is one core.  First come, first
    # served (ties by chain): A 0-5, B 5-8.  Urgency-centric: at 0 B's slack
    # is 10 - 3 - 1 = 6 ms against A's 94 ms, so B runs 0-3, then A 3-8.
    ch = [chain(100 * MS, [(5 * MS, [(1 * MS, 1.0)])]), chain(10 * MS, [(3 * MS, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "admit": False, "cpu_cores": 1, "cpu_prio": prio}
    res = des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 0)], by_est(ch))
    got = _launch_times_by_chain(res)
    if prio:
        assert got == {0: 8 * MS, 1: 3 * MS}
        assert _cpu_records(res) == [(0, 1, 1), (3 * MS, 0, 1)]
    else:
        assert got == {0: 5 * MS, 1: 8 * MS}
        assert _cpu_records(res) == [(0, 0, 1), (5 * MS, 1, 1)]
    des.check_log(ch, cfg, res["instants"])


def _launch_times_by_chain(res):
    return {d[1]: t for t, _, _, ds in res["instants"] for d in ds if d[0] == "LAUNCH"}


@pytest.mark.parametrize("prio", [False, True])
def test_urgent_segment_preempts_on_its_start(prio):
    # A (D 100 ms, CPU 5 ms) arrives at 0 and takes the core; B (D 10 ms,
    # CPU 3 ms) arrives at 2 ms.  Urgency-centric: B's segment start ranks B
    # first, A loses the core at 2 ms (2 ms of its 5 done) and resumes when
    # B's segment ends at 5 ms, finishing at 8 ms.  First come, first served:
    # A 0-5, B 5-8.
    ch = [chain(100 * MS, [(5 * MS, [(1 * MS, 1.0)])]), chain(10 * MS, [(3 * MS, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "admit": False, "cpu_cores": 1, "cpu_prio": prio}
    res = des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 2 * MS)], by_est(ch))
    got = _launch_times_by_chain(res)
    if prio:
        assert got == {1: 5 * MS, 0: 8 * MS}
        assert _cpu_records(res) == [(0, 0, 1), (2 * MS, 0, 0), (2 * MS, 1, 1), (5 * MS, 0, 1)]
    else:
        assert got == {0: 5 * MS, 1: 8 * MS}
        assert _cpu_records(res) == [(0, 0, 1), (5 * MS, 1, 1)]


def test_cpu_ranks_are_refreshed_only_at_segment_starts():
    # two cores, three segments: A (D 50, CPU 4), B (D 40, CPU 4), C (D 30,
    # CPU 4) arrive at 0, 0 and 1 ms, kernels of 1 ms.  At 0: ranks B, A; both
    # run.  At 1 ms C starts: ranks C, B, A; A (the worst) yields its core to
    # C and resumes at 4 ms, when B ends; C ends at 5 ms; A, with 3 ms left,
    # ends at 7 ms.  The sleep of A is the only preemption.
    ch = [chain(50 * MS, [(4 * MS, [(1 * MS, 1.0)])]), chain(40 * MS, [(4 * MS, [(1 * MS, 1.0)])]),
          chain(30 * MS, [(4 * MS, [(1 * MS, 1.0)])])]
    cfg = {"policy": "urgency", "admit": False, "cpu_cores": 2, "cpu_prio": True}
    res = des.simulate(ch, cfg, [(0, 0, 0), (1, 0, 0), (2, 0, 1 * MS)], by_est(ch))
    assert _cpu_records(res) == [(0, 0, 1), (0, 1, 1), (1 * MS, 0, 0), (1 * MS, 2, 1),
                                 (4 * MS, 0, 1)]
    assert _launch_times_by_chain(res) == {1: 4 * MS, 2: 5 * MS, 0: 7 * MS}
    # without a CPU model (one core per segment) all three run at once
    res = des.simulate(ch, {"policy": "urgency", "admit": False}, [(0, 0, 0), (1, 0, 0),
                                                                 (2, 0, 1 * MS)], by_est(ch))
    assert _cpu_records(res) == []
    assert _launch_times_by_chain(res) == {0: 4 * MS, 1: 4 * MS, 2: 5 * MS}


def test_cpu_model_with_enough_cores_changes_nothing():
    # with as many cores as segments can ever run at once, the CPU model
    # gives the same launches as one core per segment
    r = np.random.default_rng(3)
    chains = [chain(int(r.integers(20, 60)) * MS,
                    [(int(r.integers(0, 4)) * 500 * US, [(int(r.integers(1, 5)) * 200 * US, 1.0)
                                                         for _ in range(3)])
                     for _ in range(3)]) for _ in range(4)]
    arrivals = [(c, f, f * 10 * MS + c * 700 * US) for c in range(4) for f in range(4)]
    base = des.simulate(chains, {"policy": "urgency", "th_slack_ns": 2 * MS}, arrivals,
                        by_est(chains))
    for prio in (False, True):
        cfg = {"policy": "urgency", "th_slack_ns": 2 * MS, "cpu_cores": 64, "cpu_prio": prio}
        res = des.simulate(chains, cfg, arrivals, by_est(chains))
        strip = lambda ins: [[d for d in ds if d[0] != "CPU"] for _, _, _, ds in ins]
        assert strip(res["instants"]) == strip(base["instants"])
        assert res["completed"] == base["completed"]
