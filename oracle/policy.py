"""Oracle policy primitives: urgency, comparison, binding level, batches, threshold, metrics.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

All times are integer nanoseconds (Python ints, exact).  Urgency levels are
compared exactly as rationals; floats appear only in reporting helpers.
"""

from fractions import Fraction

import numpy as np


# --------------------------------------------------------------------------
# Eq. (2): urgency level of a chain instance
# --------------------------------------------------------------------------
def slack_ns(t, t_arr, deadline, gpu_remaining, cpu_remaining):
    """Denominator of Eq. (2): t_arr + D - sum(remaining GPU est) - sum(remaining CPU est) - t.

    ``gpu_remaining`` is the sum of the estimated kernel times from the
    currently executing kernel index to the end of the chain, and
    ``cpu_remaining`` the same over CPU segments (Sec. 4.2).
    """
    return t_arr + deadline - gpu_remaining - cpu_remaining - t


def urgency(slack):
    """UL = 1 / slack as an exact extended rational: None stands for +infinity.

    A zero slack (no time left at all) is infinitely urgent; a negative slack
    (the deadline is already lost) gives a negative urgency, below every
    positive one (Sec. 4.2, Eq. (2) taken literally).
    """
    if slack == 0:
        return None
    return Fraction(1, slack)


def ul_greater(s1, s2):
    """True iff UL(s1) > UL(s2), exactly (Eq. (2)).

    A slack of None marks an instance of a best-effort chain (no deadline):
    its urgency is below every deadline instance's, late ones included.
    """
    if s1 is None:
        return False
    if s2 is None:
        return True
    u1, u2 = urgency(s1), urgency(s2)
    if u1 is None:
        return u2 is not None
    if u2 is None:
        return False
    return u1 > u2


def more_urgent(s1, key1, s2, key2):
    """Strict total order used for every ranking: higher UL first, then the
    lower (chain id, frame index)."""
    if ul_greater(s1, s2):
        return True
    if ul_greater(s2, s1):
        return False
    return key1 < key2


def rank_sort(items):
    """Sort (slack, key, payload) triples from most to least urgent."""
    from functools import cmp_to_key

    def cmp(a, b):
        if more_urgent(a[0], a[1], b[0], b[1]):
            return -1
        if more_urgent(b[0], b[1], a[0], a[1]):
            return 1
        return 0
    return sorted(items, key=cmp_to_key(cmp))


def is_truly_urgent(slack, th_slack):
    """UL > TH_urgent (Sec. 4.4.3).

    The threshold is carried as a slack: TH_urgent = 1 / th_slack for
    th_slack > 0; th_slack <= 0 stands for TH_urgent = +infinity, which no
    urgency exceeds.
    """
    if th_slack <= 0 or slack is None:
        return False
    return ul_greater(slack, th_slack)


def ul_per_ms(slack_ns_value):
    """UL in 1/ms as a float, for reporting only."""
    if slack_ns_value == 0:
        return float("inf")
    return 1e6 / slack_ns_value


# --------------------------------------------------------------------------
# Sec. 4.4.3: stream level from the urgency rank
# --------------------------------------------------------------------------
def binding_level(rank, n, n_levels):
    """Level of a task that is not truly urgent.

    The top level (0) is reserved for truly urgent tasks; the others rank the
    urgency of the active tasks and spread the ranks evenly over levels
    1 .. n_levels-1 (rank 1 = most urgent = level 1).  With a single level
    there is nothing to reserve and every task gets level 0.
    """
    assert 1 <= rank <= n
    if n_levels <= 1:
        return 0
    return 1 + ((rank - 1) * (n_levels - 1)) // n


# --------------------------------------------------------------------------
# Sec. 4.4.5: batch partition of a task's kernels
# --------------------------------------------------------------------------
def batch_partition(est, delta):
    """Split a task's kernels (estimated times ``est``) into launch batches.

    Kernels are added to the current batch while the summed estimate stays
    within Delta_eval; the kernel whose estimate makes the sum exceed
    Delta_eval still belongs to the batch and closes it.  The task's last
    kernel always closes the last batch.  ``delta=None`` disables batching
    (one batch).  Returns a list of lists of kernel indices.
    """
    batches = []
    cur = []
    acc = 0
    for k, e in enumerate(est):
        cur.append(k)
        acc += e
        if k == len(est) - 1 or (delta is not None and acc > delta):
            batches.append(cur)
            cur = []
            acc = 0
    return batches


# --------------------------------------------------------------------------
# Sec. 4.4.3: TH_urgent from the recorded highest urgencies
# --------------------------------------------------------------------------
def threshold_from_samples(samples, pct=95):
    """TH_urgent as the nearest-rank ``pct``-th percentile of the sampled
    highest urgencies, returned as a slack (see ``is_truly_urgent``).

    ``samples`` are slacks of the most urgent active instance recorded at each
    sampling instant.  They are ordered by urgency (ascending UL) and the
    element at index ceil(pct/100 * n) - 1 is taken.  A percentile at zero or
    negative slack leaves no urgency above it, so no task is truly urgent
    (th_slack = 0).
    """
    if not samples:
        return 0
    order = rank_sort([(s, (i,), None) for i, s in enumerate(samples)])
    ascending = [s for s, _, _ in reversed(order)]
    n = len(ascending)
    idx = (pct * n + 99) // 100 - 1
    s = ascending[idx]
    return s if s > 0 else 0


# --------------------------------------------------------------------------
# Eq. (3) and latency percentiles
# --------------------------------------------------------------------------
def overall_miss_ratio(per_chain):
    """Eq. (3): mean over chains of (missed instances / total instances).

    ``per_chain`` maps chain -> (missed, total); chains with no instances are
    left out.
    """
    ratios = [Fraction(m, n) for m, n in per_chain.values() if n > 0]
    if not ratios:
        return Fraction(0)
    return sum(ratios) / len(ratios)


def is_miss(latency, deadline):
    """A chain instance misses its deadline when its latency exceeds D."""
    return latency > deadline


def percentile_nearest_rank(values, pct):
    """Nearest-rank percentile: the ceil(pct/100 * n)-th smallest value."""
    v = sorted(values)
    if not v:
        return None
    idx = max(0, -(-pct * len(v) // 100) - 1)
    return v[idx]


def percentile_numpy_inverted_cdf(values, pct):
    """The same percentile through numpy's 'inverted_cdf' method (cross-check)."""
    return np.percentile(np.asarray(values), pct, method="inverted_cdf")


# ------------------------------------------------------------ estimate noise
_M64 = (1 << 64) - 1


def splitmix64(x):
    """One output of the SplitMix64 generator (Steele, Lea and Flood, 2014)
    whose state, before the step, is ``x``: the state advances by the 64-bit
    golden ratio 0x9E3779B97F4A7C15, then is mixed by two xor-shift-multiply
    rounds and a final xor-shift."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def noise_permille(seed, c, f, j, n):
    """Noise of the estimates of task j of frame f of chain c (Sec. 6.6: noise
    drawn uniformly per task instance): an integer k uniform in [-n, n]; the
    task's estimates are taken as E * (1000 + k) / 1000.  The draw is a pure
    function of (seed, chain, frame, task): three chained SplitMix64 outputs,
    reduced modulo 2n + 1."""
    h = splitmix64(splitmix64(splitmix64((seed ^ c) & _M64) ^ f) ^ j)
    return h % (2 * n + 1) - n


def profile_estimate(points, v):
    """Estimate of a kernel for a frame of size v from its profile points
    [(v_0, E_0), (v_1, E_1), ...] (v increasing): the launch-size lookup of
    Sec. 4.1 (Tab. "Example lookup table"), read between table rows as the
    straight line through the two neighbouring points, rounded down, and as
    the nearest end point's estimate outside the table."""
    if v <= points[0][0]:
        return points[0][1]
    if v >= points[-1][0]:
        return points[-1][1]
    for (v0, e0), (v1, e1) in zip(points, points[1:]):
        if v0 <= v < v1:
            return e0 + ((e1 - e0) * (v - v0)) // (v1 - v0)
    raise AssertionError("unreachable")


# --------------------------------------------------------------------------
# Sub-deadlines of the EDF family's chain variants (policy comparison,
# Sec. 6.4: SAEDF and EQDF).  The paper names them by citation only; they are
# read here as earliest-deadline-first on a per-task deadline obtained by
# splitting the chain's remaining slack over its remaining tasks, the two
# classic serial-task rules: equal slack (every remaining task gets the same
# share; SAEDF) and equal flexibility (shares proportional to each task's
# estimated work; EQDF).
# --------------------------------------------------------------------------
def subtask_deadline(rule, t_ref, t_arr, deadline, w_task, w_rem, m):
    """Deadline of the task that started at ``t_ref``: its own estimated
    work ``w_task`` plus its share of the slack S = t_arr + D - t_ref - w_rem
    (``w_rem``: the estimated work of this and every later task, ``m``: the
    number of those tasks, m >= 1).  rule "saedf": S / m; rule "eqdf":
    S * w_task / w_rem (w_rem = 0: all of S).  Exact (a Fraction)."""
    s = t_arr + deadline - t_ref - w_rem
    if rule == "saedf":
        share = Fraction(s, m)
    elif rule == "eqdf":
        share = Fraction(s) if w_rem == 0 else Fraction(s * w_task, w_rem)
    else:
        raise ValueError(rule)
    return t_ref + w_task + share
