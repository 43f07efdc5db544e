"""Pins of the oracle's policy primitives: the paper's worked example, closed
forms, hand cases and library cross-checks."""

import json
import math
import os
from decimal import Decimal, ROUND_DOWN, ROUND_HALF_EVEN
from fractions import Fraction

import numpy as np
import pytest

from oracle import policy as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "chain_property.json")
MS = 1_000_000


def ns(ms):
    return int(Decimal(str(ms)) * MS)


def load_rows():
    with open(GOLDEN) as fh:
        return json.load(fh)["rows"]


def trunc4(x):
    return Decimal(x).quantize(Decimal("0.0001"), rounding=ROUND_DOWN)


def test_chain_property_urgency_worked_example():
    """Tab. 'Characteristics of an example workflow': Eq. (2) at t = t_arr with
    all work remaining reproduces the printed UL (truncated to 4 decimals) for
    every chain but C10, whose printed value disagrees with its own inputs."""
    rows = load_rows()
    mismatched = []
    for r in rows:
        s = P.slack_ns(0, 0, ns(r["D_ms"]), ns(r["Egpu_ms"]), ns(r["Ecpu_ms"]))
        ul = Fraction(MS, s)                     # 1/ms, exact
        got = trunc4(Decimal(ul.numerator) / Decimal(ul.denominator))
        if got != Decimal(r["UL"]):
            mismatched.append(r["chain"])
    assert mismatched == [10]
    # C10: 1 / (200 - 17.8 - 6.7) ms = 0.005698..., printed 0.0050
    s10 = P.slack_ns(0, 0, ns(200), ns(6.7), ns(17.8))
    assert s10 == ns(175.5)


def test_chain_property_rounding_reading():
    """Rounding (instead of truncation) to 4 decimals would contradict seven rows besides C10."""
    bad = []
    for r in load_rows():
        s = P.slack_ns(0, 0, ns(r["D_ms"]), ns(r["Egpu_ms"]), ns(r["Ecpu_ms"]))
        ul = Fraction(MS, s)
        rnd = (Decimal(ul.numerator) / Decimal(ul.denominator)).quantize(
            Decimal("0.0001"), rounding=ROUND_HALF_EVEN)
        if rnd != Decimal(r["UL"]):
            bad.append(r["chain"])
    assert bad == [0, 1, 2, 3, 5, 7, 8, 10]


def test_chain_property_priority_ranking():
    """PRI_C is the urgency rank (most urgent = 1).  With ties broken by the
    lower chain id every printed rank is reproduced except the C2/C7 tie,
    which the table orders the other way."""
    rows = load_rows()
    items = [(P.slack_ns(0, 0, ns(r["D_ms"]), ns(r["Egpu_ms"]), ns(r["Ecpu_ms"])),
              (r["chain"], 0), r["chain"]) for r in rows]
    order = [c for _, _, c in P.rank_sort(items)]
    rank = {c: i + 1 for i, c in enumerate(order)}
    printed = {r["chain"]: r["PRI"] for r in rows}
    diff = sorted(c for c in rank if rank[c] != printed[c])
    assert diff == [2, 7]
    assert rank[2] == printed[7] and rank[7] == printed[2]


def test_slack_T1_closed_form():
    """D = 10 ms, kernels 2, 3, 1 ms arriving at 0: slack 4 ms at t = 0; once
    the first kernel is confirmed complete at 2.5 ms, 10 - 4 - 2.5 = 3.5 ms."""
    assert P.slack_ns(0, 0, 10 * MS, 6 * MS, 0) == 4 * MS
    assert P.slack_ns(int(2.5 * MS), 0, 10 * MS, 4 * MS, 0) == int(3.5 * MS)
    # a CPU segment still to run counts against the slack as well
    assert P.slack_ns(0, 0, 10 * MS, 6 * MS, 3 * MS) == 1 * MS


def test_ul_comparison_exact():
    r = np.random.default_rng(0)
    vals = [int(v) for v in r.integers(-50, 51, 400) if v != 0]
    for a, b in zip(vals, vals[1:]):
        assert P.ul_greater(a, b) == (1.0 / a > 1.0 / b)
    assert P.ul_greater(0, 5) and P.ul_greater(0, -5) and not P.ul_greater(0, 0)
    assert not P.ul_greater(5, 0)
    assert P.ul_greater(1, 10**18) and P.ul_greater(-(10**18), -1)
    # negative slack (deadline lost) is below every positive slack
    assert P.ul_greater(10**15, -1)
    # huge slacks that differ by one nanosecond are still ordered exactly
    big = 10**17
    assert P.ul_greater(big, big + 1) and not P.ul_greater(big + 1, big)


def test_truly_urgent():
    th = 5 * MS
    assert P.is_truly_urgent(0, th)
    assert P.is_truly_urgent(1, th)
    assert P.is_truly_urgent(th - 1, th)
    assert not P.is_truly_urgent(th, th)
    assert not P.is_truly_urgent(-1, th)
    assert not P.is_truly_urgent(0, 0)          # TH = +inf
    assert not P.is_truly_urgent(1, -3)


def test_more_urgent_ties():
    assert P.more_urgent(5, (0, 1), 5, (1, 0))
    assert not P.more_urgent(5, (1, 0), 5, (0, 1))
    assert P.more_urgent(5, (0, 1), 5, (0, 2))
    assert P.more_urgent(4, (9, 9), 5, (0, 0))


def test_binding_level_hand_cases():
    L = 3
    assert [P.binding_level(r, 1, L) for r in (1,)] == [1]
    assert [P.binding_level(r, 2, L) for r in (1, 2)] == [1, 2]
    assert [P.binding_level(r, 3, L) for r in (1, 2, 3)] == [1, 1, 2]
    assert [P.binding_level(r, 4, L) for r in (1, 2, 3, 4)] == [1, 1, 2, 2]
    assert P.binding_level(1, 1, 1) == 0
    assert [P.binding_level(r, 6, 6) for r in range(1, 7)] == [1, 1, 2, 3, 4, 5]
    for n in range(1, 20):
        for Lv in range(2, 7):
            lv = [P.binding_level(r, n, Lv) for r in range(1, n + 1)]
            assert lv == sorted(lv) and lv[0] == 1 and lv[-1] <= Lv - 1


def test_batch_partition_T2():
    us = 1000
    est = [200 * us, 200 * us, 200 * us, 100 * us, 600 * us, 50 * us]
    assert P.batch_partition(est, 500 * us) == [[0, 1, 2], [3, 4], [5]]
    assert P.batch_partition(est, None) == [[0, 1, 2, 3, 4, 5]]
    # exactly Delta_eval does not close a batch (strict "exceeds")
    assert P.batch_partition([250, 250, 1], 500) == [[0, 1, 2]]
    assert P.batch_partition([250, 251, 1], 500) == [[0, 1], [2]]


def test_threshold_percentile():
    samples = [10, 1, 7, 3, 5, 9, 2, 8, 4, 6]          # slacks (ns), all positive
    # UL ascending = slack descending: 10, 9, ..., 1; index ceil(9.5) - 1 = 9
    assert P.threshold_from_samples(samples) == 1
    s20 = list(range(1, 21))
    # index ceil(19) - 1 = 18 in slack-descending order -> slack 2
    assert P.threshold_from_samples(s20) == 2
    assert P.threshold_from_samples([]) == 0
    assert P.threshold_from_samples([-5] * 30) == 0
    r = np.random.default_rng(1)
    s = [int(v) for v in r.integers(1, 10**7, 777)]
    th = P.threshold_from_samples(s)
    ul = np.array([1.0 / v for v in s])
    ref = np.percentile(ul, 95, method="inverted_cdf")
    assert math.isclose(1.0 / th, ref, rel_tol=1e-12)


def test_miss_ratio_eq3_and_percentiles():
    assert P.overall_miss_ratio({0: (1, 4), 1: (0, 2)}) == Fraction(1, 8)
    assert P.overall_miss_ratio({0: (3, 3), 1: (0, 0)}) == 1
    assert P.is_miss(11, 10) and not P.is_miss(10, 10)
    r = np.random.default_rng(2)
    v = [int(x) for x in r.integers(0, 10**6, 1001)]
    for pct in (50, 95, 99):
        assert P.percentile_nearest_rank(v, pct) == P.percentile_numpy_inverted_cdf(v, pct)
    assert P.percentile_nearest_rank([5, 1, 3], 50) == 3
    assert P.percentile_nearest_rank([5, 1, 3, 2], 50) == 2
