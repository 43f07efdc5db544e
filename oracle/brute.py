"""Exhaustive search over execution orders for tiny instances (at most ~6 kernels).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The device model is the one of ``oracle.des``: a single non-preemptive server
executing one kernel at a time.  A schedule is determined by the order in
which the server runs the kernels; given an order, starting every kernel as
early as it can (after its predecessor in the chain, after its task's CPU
segment, and after the server is free) minimises every completion time, so the
minimum over all orders is the true optimum of any objective that is monotone
in completion times.
"""

import itertools


def _chain_kernels(chain):
    out = []
    for j, task in enumerate(chain["tasks"]):
        for k in range(len(task["est_ns"])):
            out.append((j, k == 0))
    return out


def forced_order(chains, arrivals, duration_of, order):
    """Completion time of each frame when the server runs kernels in ``order``.

    ``arrivals``: one (c, 0, t_arr) per chain.  ``order``: (c, g) pairs in
    execution order, each chain's kernels in increasing g.  A task's first
    kernel becomes available after the previous task of the frame completed
    (or the arrival) plus the task's CPU segment; later kernels after their
    predecessor.  Returns {c: t_done}.
    """
    t_arr = {c: t for c, _, t in arrivals}
    kern = {c: _chain_kernels(ch) for c, ch in enumerate(chains)}
    done = {}
    free = 0
    last_end = {c: t_arr[c] for c in t_arr}
    for c, g in order:
        j, first = kern[c][g]
        avail = last_end[c] + (chains[c]["tasks"][j].get("cpu_ns", 0) if first else 0)
        start = max(free, avail)
        end = start + int(duration_of(c, 0, g))
        free = end
        last_end[c] = end
        done[c] = end
    return done


def interleavings(counts):
    """All sequences of chain ids where chain c appears counts[c] times."""
    chains = [c for c, n in enumerate(counts) for _ in range(n)]
    seen = set()
    for perm in itertools.permutations(chains):
        if perm in seen:
            continue
        seen.add(perm)
        yield perm


def all_orders(chains):
    counts = [sum(len(t["est_ns"]) for t in ch["tasks"]) for ch in chains]
    for perm in interleavings(counts):
        nxt = [0] * len(chains)
        order = []
        for c in perm:
            order.append((c, nxt[c]))
            nxt[c] += 1
        yield order


def objectives(chains, arrivals, done):
    """(misses, max lateness, summed latency) of one schedule."""
    t_arr = {c: t for c, _, t in arrivals}
    misses = 0
    max_late = None
    total = 0
    for c, ch in enumerate(chains):
        lat = done[c] - t_arr[c]
        late = lat - ch["deadline_ns"]
        misses += lat > ch["deadline_ns"]
        max_late = late if max_late is None else max(max_late, late)
        total += lat
    return misses, max_late, total


def best(chains, arrivals, duration_of):
    """Optimum over all orders of each objective separately."""
    best_m = best_l = best_s = None
    for order in all_orders(chains):
        m, l, s = objectives(chains, arrivals, forced_order(chains, arrivals, duration_of, order))
        best_m = m if best_m is None else min(best_m, m)
        best_l = l if best_l is None else min(best_l, l)
        best_s = s if best_s is None else min(best_s, s)
    return best_m, best_l, best_s
