"""Conversion between libug decision-log records and the oracle's tuples."""

import numpy as np

from paper_2509_12207_amd import capi

NAMES = {capi.REC_COMPLETE: "COMPLETE", capi.REC_TSTART: "TSTART", capi.REC_BIND: "BIND",
         capi.REC_HOLD: "HOLD", capi.REC_EVREC: "EVREC", capi.REC_LAUNCH: "LAUNCH",
         capi.REC_EXIT: "EXIT", capi.REC_CPU: "CPU"}


def record_to_tuple(r):
    t = int(r["type"])
    c, f = int(r["chain"]), int(r["frame"])
    if t == capi.REC_COMPLETE:
        return ("COMPLETE", c, f, int(r["t"]))
    if t == capi.REC_TSTART:
        return ("TSTART", c, f, int(r["task"]))
    if t == capi.REC_BIND:
        return ("BIND", c, f, int(r["task"]), int(r["a"]), int(r["b"]))
    if t == capi.REC_HOLD:
        return ("HOLD", c, f, int(r["kernel"]), int(r["a"]))
    if t == capi.REC_EVREC:
        return ("EVREC", c, f, int(r["task"]), int(r["a"]), int(r["b"]))
    if t == capi.REC_LAUNCH:
        return ("LAUNCH", c, f, int(r["kernel"]), int(r["a"]), int(r["b"]))
    if t == capi.REC_EXIT:
        return ("EXIT", c, f, int(r["task"]))
    if t == capi.REC_CPU:
        return ("CPU", c, f, int(r["task"]), int(r["a"]))
    raise ValueError(t)


def inputs_to_records(arrivals, evdones):
    n_dims = sum(len(a[3]) for a in arrivals if len(a) > 3)
    recs = np.zeros(len(arrivals) + n_dims + len(evdones), capi.RECORD_DTYPE)
    i = 0
    for a in arrivals:
        c, f, t_arr = a[:3]
        recs[i]["type"], recs[i]["chain"], recs[i]["frame"], recs[i]["t"] = capi.REC_ARRIVE, c, f, t_arr
        i += 1
        for d, v in enumerate(a[3] if len(a) > 3 else ()):
            r = recs[i]
            r["type"], r["chain"], r["frame"], r["a"], r["t"] = capi.REC_DIMS, c, f, d, v
            i += 1
    for c, f, j, kind, seq in evdones:
        r = recs[i]
        r["type"], r["chain"], r["frame"], r["task"], r["a"], r["b"] = capi.REC_EVDONE, c, f, j, kind, seq
        i += 1
    return recs


def instants_from_trace(recs):
    """Split a gate log into (t, arrivals, evdones, decisions) instants."""
    out = []
    cur = None
    for r in recs:
        t = int(r["type"])
        if t == capi.REC_INSTANT:
            if cur is not None:
                out.append(cur)
            cur = (int(r["t"]), [], [], [])
        elif t == capi.REC_ARRIVE:
            cur[1].append((int(r["chain"]), int(r["frame"]), int(r["t"])))
        elif t == capi.REC_DIMS:
            c, f, t_arr = cur[1][-1][:3]
            assert (c, f) == (int(r["chain"]), int(r["frame"]))
            dims = cur[1][-1][3] if len(cur[1][-1]) > 3 else ()
            cur[1][-1] = (c, f, t_arr, dims + (int(r["t"]),))
        elif t == capi.REC_EVDONE:
            cur[2].append((int(r["chain"]), int(r["frame"]), int(r["task"]), int(r["a"]), int(r["b"])))
        else:
            cur[3].append(record_to_tuple(r))
    if cur is not None:
        out.append(cur)
    return out


def oracle_chains(wl_or_chains, estimates=None, profiles=None):
    """Plain-data chain descriptions for the oracle from synth ChainDefs.

    ``estimates``: optional {(chain, kernel): (est_ns, util)} as read back
    from the library (the policy sees the same numbers on both sides).
    ``profiles``: optional {(chain, kernel): [(v, E), ...]} profile points of
    kernels with a per-frame size, as read back from the library."""
    chains = wl_or_chains.chains if hasattr(wl_or_chains, "chains") else wl_or_chains
    out = []
    for c, ch in enumerate(chains):
        tasks = []
        g = 0
        for task in ch.tasks:
            est, util, fdim, prof = [], [], [], []
            for k in task["kernels"]:
                e, u = estimates[(c, g)] if estimates else (k.get("est_ns", 0), k.get("util", 1.0))
                est.append(e)
                util.append(u)
                fdim.append(int(k.get("frame_dim", 0)))
                prof.append((profiles or {}).get((c, g)) or None)
                g += 1
            tasks.append({"cpu_ns": task.get("cpu_ns", 0), "est_ns": est, "util": util,
                          "frame_dim": fdim, "prof": prof})
        out.append({"deadline_ns": ch.deadline_ns, "tasks": tasks})
    return out
