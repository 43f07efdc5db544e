"""The C++ policy core built for the host with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, no HIP), driven through recorded instants of
the oracle's simulations: no sanitizer report, and every decision equal to
the oracle's."""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import des

KEYS = {"urgency": 0, "edf": 1, "sjf": 2, "hrrn": 3, "lcuf": 4, "saedf": 5,
        "eqdf": 6}   # UG_KEY_* of ug.h

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_12207_amd", "csrc")
MS, US = 1_000_000, 1_000
NAMES = {4: "COMPLETE", 5: "TSTART", 6: "BIND", 7: "HOLD", 8: "EVREC", 9: "LAUNCH", 10: "EXIT",
         12: "CPU"}


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("san")
    exe = d / "policy_replay"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "native", "policy_replay_main.cpp"),
           os.path.join(CSRC, "gate", "policy.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def _tuple(line):
    f = line.split()
    ty, c, fr, task, k, a, b, t = (int(x) for x in f)
    n = NAMES[ty]
    if n == "COMPLETE":
        return (n, c, fr, t)
    if n in ("TSTART", "EXIT"):
        return (n, c, fr, task)
    if n == "CPU":
        return (n, c, fr, task, a)
    if n == "HOLD":
        return (n, c, fr, k, a)
    if n in ("BIND", "EVREC"):
        return (n, c, fr, task, a, b)
    return (n, c, fr, k, a, b)


def _encode(chains, cfg, instants):
    c = {"policy": "urgency", "bind": True, "delay": True, "batch": True, "calibrate": False,
         "delta_eval_ns": 500_000, "delay_poll_ns": 1_000_000, "th_slack_ns": 0,
         "util_exempt": 0.1, "calib_period_ns": 1_000_000, "admit": True, "admit_tasks": 4,
         "exit": False, "no_overlap": False, "graph": False, "key": "urgency",
         "est_noise_permille": 0,
         "noise_seed": 0, "max_hold_ns": 0, "cpu_cores": 0, "cpu_prio": False,
         "lanes": [2, 6]}
    c.update(cfg)
    lines = [" ".join(str(x) for x in ["cfg", 1 if c["policy"] == "urgency" else 0, int(c["bind"]),
                                       int(c["delay"]), int(c["batch"]), int(c["calibrate"]),
                                       c["delta_eval_ns"], c["delay_poll_ns"], c["th_slack_ns"],
                                       c["util_exempt"], c["calib_period_ns"], int(c["admit"]),
                                       c["admit_tasks"], int(c["exit"]),
                                       int(c["no_overlap"]), int(c["graph"]), KEYS[c["key"]],
                                       c["est_noise_permille"], c["noise_seed"],
                                       c["max_hold_ns"], c["cpu_cores"], int(c["cpu_prio"]),
                                       len(c["lanes"]),
                                       *c["lanes"]])]
    for ch in chains:
        lines.append(f"chain {ch['deadline_ns']} {ch.get('period_ns', 0)} {len(ch['tasks'])}")
        for t in ch["tasks"]:
            nk = len(t["est_ns"])
            ks = []
            for e, u, fd, pts in zip(t["est_ns"], t["util"], t.get("frame_dim", [0] * nk),
                                     t.get("prof", [None] * nk)):
                pts = pts or []
                ks.append(f"{e} {u!r} {fd} {len(pts)} " + " ".join(f"{v} {x}" for v, x in pts))
            lines.append(f"task {t['cpu_ns']} {nk} {' '.join(ks)}")
    for t, arr, evs, _ in instants:
        lines.append(f"instant {t} {len(arr)} {len(evs)}")
        for a in arr:
            dims = a[3] if len(a) > 3 else ()
            lines.append(f"a {a[0]} {a[1]} {a[2]} {len(dims)} " + " ".join(map(str, dims)))
        lines += [f"e {a} {b} {j} {k} {s}" for a, b, j, k, s in evs]
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("sized", [False, True])
@pytest.mark.parametrize("seed", range(4))
def test_sanitized_policy_matches_oracle(driver, seed, sized):
    r = np.random.default_rng(900 + seed)
    chains, arrivals = [], []
    for ci in range(int(r.integers(2, 6))):
        tasks = []
        for _ in range(int(r.integers(1, 4))):
            n = int(r.integers(1, 9))
            tasks.append({"cpu_ns": int(r.integers(0, 3)) * 150 * US,
                          "est_ns": [int(r.integers(20, 400)) * US for _ in range(n)],
                          "util": [float(r.choice([0.05, 0.1, 0.5, 1.0])) for _ in range(n)]})
        period = int(r.integers(3, 12)) * MS
        # one chain in five is best-effort (deadline 0)
        deadline = 0 if r.random() < 0.2 else int(period * r.choice([0.5, 1.0]))
        chains.append({"deadline_ns": deadline, "tasks": tasks, "period_ns": period})
        phase = int(r.integers(0, period))
        for f in range(int(r.integers(2, 6))):
            arrivals.append((ci, f, phase + f * period + int(r.integers(0, 500)) * US))
    if sized:
        # per-frame sizes on some kernels, with profile points (frame values
        # 1024..3071); every frame draws its value
        for ch in chains:
            for t in ch["tasks"]:
                n = len(t["est_ns"])
                t["frame_dim"] = [int(r.random() < 0.5) for _ in range(n)]
                t["prof"] = [sorted((int(v), int(r.integers(20, 600)) * US)
                                    for v in r.choice(np.arange(1024, 3072), 2, replace=False))
                             if fd else None for fd in t["frame_dim"]]
        arrivals = [(c, f, t, (int(r.integers(1024, 3072)),)) for c, f, t in arrivals]
    noise = {}

    def dur(c, f, g):
        if (c, f, g) not in noise:
            est = [e for t in chains[c]["tasks"] for e in t["est_ns"]]
            noise[(c, f, g)] = max(1, int(est[g] * r.uniform(0.5, 1.6)))
        return noise[(c, f, g)]

    for cfg in ({"th_slack_ns": 3 * MS}, {"th_slack_ns": 3 * MS, "delay_poll_ns": 0},
                {"th_slack_ns": 0, "lanes": [2, 8, 8], "calibrate": True, "delay": False},
                {"th_slack_ns": 2 * MS, "admit": False}, {"th_slack_ns": 0, "admit_tasks": 1},
                {"th_slack_ns": 2 * MS, "exit": True},
                {"th_slack_ns": 2 * MS, "no_overlap": True},
                {"th_slack_ns": 2 * MS, "no_overlap": True, "delta_eval_ns": 0},
                {"th_slack_ns": 2 * MS, "key": "edf"}, {"th_slack_ns": 2 * MS, "key": "sjf"},
                {"th_slack_ns": 2 * MS, "key": "hrrn"}, {"th_slack_ns": 2 * MS, "key": "lcuf"},
                {"th_slack_ns": 2 * MS, "key": "saedf"}, {"th_slack_ns": 2 * MS, "key": "eqdf"},
                {"th_slack_ns": 2 * MS, "est_noise_permille": 300, "noise_seed": 11},
                {"th_slack_ns": 2 * MS, "graph": True},
                {"th_slack_ns": 3 * MS, "max_hold_ns": 2 * MS},
                {"th_slack_ns": 0, "max_hold_ns": 1 * MS, "admit_tasks": 1, "delay_poll_ns": 0},
                {"th_slack_ns": 3 * MS, "cpu_cores": 1, "cpu_prio": True},
                {"th_slack_ns": 3 * MS, "cpu_cores": 2},
                {"policy": "fifo"}):
        res = des.simulate(chains, cfg, arrivals, dur)
        text = _encode(chains, cfg, res["instants"])
        p = subprocess.run([str(driver)], input=text, capture_output=True, text=True)
        assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
        assert "ERROR: AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr
        lines = p.stdout.splitlines()
        i = 0
        for t, _, _, dec in res["instants"]:
            head = lines[i].split()
            assert head[0] == "instant" and int(head[1]) == t
            n = int(head[2])
            got = [_tuple(l) for l in lines[i + 1: i + 1 + n]]
            assert got == list(dec), (cfg, t)
            i += 1 + n
        if cfg.get("calibrate"):
            assert lines[i] == f"samples {len(res['gate'].samples)}"
