"""The gate's threads under ThreadSanitizer, on the CPU: the real runtime
(gate thread, submission and completion queues, statistics, error
messages, policy, task graphs) built for the host with clang++
-fsanitize=thread against a host-only HIP stand-in (tests/native/hip_stub:
launches accepted, events complete 20 us after they are recorded), driven
by a submitting thread, a polling thread and a thread making failing calls.
Every frame must complete once and ThreadSanitizer must report nothing.
The tail executor is not covered (its other side is a GPU kernel)."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_12207_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"


@pytest.fixture(scope="module")
def gate_tsan(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("ROCm's clang++ is not installed")
    exe = str(tmp_path_factory.mktemp("tsan") / "gate_tsan")
    # clang's ThreadSanitizer runtime (ROCm's LLVM): it intercepts the
    # pthread_cond_clockwait behind std::condition_variable::wait_until,
    # which GCC 11's does not (it then reports false races around ug_drain)
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
           "-I", os.path.join(NATIVE, "hip_stub"), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "gate", "runtime.cpp"), os.path.join(CSRC, "gate", "policy.cpp"),
           os.path.join(CSRC, "gate", "tails.cpp"), os.path.join(CSRC, "kernels", "tiles.cpp"),
           "-x", "c++", os.path.join(CSRC, "kernels", "launch.hip"), "-x", "none",
           os.path.join(NATIVE, "hip_stub.cpp"), os.path.join(NATIVE, "gate_tsan_main.cpp"),
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


@pytest.mark.parametrize("mode", ["kernels", "graphs"])
def test_gate_threads_race_free(gate_tsan, mode):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=0 exitcode=66")
    r = subprocess.run([gate_tsan] + (["g"] if mode == "graphs" else []), capture_output=True,
                       text=True, timeout=300, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[:4000]
    assert r.returncode == 0, (r.stdout, r.stderr[:2000])
    assert "submitted 240 completed 240" in r.stdout
