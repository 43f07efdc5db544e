"""CPU oracle for the urgency-gated task-chain path (UrgenGo, arXiv 2509.12207).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

The oracle shares no code with the HIP path.  It is written to be slow and
obviously correct:

* ``oracle.kernels`` -- the six data-parallel operations by their plain
  definitions (fp64 for floating point; fp32 exactly where the kernel's fp32
  arithmetic decides a bit-exact or integer result).
* ``oracle.policy`` -- the urgency level of Eq. (2), its exact comparison, the
  stream-binding level (Sec. 4.4.3), the batch partition (Sec. 4.4.5), the
  95th-percentile threshold (Sec. 4.4.3) and the metrics of Eq. (3).
* ``oracle.gate`` -- the launch gate as a state machine, one decision instant
  at a time, following Sec. 4.4.2-4.4.5 in the paper's order.
* ``oracle.des`` -- a discrete-event simulation that drives ``oracle.gate``
  against a serial, non-preemptive device model, and a replay driver that
  re-runs a recorded sequence of instants.
* ``oracle.brute`` -- exhaustive search over execution orders for tiny
  instances.

Every function cites the passage of the paper it follows.  Places where the
paper is silent or ambiguous follow the readings listed in the design notes
of the repository.
"""
