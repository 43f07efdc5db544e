"""Oracle model of fused tails served from a device-side urgency queue.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Batched launching (Sec. 4.4.5) exists because every launch and every
synchronisation of a short kernel costs time the chains cannot spare; the
fused form of the path goes one step further for the short kernels that
follow a contraction: the bias+ReLU of its output, and the row softmax and
row sum of that result.  Such a run of kernels (a *tail*) is not launched
kernel by kernel; it becomes one work item of a long-lived kernel that takes
items from a queue in device memory, the most urgent first, where urgency is
the urgency of Eq. (2) of the item's chain instance as the gate ranks it
(Sec. 4.2: the higher the urgency level, the earlier the work should run).

Readings (the paper has no fused form; these are the choices built):

* A tail is a bias+ReLU kernel whose input is the output of the kernel right
  before it in the task, that kernel being a contraction (FP32 or BF16 GEMM,
  FP32 or BF16 3x3 convolution), followed by at most one row softmax and
  at most one row sum (in either order) that read the bias+ReLU output with
  the same rows and row length.  Rows are a multiple of 4 floats long, at
  most 4096 with a softmax, and no kernel of the tail or its producer takes
  a per-frame size (these are limits of the executor built).  Only short
  kernels are fused: the bias+ReLU input is at most 1 MiB.  A larger tail
  runs at full-device bandwidth as ordinary launches, where the launch cost
  that batching saves is a small part of its time; on the executor it
  would occupy a few workgroups for much longer.  It is fused
  only if no later kernel of the task writes a buffer the tail reads or
  writes, or reads a buffer the tail writes, so that running it outside the
  task's stream order changes no result; the task counts as finished only
  once its tails have.
* An item's key is (rank of its chain instance in the gate's most recent
  urgency order, publication number): smaller keys are served first; two
  items of one instance keep their publication order.
* The executor serves tiles (groups of rows) one at a time: the next tile
  comes from the ready item with the smallest key that still has tiles
  left, tiles of an item in index order.  An item is ready once its
  contraction has finished.

The arithmetic of a tail is that of its kernels one after the other
(``oracle.kernels``); fusing changes where they run, not what they compute.
"""

from . import kernels as K

CONTRACTIONS = ("gemm", "conv3x3", "gemm_bf16", "conv3x3_bf16")
MAX_SOFTMAX_ROW = 4096     # a fused softmax holds its row in registers
MAX_TAIL_BYTES = 1 << 20   # short kernels only: at most 1 MiB of FP32 input


def tail_outputs(x, bias, axis, softmax, rowsum):
    """The outputs of one tail on X[R, C]: y = bias+ReLU (bit-exact FP32),
    then the softmax of each row of y (fp64) and the sum of each row of y
    (fp64), the last two only when asked for.  Returns (y, sm or None,
    (rs, rs_abs) or None)."""
    y = K.bias_relu_f32(x, bias, axis)
    sm = K.softmax_f64(y) if softmax else None
    rs = K.rowsum_f64(y) if rowsum else None
    return y, sm, rs


def _slots(seq):
    return set(s for s in seq if s is not None and s >= 0)


def tail_runs(kernels):
    """Tails of one task's kernel list (dicts with "op", "shape", "in",
    "out"), as (first, end) index ranges of the kernels fused into one item;
    the contraction right before ``first`` is the item's producer.

    Kernels before the tail finish before its producer starts (stream order)
    and the tail starts after its producer has finished, so only the
    kernels after the tail can overlap it: the tail is fused iff none of
    them writes a buffer the tail reads or writes, or reads a buffer the
    tail writes."""
    runs = []
    n = len(kernels)
    i = 1
    while i < n:
        k, prev = kernels[i], kernels[i - 1]
        if not (k["op"] == "bias_relu" and prev["op"] in CONTRACTIONS
                and k["in"][0] == prev["out"][0]):
            i += 1
            continue
        R, C = k["shape"][0], k["shape"][1]
        y = k["out"][0]
        end = i + 1
        seen = set()
        while end < n and kernels[end]["op"] in ("softmax", "rowsum") \
                and kernels[end]["op"] not in seen \
                and kernels[end]["in"][0] == y \
                and tuple(kernels[end]["shape"][:2]) == (R, C):
            seen.add(kernels[end]["op"])
            end += 1
        if C % 4 or ("softmax" in seen and C > MAX_SOFTMAX_ROW) \
                or 4 * R * C > MAX_TAIL_BYTES \
                or any(kk.get("frame_dim", 0) for kk in kernels[i - 1:end]):
            i = end
            continue
        reads, writes = set(), set()
        for kk in kernels[i:end]:
            reads |= _slots(kk["in"])
            writes |= _slots(kk["out"])
        ok = True
        for kk in kernels[end:]:
            if _slots(kk["out"]) & (reads | writes) or _slots(kk["in"]) & writes:
                ok = False
                break
        if ok:
            runs.append((i, end))
        i = end
    return runs


def item_key(rank, seq):
    """Key of an item: instance rank first (1 = most urgent), then
    publication number; the smaller key is served first."""
    return (rank, seq)


def service_order(items, rekey=None):
    """Tiles in the order one executor serves them.

    ``items``: list of dicts with "key", "tiles" and "ready" (the step from
    which the item may be served; step s is the s-th tile served, from 0).
    ``rekey``: optional {step: {item index: new key}} applied before the
    tile of that step is chosen (the gate rewriting priorities).  Returns
    the list of (item index, tile index); a step at which nothing is ready
    is skipped to the next ready step."""
    left = [it["tiles"] for it in items]
    key = [it["key"] for it in items]
    nxt = [0] * len(items)
    out = []
    step = 0
    pending = sorted((rekey or {}).items())
    while any(left):
        while pending and pending[0][0] <= step:
            for i, k in pending.pop(0)[1].items():
                key[i] = k
        ready = [i for i in range(len(items)) if left[i] and items[i]["ready"] <= step]
        if not ready:
            step = min(items[i]["ready"] for i in range(len(items)) if left[i])
            continue
        i = min(ready, key=lambda j: key[j])
        out.append((i, nxt[i]))
        nxt[i] += 1
        left[i] -= 1
        step += 1
    return out
