"""Pins of the oracle's fused-tail model: hand-computed tail outputs, hand
task lists for which tails may leave stream order, and hand service orders of
the urgency-ordered device queue."""

import math

import numpy as np

from oracle import fused as F


def test_tail_outputs_hand_values():
    x = np.array([[1.0, -2.0], [3.0, -0.0]], dtype=np.float32)
    b = np.array([0.5, 1.0], dtype=np.float32)
    y, sm, (rs, ra) = F.tail_outputs(x, b, 0, True, True)
    assert y.tolist() == [[1.5, 0.0], [3.5, 1.0]]
    assert not np.signbit(y).any()
    e = math.exp(1.5)
    assert np.allclose(sm[0], [e / (e + 1.0), 1.0 / (e + 1.0)], rtol=0, atol=1e-15)
    e = math.exp(2.5)
    assert np.allclose(sm[1], [e / (e + 1.0), 1.0 / (e + 1.0)], rtol=0, atol=1e-15)
    assert rs.tolist() == [1.5, 4.5] and ra.tolist() == [1.5, 4.5]
    # per-row bias (channel-major convolution output), no softmax, no row sum
    y, sm, rs = F.tail_outputs(x, np.array([-1.0, -4.0], dtype=np.float32), 1, False, False)
    assert y.tolist() == [[0.0, 0.0], [0.0, 0.0]] and sm is None and rs is None


def gemm(a, b, c):
    return {"op": "gemm", "shape": (64, 32, 16), "in": (a, b), "out": (c,)}


def conv(x, w, y):
    return {"op": "conv3x3", "shape": (1, 8, 4, 4), "in": (x, w), "out": (y,)}


def br(x, bias, y, R=64, C=32, axis=0):
    return {"op": "bias_relu", "shape": (R, C, axis), "in": (x, bias), "out": (y,)}


def sm(x, y, R=64, C=32):
    return {"op": "softmax", "shape": (R, C), "in": (x,), "out": (y,)}


def rs(x, y, R=64, C=32):
    return {"op": "rowsum", "shape": (R, C), "in": (x,), "out": (y,)}


def test_tail_runs_private_buffers_fuse():
    # two blocks with buffers of their own: both tails fuse, each with its
    # softmax / row sum
    ks = [gemm(0, 1, 2), br(2, 3, 2), sm(2, 4), rs(2, 5),
          conv(6, 7, 8), br(8, 9, 8, R=8, C=16, axis=1), rs(8, 10, R=8, C=16)]
    assert F.tail_runs(ks) == [(1, 4), (5, 7)]


def test_tail_runs_reused_buffers_stay_in_order():
    # double-buffered outputs: the third block rewrites the first block's
    # output, so the first tail stays in stream order; the others are not
    # rewritten later (sharing the bias is a read beside a read)
    ks = [gemm(0, 1, 2), br(2, 3, 2), gemm(0, 1, 4), br(4, 3, 4), gemm(0, 1, 2), br(2, 3, 2)]
    assert F.tail_runs(ks) == [(3, 4), (5, 6)]
    # a later kernel that reads the tail's output (write then read)
    ks = [gemm(0, 1, 2), br(2, 3, 2), gemm(2, 1, 4), br(4, 5, 4)]
    assert F.tail_runs(ks) == [(3, 4)]
    # a later kernel that writes the tail's bias (read then write)
    ks = [gemm(0, 1, 2), br(2, 3, 2), gemm(0, 1, 3), br(3, 5, 3)]
    assert F.tail_runs(ks) == [(3, 4)]
    # a shared softmax output keeps the first softmax tail in order
    ks = [gemm(0, 1, 2), br(2, 3, 2), sm(2, 9), gemm(0, 1, 4), br(4, 5, 4), sm(4, 9)]
    assert F.tail_runs(ks) == [(4, 6)]
    # kernels before the tail do not matter: they finish before the producer
    ks = [gemm(0, 1, 2), sm(2, 9), gemm(0, 1, 2), br(2, 9, 2)]
    assert F.tail_runs(ks) == [(3, 4)]


def test_tail_runs_needs_a_contraction_producing_the_input():
    # bias+ReLU at the start of a task, after a softmax, or on a buffer the
    # contraction did not write: not a tail
    assert F.tail_runs([br(2, 3, 2), gemm(0, 1, 4)]) == []
    assert F.tail_runs([gemm(0, 1, 2), sm(2, 4), br(4, 3, 4)]) == []
    assert F.tail_runs([gemm(0, 1, 2), br(5, 3, 5)]) == []
    # a softmax of another shape ends the tail before it, and then reads the
    # tail's output later: nothing fuses
    ks = [gemm(0, 1, 2), br(2, 3, 2), sm(2, 4, R=32, C=64)]
    assert F.tail_runs(ks) == []
    # the producer may read the tail's bias (it only writes the input)
    ks = [gemm(0, 3, 2), br(2, 3, 2)]
    assert F.tail_runs(ks) == [(1, 2)]


def test_tail_runs_executor_limits():
    # a second softmax ends the tail (and reads its output later)
    ks = [gemm(0, 1, 2), br(2, 3, 2), sm(2, 4), sm(2, 5)]
    assert F.tail_runs(ks) == []
    # row sum then softmax is fine; rows of 4098 floats are not
    ks = [gemm(0, 1, 2), br(2, 3, 2), rs(2, 5), sm(2, 4)]
    assert F.tail_runs(ks) == [(1, 4)]
    ks = [gemm(0, 1, 2), br(2, 3, 2, C=4098)]
    assert F.tail_runs(ks) == []
    # long rows without a softmax fuse; with one they do not
    ks = [gemm(0, 1, 2), br(2, 3, 2, R=8, C=8192), rs(2, 5, R=8, C=8192)]
    assert F.tail_runs(ks) == [(1, 3)]
    ks = [gemm(0, 1, 2), br(2, 3, 2, R=8, C=8192), sm(2, 5, R=8, C=8192)]
    assert F.tail_runs(ks) == []
    # a per-frame size anywhere in the producer or the tail
    ks = [dict(gemm(0, 1, 2), frame_dim=1), br(2, 3, 2)]
    assert F.tail_runs(ks) == []
    # short kernels only: 1 MiB of input fuses, a row more does not
    ks = [gemm(0, 1, 2), br(2, 3, 2, R=512, C=512), sm(2, 4, R=512, C=512)]
    assert F.tail_runs(ks) == [(1, 3)]
    ks = [gemm(0, 1, 2), br(2, 3, 2, R=513, C=512), sm(2, 4, R=513, C=512)]
    assert F.tail_runs(ks) == []
    ks = [gemm(0, 1, 2), br(2, 3, 2, R=64, C=4100)]
    assert F.tail_runs(ks) == []


def test_service_order_by_key_then_tiles():
    items = [{"key": (2, 0), "tiles": 2, "ready": 0},
             {"key": (1, 1), "tiles": 1, "ready": 0},
             {"key": (3, 2), "tiles": 1, "ready": 0}]
    assert F.service_order(items) == [(1, 0), (0, 0), (0, 1), (2, 0)]


def test_service_order_waits_for_readiness():
    # the most urgent item becomes ready only after two tiles of another
    items = [{"key": (1, 0), "tiles": 2, "ready": 2},
             {"key": (2, 1), "tiles": 3, "ready": 0}]
    assert F.service_order(items) == [(1, 0), (1, 1), (0, 0), (0, 1), (1, 2)]
    # nothing ready at first: the first ready item starts
    items = [{"key": (1, 0), "tiles": 1, "ready": 5}, {"key": (2, 1), "tiles": 1, "ready": 3}]
    assert F.service_order(items) == [(1, 0), (0, 0)]


def test_service_order_follows_rewritten_keys():
    # the gate re-ranks before the second tile: item 2 overtakes item 0
    items = [{"key": (1, 0), "tiles": 3, "ready": 0},
             {"key": (2, 1), "tiles": 1, "ready": 0},
             {"key": (3, 2), "tiles": 2, "ready": 0}]
    out = F.service_order(items, rekey={1: {2: (0, 2)}})
    assert out == [(0, 0), (2, 0), (2, 1), (0, 1), (0, 2), (1, 0)]
    # a re-rank scheduled at a step that is skipped still applies
    items = [{"key": (1, 0), "tiles": 1, "ready": 4}, {"key": (2, 1), "tiles": 1, "ready": 4}]
    assert F.service_order(items, rekey={2: {1: (0, 1)}}) == [(1, 0), (0, 0)]


def test_item_key_orders_rank_then_publication():
    keys = [F.item_key(2, 5), F.item_key(1, 9), F.item_key(2, 3)]
    assert sorted(keys) == [(1, 9), (2, 3), (2, 5)]
