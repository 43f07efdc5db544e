"""Every tile variant the autotuner may choose computes the operation: the
FP32 GEMM's three and the FP32 convolution's five, on ragged shapes, with
integer-valued inputs bit-exact and random inputs within 1e-5 of the fp64
oracle (scaled by the absolute-value computation); and a tuning-table entry
changes which variant a launch takes."""

import numpy as np
import pytest
import torch

from oracle import kernels as OK
from paper_2509_12207_amd import capi

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("M,N,K", [(130, 70, 37), (257, 132, 64), (512, 384, 96)])
@pytest.mark.parametrize("integer", [False, True])
def test_gemm_every_variant(M, N, K, integer):
    r = np.random.default_rng(M + N + K)
    if integer:
        A = r.integers(-2, 3, (M, K)).astype(np.float32)
        B = r.integers(-2, 3, (K, N)).astype(np.float32)
    else:
        A = r.uniform(-1, 1, (M, K)).astype(np.float32)
        B = r.uniform(-1, 1, (K, N)).astype(np.float32)
    ref, sc = OK.gemm_f64(A, B), OK.gemm_abs_f64(A, B)
    a, b = _dev(A), _dev(B)
    for v in range(capi.tile_variants("gemm")):
        c = torch.full((M, N), float("nan"), device="cuda")
        capi.kernel_launch_variant({"op": "gemm", "shape": (M, N, K), "in": (0, 1), "out": (2,)},
                                   [a.data_ptr(), b.data_ptr(), c.data_ptr()], v)
        got = c.cpu().numpy()
        if integer:
            assert np.array_equal(got, ref.astype(np.float32)), v
        else:
            assert np.all(np.abs(got - ref) <= TOL * sc), v


@pytest.mark.parametrize("C,H,W", [(16, 13, 21), (64, 32, 48), (130, 20, 20)])
@pytest.mark.parametrize("integer", [False, True])
def test_conv_every_variant(C, H, W, integer):
    r = np.random.default_rng(C * H + W)
    if integer:
        X = r.integers(-2, 3, (1, C, H, W)).astype(np.float32)
        Wt = r.integers(-2, 3, (C, C, 3, 3)).astype(np.float32)
    else:
        X = r.uniform(-1, 1, (1, C, H, W)).astype(np.float32)
        Wt = r.uniform(-1, 1, (C, C, 3, 3)).astype(np.float32)
    ref, sc = OK.conv3x3_f64(X, Wt), OK.conv3x3_abs_f64(X, Wt)
    x, w = _dev(X), _dev(Wt)
    for v in range(capi.tile_variants("conv3x3")):
        y = torch.full((1, C, H, W), float("nan"), device="cuda")
        capi.kernel_launch_variant({"op": "conv3x3", "shape": (1, C, H, W), "in": (0, 1),
                                    "out": (2,)}, [x.data_ptr(), w.data_ptr(), y.data_ptr()], v)
        got = y.cpu().numpy()
        if integer:
            assert np.array_equal(got, ref.astype(np.float32)), v
        else:
            assert np.all(np.abs(got - ref) <= TOL * sc), v


def test_table_entry_changes_the_launch():
    # a conv whose rule picks one variant; a table entry sends the ordinary
    # launch to another, with the same result
    C, H, W = 32, 64, 64
    k = {"op": "conv3x3", "shape": (1, C, H, W), "in": (0, 1), "out": (2,)}
    capi.tile_clear()
    rule = capi.tile_get(k)
    r = np.random.default_rng(1)
    X = r.integers(-2, 3, (1, C, H, W)).astype(np.float32)
    Wt = r.integers(-2, 3, (C, C, 3, 3)).astype(np.float32)
    x, w = _dev(X), _dev(Wt)
    outs = []
    for v in (None, (rule + 2) % 5):
        if v is not None:
            capi.tile_set("conv3x3", k["shape"], v)
            assert capi.tile_get(k) == v
        y = torch.empty((1, C, H, W), device="cuda")
        capi.kernel_launch(k, [x.data_ptr(), w.data_ptr(), y.data_ptr()])
        outs.append(y.cpu().numpy())
    capi.tile_clear()
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], OK.conv3x3_f64(X, Wt).astype(np.float32))
