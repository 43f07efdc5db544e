"""Measured error of the low-precision kernels against fp64, per kernel.

Two references for each: the exact product of the rounded operands (the
oracle's fp64 result: isolates the kernel's FP32 accumulation) and the fp64
product of the FP32 values before they were rounded to BF16 / FP8 E4M3
(adds the operands' quantisation).  Operands are random normals rounded to
nearest.  Each test prints its figures (run with -s to see them) and holds
them to bounds derived from the formats: FP32 accumulation (2^-23 a step,
relative to the sum of |products|) for the rounded reference, and the
operands' unit roundoff (BF16 2^-9, E4M3 2^-4, two operands) for the FP32
one."""

import json

import numpy as np
import pytest

from oracle import kernels as OK

import test_gpu_kernels as G

pytestmark = pytest.mark.gpu


def f32_to_bf16(x):
    """Nearest-even bfloat16 codes of float32 values (finite)."""
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def f32_to_e4m3(x):
    """Nearest E4M3 codes (ties to the smaller magnitude step's lower code)
    of float32 values within the format's range."""
    codes = np.arange(256, dtype=np.uint8)
    vals = OK.e4m3_decode(codes)
    ok = np.isfinite(vals)
    cv, vv = codes[ok], vals[ok]
    order = np.argsort(vv, kind="stable")
    cv, vv = cv[order], vv[order]
    idx = np.clip(np.searchsorted(vv, x), 1, len(vv) - 1)
    lo, hi = vv[idx - 1], vv[idx]
    return cv[np.where(np.abs(x - lo) <= np.abs(hi - x), idx - 1, idx)]


def figures(C, ref, abs_sum):
    d = np.abs(C.astype(np.float64) - ref)
    return {"max_over_abs_sum": float((d / np.maximum(abs_sum, 1e-300)).max()),
            "rms_rel": float(np.sqrt(np.mean((d / np.abs(ref).max()) ** 2)))}


def conv_nhwc_f64(X, Wo):
    """3x3 convolution (zero padding) of an [H, W, C] image with [O, 3, 3, C]
    weights in fp64, NCHW result with a leading batch of one."""
    H, W, C = X.shape
    P = np.zeros((H + 2, W + 2, C))
    P[1:-1, 1:-1] = X
    out = np.zeros((Wo.shape[0], H, W))
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("hwc,oc->ohw", P[dy:dy + H, dx:dx + W], Wo[:, dy, dx, :])
    return out[None]


def test_bf16_gemm_error_against_fp64():
    r = np.random.default_rng(7)
    M = N = K = 1024
    A = r.standard_normal((M, K)).astype(np.float32)
    B = r.standard_normal((N, K)).astype(np.float32)
    A16, B16 = f32_to_bf16(A), f32_to_bf16(B)
    C = G.run_gemm_bf16(A16, B16)
    rnd = figures(C, OK.gemm_bf16_f64(A16, B16), OK.gemm_bf16_abs_f64(A16, B16))
    f32 = figures(C, A.astype(np.float64) @ B.astype(np.float64).T,
                  np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64).T)
    print(json.dumps({"gemm_bf16 1024^3": {"vs_rounded": rnd, "vs_fp32_inputs": f32}}))
    assert rnd["max_over_abs_sum"] <= K * 2.0 ** -23
    assert f32["max_over_abs_sum"] <= 2 * 2.0 ** -8 + K * 2.0 ** -23


def test_fp8_gemm_error_against_fp64():
    r = np.random.default_rng(8)
    M = N = K = 1024
    A = (r.standard_normal((M, K)) * 4).astype(np.float32)
    B = (r.standard_normal((N, K)) * 4).astype(np.float32)
    A8, B8 = f32_to_e4m3(A), f32_to_e4m3(B)
    C = G.run_gemm_fp8(A8, B8)
    rnd = figures(C, OK.gemm_fp8_f64(A8, B8), OK.gemm_fp8_abs_f64(A8, B8))
    f32 = figures(C, A.astype(np.float64) @ B.astype(np.float64).T,
                  np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64).T)
    print(json.dumps({"gemm_fp8 1024^3": {"vs_rounded": rnd, "vs_fp32_inputs": f32}}))
    # the instruction's 64-product window (2^-13 below a block's largest
    # product) and FP32 steps
    assert rnd["max_over_abs_sum"] <= 2.0 ** -13 + (K / 64 + 1) * 2.0 ** -23
    assert f32["max_over_abs_sum"] <= 2 * 2.0 ** -4 + 2.0 ** -13


def test_bf16_conv3x3_error_against_fp64():
    r = np.random.default_rng(9)
    Cc, H, W = 64, 48, 48
    X = r.standard_normal((H, W, Cc)).astype(np.float32)
    Wt = (r.standard_normal((Cc, 3, 3, Cc)) / 8).astype(np.float32)
    X16, W16 = f32_to_bf16(X), f32_to_bf16(Wt)
    C = G.run_conv_bf16(X16, W16)
    ref = OK.conv3x3_bf16_f64(X16, W16)
    # the fp64 reference below follows the oracle's orientation
    assert np.allclose(conv_nhwc_f64(OK.bf16_decode(X16), OK.bf16_decode(W16)), ref,
                       rtol=1e-12, atol=1e-12)
    rnd = figures(C, ref, OK.conv3x3_bf16_abs_f64(X16, W16))
    f32 = figures(C, conv_nhwc_f64(X.astype(np.float64), Wt.astype(np.float64)),
                  conv_nhwc_f64(np.abs(X).astype(np.float64), np.abs(Wt).astype(np.float64)))
    print(json.dumps({"conv3x3_bf16 C64 48^2": {"vs_rounded": rnd, "vs_fp32_inputs": f32}}))
    assert rnd["max_over_abs_sum"] <= 9 * Cc * 2.0 ** -23
    assert f32["max_over_abs_sum"] <= 2 * 2.0 ** -8 + 9 * Cc * 2.0 ** -23
