"""Pins of the oracle kernels against facts other than the oracle itself.

Each test fixes a result by something independent of ``oracle.kernels``:
integer arithmetic (exact in any order), hand-computed special cases, brute
force over explicit loops, library routines (torch on the CPU), and closed
forms.  Transposed operands, a flipped convolution window, a wrong padding, a
mis-signed bias, a wrong axis or a transposed voxel index each fail at least
one of them.
"""

import math

import numpy as np
import pytest
import torch

from oracle import kernels as K


def rng(seed=0):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------- GEMM
def test_gemm_integer_inputs_exact():
    r = rng(1)
    A = r.integers(-2, 3, size=(37, 53)).astype(np.float32)
    B = r.integers(-2, 3, size=(53, 29)).astype(np.float32)
    exact = A.astype(np.int64) @ B.astype(np.int64)           # integer matmul
    got = K.gemm_f64(A, B)
    assert got.shape == (37, 29)
    assert np.array_equal(got, exact.astype(np.float64))


def test_gemm_hand_example():
    A = np.array([[1, 2, 3], [4, 5, 6]], np.float32)
    B = np.array([[7, 8], [9, 10], [11, 12]], np.float32)
    assert K.gemm_f64(A, B).tolist() == [[58.0, 64.0], [139.0, 154.0]]
    v, s = K.gemm_entry_f64(A, B, 1, 0)
    assert v == 139.0 and s == 139.0


def test_gemm_abs_scale_bounds_error():
    r = rng(2)
    A = r.uniform(-1, 1, (64, 256)).astype(np.float32)
    B = r.uniform(-1, 1, (256, 48)).astype(np.float32)
    c32 = (torch.from_numpy(A) @ torch.from_numpy(B)).numpy()
    c64 = K.gemm_f64(A, B)
    scale = K.gemm_abs_f64(A, B)
    # gamma_K bound of float32 summation: K u / (1 - K u)
    u = 2.0 ** -24
    gam = 256 * u / (1 - 256 * u)
    assert np.all(np.abs(c32 - c64) <= gam * scale + 1e-30)


# --------------------------------------------------------------- bias+ReLU
def test_bias_relu_special_values():
    X = np.array([[-0.0, np.nan, 1.5, -3.0],
                  [2.0, 0.25, -0.25, np.inf]], np.float32)
    b = np.array([0.0, 1.0, -1.5, 1.0], np.float32)        # per column
    y = K.bias_relu_f32(X, b, axis=0)
    want = np.array([[0.0, 0.0, 0.0, 0.0],
                     [2.0, 1.25, 0.0, np.inf]], np.float32)
    assert np.array_equal(y, want)
    assert not np.any(np.signbit(y))                        # -0 maps to +0


def test_bias_relu_single_rounding():
    # 1 + 2^-24 is a tie in float32 and rounds to even (1.0); a two-step or
    # float64 sum would give a different bit pattern.
    X = np.array([[1.0, 1.0]], np.float32)
    b = np.array([2.0 ** -24, 3 * 2.0 ** -24], np.float32)
    y = K.bias_relu_f32(X, b, axis=0)
    assert y[0, 0] == np.float32(1.0)
    assert y[0, 1] == np.float32(1.0 + 2.0 ** -22)


def test_bias_relu_axis_orientation():
    X = np.zeros((2, 3), np.float32)
    yc = K.bias_relu_f32(X, np.array([1, 2, 3], np.float32), axis=0)
    yr = K.bias_relu_f32(X, np.array([5, 7], np.float32), axis=1)
    assert yc.tolist() == [[1, 2, 3], [1, 2, 3]]
    assert yr.tolist() == [[5, 5, 5], [7, 7, 7]]


# ------------------------------------------------------------------- conv
def conv_loops(X, W):
    """Six nested loops over the definition, Python ints/floats."""
    n, c, h, w = X.shape
    o = W.shape[0]
    Y = np.zeros((n, o, h, w))
    for b in range(n):
        for oc in range(o):
            for y in range(h):
                for x in range(w):
                    acc = 0.0
                    for ic in range(c):
                        for dy in range(3):
                            for dx in range(3):
                                yy, xx = y + dy - 1, x + dx - 1
                                if 0 <= yy < h and 0 <= xx < w:
                                    acc += float(W[oc, ic, dy, dx]) * float(X[b, ic, yy, xx])
                    Y[b, oc, y, x] = acc
    return Y


def test_conv_integer_bruteforce():
    r = rng(3)
    X = r.integers(-2, 3, (1, 3, 5, 6)).astype(np.float32)
    W = r.integers(-2, 3, (3, 3, 3, 3)).astype(np.float32)
    assert np.array_equal(K.conv3x3_f64(X, W), conv_loops(X, W))


def test_conv_identity_and_shift():
    r = rng(4)
    X = r.uniform(-1, 1, (1, 2, 4, 5)).astype(np.float32)
    W = np.zeros((2, 2, 3, 3), np.float32)
    W[0, 0, 1, 1] = 1.0
    W[1, 1, 1, 1] = 1.0
    assert np.array_equal(K.conv3x3_f64(X, W), X.astype(np.float64))
    # tap (dy, dx) = (0, 0) reads X[y-1, x-1] (cross-correlation, zero pad)
    W = np.zeros((2, 2, 3, 3), np.float32)
    W[0, 0, 0, 0] = 1.0
    W[1, 1, 0, 0] = 1.0
    Y = K.conv3x3_f64(X, W)
    assert np.all(Y[:, :, 0, :] == 0) and np.all(Y[:, :, :, 0] == 0)
    assert np.array_equal(Y[:, :, 1:, 1:], X[:, :, :-1, :-1].astype(np.float64))


def test_conv_matches_torch_cpu_f64():
    r = rng(5)
    X = r.uniform(-1, 1, (2, 5, 9, 7)).astype(np.float32)
    W = r.uniform(-1, 1, (5, 5, 3, 3)).astype(np.float32)
    ref = torch.nn.functional.conv2d(torch.from_numpy(X).double(),
                                     torch.from_numpy(W).double(), padding=1).numpy()
    np.testing.assert_allclose(K.conv3x3_f64(X, W), ref, rtol=1e-13, atol=1e-13)
    v, s = K.conv3x3_entry_f64(X, W, 1, 3, 0, 6)
    assert abs(v - ref[1, 3, 0, 6]) < 1e-12
    assert abs(s - K.conv3x3_abs_f64(X, W)[1, 3, 0, 6]) < 1e-12


# ----------------------------------------------------------------- rowsum
def test_rowsum_integer_exact_and_closed_form():
    r = rng(6)
    Z = r.integers(-2, 3, (17, 301)).astype(np.float32)
    s, a = K.rowsum_f64(Z)
    assert np.array_equal(s, Z.astype(np.int64).sum(axis=1).astype(np.float64))
    assert np.array_equal(a, np.abs(Z).astype(np.int64).sum(axis=1).astype(np.float64))
    ones = np.ones((3, 1000), np.float32)
    assert K.rowsum_f64(ones)[0].tolist() == [1000.0] * 3


# ---------------------------------------------------------------- softmax
def test_softmax_closed_forms():
    y = K.softmax_f64(np.array([[0.0, math.log(3.0)]]))
    np.testing.assert_allclose(y, [[0.25, 0.75]], rtol=1e-15)
    c = K.softmax_f64(np.full((2, 7), 3.25, np.float32))
    assert np.all(c == 1.0 / 7.0)


def test_softmax_sums_and_shift_invariance():
    r = rng(7)
    X = r.uniform(-30, 30, (9, 513))
    y = K.softmax_f64(X)
    np.testing.assert_allclose(y.sum(axis=1), 1.0, rtol=1e-14)
    np.testing.assert_allclose(K.softmax_f64(X + 17.0), y, rtol=1e-12)
    assert np.argmax(y[0]) == np.argmax(X[0])
    ref = torch.softmax(torch.from_numpy(X), dim=1).numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-12)


# ----------------------------------------------------------------- voxels
def test_voxel_cell_centres_and_orientation():
    # nx != ny so a transposed index is caught; points at cell centres are
    # unambiguous whatever the rounding.
    nx, ny = 7, 5
    xmin, ymin, scale = np.float32(-1.4), np.float32(-1.0), np.float32(5.0)
    pts = []
    want = []
    for iy in range(ny):
        for ix in range(nx):
            pts.append([-1.4 + (ix + 0.5) * 0.2, -1.0 + (iy + 0.5) * 0.2, 0.0, 0.0])
            want.append(iy * nx + ix)
    got = K.voxel_cell_f32(np.array(pts, np.float32), nx, ny, xmin, ymin, scale)
    assert got.tolist() == want


def test_voxel_boundaries():
    P = np.array([
        [-51.2, 0.1, 0, 0],          # left edge is inside: ix = 0
        [51.2, 0.1, 0, 0],           # right edge is outside (half open)
        [-51.2001, 0.1, 0, 0],       # just left of the grid
        [51.19, 51.19, 0, 0],        # last cell
        [0.1, -51.2, 0, 0],          # bottom edge inside
        [0.1, 51.2, 0, 0],           # top edge outside
        [np.nan, 0.0, 0, 0],
        [np.inf, 0.0, 0, 0],
        [0.0, -np.inf, 0, 0],
    ], np.float32)
    v = K.voxel_cell_f32(P)
    assert v[0] == 256 * 512 + 0
    assert v[1] == -1 and v[2] == -1
    assert v[3] == 511 * 512 + 511
    assert v[4] == 0 * 512 + 256
    assert v[5] == -1 and v[6] == -1 and v[7] == -1 and v[8] == -1


def test_voxel_reductions_bruteforce():
    r = rng(8)
    n = 3000
    pts = np.stack([r.normal(0, 0.3, n), r.normal(0, 0.3, n),
                    r.normal(0, 1, n), r.uniform(0, 1, n)], axis=1).astype(np.float32)
    pts[::97, 0] = 60.0                                  # some points outside
    nx, ny = 8, 6
    xmin, ymin, scale = np.float32(-0.8), np.float32(-0.6), np.float32(5.0)
    vidx, count, zmax, first = K.voxel_scatter(pts, nx, ny, xmin, ymin, scale)
    cells = {}
    for p in range(n):
        v = int(vidx[p])
        if v < 0:
            continue
        cells.setdefault(v, []).append(p)
    for v in range(nx * ny):
        members = cells.get(v, [])
        assert count[v] == len(members)
        if members:
            assert zmax[v] == max(pts[p, 2] for p in members)
            assert first[v] == min(members)
        else:
            assert zmax[v] == -np.inf and first[v] == -1
    assert count.sum() == int((vidx >= 0).sum())


def test_voxel_signed_zero_max():
    pts = np.array([[0.1, 0.1, -0.0, 0], [0.1, 0.1, 0.0, 0], [0.3, 0.1, -0.0, 0]], np.float32)
    _, _, zmax, _ = K.voxel_scatter(pts)
    v0 = K.voxel_cell_f32(pts[:1])[0]
    v2 = K.voxel_cell_f32(pts[2:])[0]
    assert zmax[v0] == 0 and not np.signbit(zmax[v0])
    assert zmax[v2] == 0 and np.signbit(zmax[v2])


# ------------------------------------------------------------- FP8 (E4M3)
def test_e4m3_published_values():
    # OCP 8-bit floating point specification, E4M3 table: max normal 448,
    # min normal 2^-6, min subnormal 2^-9, NaN at S.1111.111, no infinities
    d = K.e4m3_decode(np.array([0x7E, 0x08, 0x01, 0x00, 0x80, 0x38, 0xC0, 0x7F, 0xFF, 0x78],
                               np.uint8))
    assert d[0] == 448.0 and d[1] == 2.0 ** -6 and d[2] == 2.0 ** -9
    assert d[3] == 0.0 and not np.signbit(d[3]) and d[4] == 0.0 and np.signbit(d[4])
    assert d[5] == 1.0 and d[6] == -2.0 and np.isnan(d[7]) and np.isnan(d[8])
    assert d[9] == 256.0                        # 0x78: exponent field 15, mantissa 0
    assert np.all(np.isfinite(np.delete(K.e4m3_decode(np.arange(256)), [0x7F, 0xFF])))


def test_e4m3_all_codes_match_torch_float8():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = K.e4m3_decode(codes)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(got[ok], ref[ok])
    assert np.array_equal(np.signbit(got[ok]), np.signbit(ref[ok]))
    # monotone on the positive finite codes
    assert np.all(np.diff(got[:0x7F]) > 0)


def test_gemm_fp8_integer_codes_exact():
    # codes of 0, +-1, +-2: the product is an integer matrix product
    r = np.random.default_rng(4)
    table = np.array([0x00, 0x38, 0xB8, 0x40, 0xC0], np.uint8)
    value = np.array([0, 1, -1, 2, -2], np.int64)
    ia, ib = r.integers(0, 5, (9, 37)), r.integers(0, 5, (11, 37))
    C = K.gemm_fp8_f64(table[ia], table[ib])
    assert np.array_equal(C, (value[ia] @ value[ib].T).astype(np.float64))


def test_gemm_fp8_matches_torch_float8_path():
    r = np.random.default_rng(5)
    A8 = r.integers(0, 256, (33, 70), dtype=np.uint8)
    B8 = r.integers(0, 256, (21, 70), dtype=np.uint8)
    A8[A8 & 0x7F == 0x7F] = 0x30                # no NaN codes
    B8[B8 & 0x7F == 0x7F] = 0xB1
    a = torch.from_numpy(A8).view(torch.float8_e4m3fn).to(torch.float64)
    b = torch.from_numpy(B8).view(torch.float8_e4m3fn).to(torch.float64)
    ref = (a @ b.T).numpy()
    got = K.gemm_fp8_f64(A8, B8)
    assert np.allclose(got, ref, rtol=0, atol=1e-9 * np.abs(ref).max())
    v, sc = K.gemm_fp8_entry_f64(A8, B8, 5, 7)
    assert v == got[5, 7] and sc == K.gemm_fp8_abs_f64(A8, B8)[5, 7]


# ------------------------------------------------------------------- BF16
def test_bf16_published_values():
    # bfloat16 = sign, 8 exponent bits (bias 127), 7 mantissa bits: 1.0 is
    # 0x3F80, pi rounds to 0x4049 = 3.140625, the largest finite value is
    # (2 - 2^-7) 2^127, the smallest subnormal 2^-133
    d = K.bf16_decode(np.array([0x3F80, 0xBF80, 0x4049, 0x0001, 0x7F7F, 0x7F80, 0xFF80, 0x7FC0,
                                0x8000, 0x0080, 0x4000], np.uint16))
    assert d[0] == 1.0 and d[1] == -1.0 and d[2] == 3.140625 and d[3] == 2.0 ** -133
    assert d[4] == (2 - 2.0 ** -7) * 2.0 ** 127
    assert d[5] == np.inf and d[6] == -np.inf and np.isnan(d[7])
    assert d[8] == 0.0 and np.signbit(d[8]) and d[9] == 2.0 ** -126 and d[10] == 2.0


def test_bf16_all_codes_match_float32_upper_half():
    # every code is the upper 16 bits of the binary32 with the same value
    codes = np.arange(1 << 16, dtype=np.uint32)
    with np.errstate(invalid="ignore"):      # NaN payloads widened to float64
        ref = (codes << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    got = K.bf16_decode(codes.astype(np.uint16))
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(got[ok], ref[ok])
    assert np.array_equal(np.signbit(got[ok]), np.signbit(ref[ok]))


def test_gemm_bf16_integer_codes_exact():
    # codes of 0, +-1, +-2, +-3: the product is an integer matrix product
    r = np.random.default_rng(6)
    table = np.array([0x0000, 0x3F80, 0xBF80, 0x4000, 0xC000, 0x4040, 0xC040], np.uint16)
    value = np.array([0, 1, -1, 2, -2, 3, -3], np.int64)
    ia, ib = r.integers(0, 7, (13, 96)), r.integers(0, 7, (7, 96))
    C = K.gemm_bf16_f64(table[ia], table[ib])
    assert np.array_equal(C, (value[ia] @ value[ib].T).astype(np.float64))
    v, sc = K.gemm_bf16_entry_f64(table[ia], table[ib], 3, 4)
    assert v == C[3, 4] and sc == K.gemm_bf16_abs_f64(table[ia], table[ib])[3, 4]


def test_gemm_bf16_matches_torch_bfloat16_path():
    r = np.random.default_rng(7)
    A = r.standard_normal((17, 64)).astype(np.float32)
    B = r.standard_normal((9, 64)).astype(np.float32)
    a16 = torch.from_numpy(A).to(torch.bfloat16)
    b16 = torch.from_numpy(B).to(torch.bfloat16)
    ref = (a16.to(torch.float64) @ b16.to(torch.float64).T).numpy()
    got = K.gemm_bf16_f64(a16.view(torch.int16).numpy().view(np.uint16),
                          b16.view(torch.int16).numpy().view(np.uint16))
    assert np.array_equal(got, ref)



# ----------------------------------------------------------------- vector add
def test_vecadd_is_the_rounded_exact_sum():
    # the sum of two float32 values is exact in float64; rounding it once to
    # float32 is the IEEE float32 addition
    r = np.random.default_rng(12)
    a = (r.standard_normal(4096) * np.exp2(r.integers(-30, 30, 4096))).astype(np.float32)
    b = (r.standard_normal(4096) * np.exp2(r.integers(-30, 30, 4096))).astype(np.float32)
    want = (a.astype(np.float64) + b.astype(np.float64)).astype(np.float32)
    assert np.array_equal(K.vecadd_f32(a, b).view(np.uint32), want.view(np.uint32))
    with np.errstate(invalid="ignore"):     # inf - inf
        sp = K.vecadd_f32(np.array([np.inf, -0.0, -0.0, 1.0], np.float32),
                          np.array([-np.inf, -0.0, 0.0, -1.0], np.float32))
    assert np.isnan(sp[0]) and np.signbit(sp[1]) and not np.signbit(sp[2])
    assert sp[3] == 0 and not np.signbit(sp[3])



def test_conv3x3_bf16_layouts_against_brute_force():
    # NHWC activations, OHWI weights: a direct six-loop sum in those layouts
    r = np.random.default_rng(13)
    H, W, C, O = 3, 4, 2, 3
    table = np.array([0x0000, 0x3F80, 0xBF80, 0x4000, 0xC000, 0x3F00, 0x4040], np.uint16)
    X16 = table[r.integers(0, 7, (H, W, C))]
    W16 = table[r.integers(0, 7, (O, 3, 3, C))]
    x, w = K.bf16_decode(X16), K.bf16_decode(W16)
    want = np.zeros((1, O, H, W))
    for o in range(O):
        for y in range(H):
            for xx in range(W):
                for dy in range(3):
                    for dx in range(3):
                        yy, xc = y + dy - 1, xx + dx - 1
                        if 0 <= yy < H and 0 <= xc < W:
                            for c in range(C):
                                want[0, o, y, xx] += w[o, dy, dx, c] * x[yy, xc, c]
    assert np.array_equal(K.conv3x3_bf16_f64(X16, W16), want)
    assert np.array_equal(K.conv3x3_bf16_abs_f64(X16, W16),
                          K.conv3x3_bf16_f64(X16 & 0x7FFF, W16 & 0x7FFF))
