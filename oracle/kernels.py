"""Oracle kernels: plain definitions of the six data-parallel operations.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper schedules third-party GPU kernels (TensorRT networks, point-cloud
libraries, Rodinia codes; Sec. 5, Tab. "GPU task profiling results") and does
not define any kernel itself.  The synthetic chains stand in for that work with
six operations whose results have a plain mathematical definition, so each
function below is that definition written out, with no blocking, fusion or
reordering:

* matrix product  C = A B                          (dense layers, LLM, ICP)
* bias + ReLU     y = max(x + b, 0)               (pointwise epilogues)
* 3x3 convolution (cross-correlation, zero pad 1)  (camera networks)
* row sum         r_i = sum_j Z_ij                 (reductions, histograms)
* row softmax     y_ij = exp(x_ij - m_i) / sum_l exp(x_il - m_i)
* voxel scatter   bird's-eye-view pillar binning of a point cloud (LiDAR
  3D detection front end): per-point cell index and per-cell count, highest
  z and first point index.
* FP8 matrix product  C = A B with A, B in the OCP FP8 E4M3 format and an
  FP32 result (the best-effort overload load: large low-precision products
  that share the GPU with the deadline chains).
* BF16 matrix product  C = A B with A, B in bfloat16 and an FP32 result
  (the reduced-precision form of the dense layers).
* BF16 3x3 convolution  the same convolution with bfloat16 activations in
  NHWC and weights in OHWI (channels innermost) and an FP32 NCHW result.
* vector add      c = a + b (the custom kernel of the sensitivity
  experiments, whose utilisation and duration are set directly).

Floating point results are computed in float64 from the float32 inputs.  The
two operations whose results must be bit-exact take their decisions in
float32, the precision the kernels compute in: bias+ReLU is a single float32
add followed by a sign test, and the voxel scatter decides each cell index
from float32 arithmetic.
"""

import numpy as np


# --------------------------------------------------------------------------
# matrix product
# --------------------------------------------------------------------------
def gemm_f64(A, B):
    """C[m, n] = sum_k A[m, k] * B[k, n], row-major, accumulated in float64.

    Each float32 product is exact in float64, so this is effectively the exact
    result up to the float64 summation error (far below the float32 bound).
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    assert A.ndim == 2 and B.ndim == 2 and A.shape[1] == B.shape[0]
    return A @ B


def gemm_abs_f64(A, B):
    """(|A| |B|)[m, n]: the scale of the componentwise error bound of C."""
    return np.abs(np.asarray(A, np.float64)) @ np.abs(np.asarray(B, np.float64))


def gemm_entry_f64(A, B, m, n):
    """One entry C[m, n] as an explicit dot product (for sampled checks)."""
    a = np.asarray(A[m, :], dtype=np.float64)
    b = np.asarray(B[:, n], dtype=np.float64)
    return float(np.dot(a, b)), float(np.dot(np.abs(a), np.abs(b)))


# --------------------------------------------------------------------------
# bias + ReLU
# --------------------------------------------------------------------------
def bias_relu_f32(X, bias, axis):
    """y = s > 0 ? s : +0 with s = fl32(x + b), elementwise on X[R, C].

    ``axis == 0``: one bias per column (bias has C entries; dense layer
    outputs).  ``axis == 1``: one bias per row (bias has R entries; a
    channel-major NCHW tensor viewed as [channels, H*W]).

    The sum is one IEEE float32 addition (round to nearest even); the sign test
    maps -0 and NaN to +0.  This is the bit-exact reference.
    """
    X = np.asarray(X, dtype=np.float32)
    bias = np.asarray(bias, dtype=np.float32)
    if axis == 0:
        assert bias.shape == (X.shape[1],)
        s = X + bias[None, :]
    else:
        assert bias.shape == (X.shape[0],)
        s = X + bias[:, None]
    assert s.dtype == np.float32
    return np.where(s > np.float32(0.0), s, np.float32(0.0)).astype(np.float32)


# --------------------------------------------------------------------------
# 3x3 convolution
# --------------------------------------------------------------------------
def conv3x3_f64(X, W):
    """Y[n, o, y, x] = sum_c sum_{dy,dx in 0..2} W[o, c, dy, dx] X[n, c, y+dy-1, x+dx-1].

    NCHW input, OIHW weights, stride 1, zero padding 1, cross-correlation (no
    kernel flip), no bias, as many output channels as W has rows.  The sum over
    c at each of the nine offsets is a matrix product (library primitive,
    dispatched to BLAS by einsum's optimiser).
    """
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    n, c, h, w = X.shape
    o = W.shape[0]
    assert W.shape == (o, c, 3, 3)
    Xp = np.zeros((n, c, h + 2, w + 2), dtype=np.float64)
    Xp[:, :, 1:h + 1, 1:w + 1] = X
    Y = np.zeros((n, o, h, w), dtype=np.float64)
    for dy in range(3):
        for dx in range(3):
            patch = Xp[:, :, dy:dy + h, dx:dx + w]          # [n, c, h, w]
            Y += np.einsum("oc,nchw->nohw", W[:, :, dy, dx], patch, optimize=True)
    return Y


def conv3x3_abs_f64(X, W):
    """(|W| * |X|): the scale of the componentwise error bound of Y."""
    return conv3x3_f64(np.abs(np.asarray(X, np.float64)),
                       np.abs(np.asarray(W, np.float64)))


def conv3x3_entry_f64(X, W, n, o, y, x):
    """One output entry Y[n, o, y, x] and its |W|*|X| scale, by direct summation."""
    X = np.asarray(X)
    W = np.asarray(W)
    _, c, h, w = X.shape
    acc = 0.0
    scale = 0.0
    for dy in range(3):
        yy = y + dy - 1
        if yy < 0 or yy >= h:
            continue
        for dx in range(3):
            xx = x + dx - 1
            if xx < 0 or xx >= w:
                continue
            a = np.asarray(W[o, :, dy, dx], np.float64)
            b = np.asarray(X[n, :, yy, xx], np.float64)
            acc += float(np.dot(a, b))
            scale += float(np.dot(np.abs(a), np.abs(b)))
    return acc, scale


# --------------------------------------------------------------------------
# row sum
# --------------------------------------------------------------------------
def rowsum_f64(Z):
    """r[i] = sum_j Z[i, j] in float64, and the scale sum_j |Z[i, j]|."""
    Z = np.asarray(Z, dtype=np.float64)
    return Z.sum(axis=1), np.abs(Z).sum(axis=1)


# --------------------------------------------------------------------------
# row softmax
# --------------------------------------------------------------------------
def softmax_f64(X):
    """y_ij = exp(x_ij - m_i) / sum_l exp(x_il - m_i) with m_i = max_l x_il."""
    X = np.asarray(X, dtype=np.float64)
    m = X.max(axis=1, keepdims=True)
    e = np.exp(X - m)
    return e / e.sum(axis=1, keepdims=True)


# --------------------------------------------------------------------------
# voxel scatter (bird's-eye-view pillars)
# --------------------------------------------------------------------------
VOXEL_NX = 512
VOXEL_NY = 512
VOXEL_XMIN = np.float32(-51.2)
VOXEL_YMIN = np.float32(-51.2)
VOXEL_SCALE = np.float32(5.0)    # 1 / (0.2 m), exactly representable


def voxel_cell_f32(pts, nx=VOXEL_NX, ny=VOXEL_NY, xmin=VOXEL_XMIN,
                   ymin=VOXEL_YMIN, scale=VOXEL_SCALE):
    """Per-point cell index over a half-open grid, decided in float32.

    fx = fl32(fl32(x - xmin) * scale), fy likewise; ix = floor(fx),
    iy = floor(fy).  A point is inside iff 0 <= fx < nx and 0 <= fy < ny
    (NaN and infinities fall outside); its cell is iy * nx + ix, else -1.
    """
    pts = np.asarray(pts, dtype=np.float32)
    assert pts.ndim == 2 and pts.shape[1] == 4
    x = pts[:, 0]
    y = pts[:, 1]
    fx = ((x - np.float32(xmin)).astype(np.float32) * np.float32(scale)).astype(np.float32)
    fy = ((y - np.float32(ymin)).astype(np.float32) * np.float32(scale)).astype(np.float32)
    with np.errstate(invalid="ignore"):
        inside = (fx >= 0) & (fx < np.float32(nx)) & (fy >= 0) & (fy < np.float32(ny))
    ix = np.zeros(len(pts), dtype=np.int64)
    iy = np.zeros(len(pts), dtype=np.int64)
    ix[inside] = np.floor(fx[inside]).astype(np.int64)
    iy[inside] = np.floor(fy[inside]).astype(np.int64)
    v = np.where(inside, iy * nx + ix, -1)
    return v.astype(np.int32)


def voxel_scatter(pts, nx=VOXEL_NX, ny=VOXEL_NY, xmin=VOXEL_XMIN,
                  ymin=VOXEL_YMIN, scale=VOXEL_SCALE):
    """Cell index per point and count / max z / first index per cell.

    Returns (vidx[N] int32, count[G] int32, zmax[G] float32, first[G] int32)
    with G = nx * ny.  An empty cell has count 0, zmax = -inf, first = -1.
    All three per-cell reductions are order independent (a count, a maximum
    and a minimum), so the result is unique.  z is assumed not NaN.
    """
    pts = np.asarray(pts, dtype=np.float32)
    g = nx * ny
    vidx = voxel_cell_f32(pts, nx, ny, xmin, ymin, scale)
    sel = np.nonzero(vidx >= 0)[0]
    cells = vidx[sel].astype(np.int64)
    count = np.bincount(cells, minlength=g).astype(np.int32)
    z = pts[sel, 2]
    zmax = np.full(g, -np.inf, dtype=np.float32)
    np.maximum.at(zmax, cells, z)
    # The maximum is taken in the total order where -0 < +0: a cell whose
    # largest z is a zero holds +0 if any of its points has z = +0.
    pos_zero = np.zeros(g, dtype=bool)
    pz = (z == 0) & ~np.signbit(z)
    pos_zero[cells[pz]] = True
    zero_cells = zmax == 0
    zmax[zero_cells & pos_zero] = np.float32(0.0)
    zmax[zero_cells & ~pos_zero] = np.float32(-0.0)
    first = np.full(g, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(first, cells, sel.astype(np.int64))
    first = np.where(count > 0, first, -1).astype(np.int32)
    return vidx, count, zmax, first


# --------------------------------------------------------------------------
# FP8 (OCP E4M3) matrix product with an FP32 result
# --------------------------------------------------------------------------
def e4m3_decode(codes):
    """Value of each OCP FP8 E4M3 code as float64.

    Bit 7 is the sign, bits 6..3 the exponent field e (bias 7), bits 2..0 the
    mantissa m.  e = 0 encodes subnormals (m / 8) * 2^-6; otherwise the value
    is (1 + m / 8) * 2^(e - 7).  The format has no infinities: exponent and
    mantissa all ones (0x7f, 0xff) is NaN, so the largest finite magnitude is
    0x7e = 1.75 * 2^8 = 448.
    """
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = (c & 0x7).astype(np.float64)
    mag = np.where(e == 0, (m / 8.0) * 2.0 ** -6, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    mag = np.where((e == 0xF) & (c & 0x7 == 0x7), np.nan, mag)
    return sign * mag


def gemm_fp8_f64(A8, Bt8):
    """C[m, n] = sum_k a(A8[m, k]) * a(Bt8[n, k]), a = e4m3_decode.

    A8 is [M, K] and Bt8 is B transposed, [N, K] (both K-contiguous), as
    uint8 codes.  A product of two E4M3 values has at most 8 significant bits
    and is exact in float64, as are sums of up to 2^40 of them at these
    magnitudes, so this is the exact product for the sizes used here.
    """
    A = e4m3_decode(A8)
    B = e4m3_decode(Bt8)
    assert A.ndim == 2 and B.ndim == 2 and A.shape[1] == B.shape[1]
    return A @ B.T


def gemm_fp8_abs_f64(A8, Bt8):
    """|A| |B| for the componentwise error scale of the FP8 product."""
    return np.abs(e4m3_decode(A8)) @ np.abs(e4m3_decode(Bt8)).T


def gemm_fp8_entry_f64(A8, Bt8, m, n):
    """One entry C[m, n] and its scale (|A| |B|)[m, n] for sampled checks."""
    a = e4m3_decode(A8[m])
    b = e4m3_decode(Bt8[n])
    return float(np.dot(a, b)), float(np.dot(np.abs(a), np.abs(b)))


def bf16_decode(codes):
    """Value of each bfloat16 code as float64.

    Bit 15 is the sign, bits 14..7 the exponent field e (bias 127), bits
    6..0 the mantissa m.  e = 0 encodes zero and subnormals (m / 128) *
    2^-126; e = 255 encodes infinity (m = 0) and NaN (m != 0); otherwise the
    value is (1 + m / 128) * 2^(e - 127).  (The format is the upper half of
    an IEEE binary32.)
    """
    c = np.asarray(codes, dtype=np.uint16).astype(np.int64)
    sign = np.where(c & 0x8000, -1.0, 1.0)
    e = (c >> 7) & 0xFF
    m = (c & 0x7F).astype(np.float64)
    with np.errstate(over="ignore"):
        mag = np.where(e == 0, (m / 128.0) * 2.0 ** -126, (1.0 + m / 128.0) * np.exp2(e - 127.0))
    mag = np.where(e == 0xFF, np.where(m == 0, np.inf, np.nan), mag)
    return sign * mag


def gemm_bf16_f64(A16, Bt16):
    """C[m, n] = sum_k d(A16[m, k]) * d(Bt16[n, k]), d = bf16_decode.

    A16 is [M, K] and Bt16 is B transposed, [N, K], as uint16 codes.  A
    product of two bfloat16 values has at most 16 significant bits and is
    exact in float64; for inputs whose exponents span a few binades (the
    generators here) the sums of K <= 2^20 products stay within 53 bits, so
    this is the exact product.
    """
    A = bf16_decode(A16)
    B = bf16_decode(Bt16)
    assert A.ndim == 2 and B.ndim == 2 and A.shape[1] == B.shape[1]
    return A @ B.T


def gemm_bf16_abs_f64(A16, Bt16):
    """|A| |B| for the componentwise error scale of the BF16 product."""
    return np.abs(bf16_decode(A16)) @ np.abs(bf16_decode(Bt16)).T


def gemm_bf16_entry_f64(A16, Bt16, m, n):
    """One entry C[m, n] and its scale (|A| |B|)[m, n] for sampled checks."""
    a = bf16_decode(A16[m])
    b = bf16_decode(Bt16[n])
    return float(np.dot(a, b)), float(np.dot(np.abs(a), np.abs(b)))


def vecadd_f32(A, B):
    """c = fl32(a + b) elementwise: one IEEE float32 addition (round to
    nearest even).  The bit-exact reference of the custom vector-add kernel."""
    return np.asarray(A, dtype=np.float32) + np.asarray(B, dtype=np.float32)


def conv3x3_bf16_f64(X16, W16):
    """The 3x3 convolution of conv3x3_f64 on bfloat16 operands in channels-
    innermost layouts: X16 is [H, W, C] (NHWC of one image), W16 is
    [C_out, 3, 3, C_in] (OHWI), both uint16 codes; the result is [1, C_out,
    H, W] (NCHW) in float64, exact for the sizes used here (every product
    has 16 significant bits)."""
    X = bf16_decode(X16)
    Wt = bf16_decode(W16)
    assert X.ndim == 3 and Wt.ndim == 4 and Wt.shape[1:3] == (3, 3) and Wt.shape[3] == X.shape[2]
    return conv3x3_f64(X.transpose(2, 0, 1)[None], Wt.transpose(0, 3, 1, 2))


def conv3x3_bf16_abs_f64(X16, W16):
    """|W| * |X| for the componentwise error scale of the BF16 convolution."""
    X = np.abs(bf16_decode(X16))
    Wt = np.abs(bf16_decode(W16))
    return conv3x3_f64(X.transpose(2, 0, 1)[None], Wt.transpose(0, 3, 1, 2))
