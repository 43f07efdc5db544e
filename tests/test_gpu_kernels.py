"""Parity of each gfx950 kernel with the oracle, called through the C-ABI
(ug_kernel_launch) on torch-allocated device memory.

Tolerances: bias+ReLU and the voxel scatter are bit-exact; GEMM, conv and row
sum are componentwise within 1e-5 of the absolute-value computation
(|A||B|, |W|*|X|, sum |Z|); softmax within 1e-5 relative per element.
Integer-valued inputs make every partial sum exact, so there the contractions
must match bit for bit.
"""

import numpy as np
import pytest
import torch

from oracle import kernels as OK
from paper_2509_12207_amd import capi

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def launch(desc, tensors):
    capi.kernel_launch(desc, [int(t.data_ptr()) for t in tensors])
    torch.cuda.synchronize()


def rng(seed):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------- GEMM
def run_gemm(A, B):
    M, K = A.shape
    N = B.shape[1]
    a, b = dev(A), dev(B)
    c = torch.full((M, N), float("nan"), device=DEV)
    launch({"op": "gemm", "shape": (M, N, K), "in": (0, 1), "out": (2,)}, [a, b, c])
    return c.cpu().numpy()


# tile variants: small 32x32 with a 4-way K split (most), mid 64x64
# (1024 x 1024, 2048 x 1024), big 128x128 (the full-size test below)
@pytest.mark.parametrize("M,N,K", [(128, 128, 128), (256, 512, 384), (130, 70, 37),
                                   (257, 132, 64), (1, 1, 1), (33, 1000, 19), (512, 256, 4096),
                                   (1024, 1024, 300), (2048, 1024, 64), (1000, 1030, 17)])
def test_gemm_parity(M, N, K):
    r = rng(M * 7 + N * 3 + K)
    A = r.uniform(-1, 1, (M, K)).astype(np.float32)
    B = r.uniform(-1, 1, (K, N)).astype(np.float32)
    C = run_gemm(A, B)
    ref = OK.gemm_f64(A, B)
    scale = OK.gemm_abs_f64(A, B)
    assert np.all(np.abs(C - ref) <= TOL * scale), np.max(np.abs(C - ref) / scale)


@pytest.mark.parametrize("M,N,K", [(128, 128, 128), (300, 200, 100), (64, 96, 2048)])
def test_gemm_integer_inputs_bit_exact(M, N, K):
    r = rng(11 + M)
    A = r.integers(-2, 3, (M, K)).astype(np.float32)
    B = r.integers(-2, 3, (K, N)).astype(np.float32)
    C = run_gemm(A, B)
    assert np.array_equal(C, (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32))


def test_gemm_full_size_sampled():
    """4096^3 (the largest configuration shape), checked on sampled entries."""
    M = N = K = 4096
    g = torch.Generator(device="cpu").manual_seed(5)
    A = (torch.rand(M, K, generator=g) * 2 - 1).numpy()
    B = (torch.rand(K, N, generator=g) * 2 - 1).numpy()
    C = run_gemm(A, B)
    r = rng(6)
    for m, n in zip(r.integers(0, M, 64), r.integers(0, N, 64)):
        v, s = OK.gemm_entry_f64(A, B, m, n)
        assert abs(C[m, n] - v) <= TOL * s
    assert np.isfinite(C).all()


# ---------------------------------------------------------------- bias+ReLU
# (4096, 4100) and (4100, 4096) are over 64 MiB: the streaming (nontemporal) path
@pytest.mark.parametrize("R,Cn,axis", [(128, 128, 0), (16, 4096, 1), (37, 53, 0), (5, 7, 1),
                                       (1024, 1024, 0), (4096, 4100, 0), (4100, 4096, 1)])
def test_bias_relu_bit_exact(R, Cn, axis):
    r = rng(R + Cn + axis)
    X = r.uniform(-1, 1, (R, Cn)).astype(np.float32)
    X.flat[::17] = -0.0
    X.flat[::23] = np.nan
    b = r.uniform(-0.5, 0.5, Cn if axis == 0 else R).astype(np.float32)
    x, bb = dev(X), dev(b)
    y = torch.empty_like(x)
    launch({"op": "bias_relu", "shape": (R, Cn, axis), "in": (0, 1), "out": (2,)}, [x, bb, y])
    want = OK.bias_relu_f32(X, b, axis)
    got = y.cpu().numpy()
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    # in place
    launch({"op": "bias_relu", "shape": (R, Cn, axis), "in": (0, 1), "out": (0,)}, [x, bb])
    assert np.array_equal(x.cpu().numpy().view(np.uint32), want.view(np.uint32))


# --------------------------------------------------------------------- conv
def run_conv(X, W):
    n, c, h, w = X.shape
    x, wt = dev(X), dev(W)
    y = torch.full((n, c, h, w), float("nan"), device=DEV)
    launch({"op": "conv3x3", "shape": (n, c, h, w), "in": (0, 1), "out": (2,)}, [x, wt, y])
    return y.cpu().numpy()


# tile variants: (1, 96, 96, 96) -> 64 ch x 2x16 px with a K split,
# (1, 64, 128, 128) and (1, 32, 256, 256) -> 32 ch x 8x16 px, (1, 1, 1, 1) ->
# 32 ch x 8x16 px (one workgroup either way; ties go to the larger tile), the
# rest -> 32 ch x 2x16 px with a K split; 64 ch x 8x16 px and 128 ch x 8x16 px
# in the sampled tests below
@pytest.mark.parametrize("n,c,h,w", [(1, 16, 64, 64), (1, 32, 32, 32), (1, 64, 32, 48),
                                     (1, 130, 20, 20), (2, 3, 13, 21), (1, 1, 1, 1),
                                     (1, 256, 16, 16), (1, 64, 128, 128), (1, 32, 256, 256),
                                     (1, 100, 33, 47), (1, 96, 96, 96)])
def test_conv_parity(n, c, h, w):
    r = rng(n + 5 * c + 7 * h + w)
    X = r.uniform(-1, 1, (n, c, h, w)).astype(np.float32)
    W = r.uniform(-1, 1, (c, c, 3, 3)).astype(np.float32)
    Y = run_conv(X, W)
    ref = OK.conv3x3_f64(X, W)
    scale = OK.conv3x3_abs_f64(X, W)
    assert np.all(np.abs(Y - ref) <= TOL * scale + 1e-30), np.nanmax(np.abs(Y - ref) / (scale + 1e-30))


def test_conv_integer_inputs_bit_exact():
    r = rng(77)
    X = r.integers(-2, 3, (1, 48, 24, 40)).astype(np.float32)
    W = r.integers(-2, 3, (48, 48, 3, 3)).astype(np.float32)
    assert np.array_equal(run_conv(X, W), OK.conv3x3_f64(X, W).astype(np.float32))


@pytest.mark.parametrize("c", [256, 64])
def test_conv_full_size_sampled(c):
    """C = 256, H = W = 256 (the largest configuration shape; 128-channel
    tiles) and C = 64 (64-channel tiles), sampled entries."""
    r = rng(78 + c)
    X = r.uniform(-1, 1, (1, c, 256, 256)).astype(np.float32)
    W = r.uniform(-1, 1, (c, c, 3, 3)).astype(np.float32)
    Y = run_conv(X, W)
    pts = list(zip(r.integers(0, c, 48), r.integers(0, 256, 48), r.integers(0, 256, 48)))
    pts += [(0, 0, 0), (c - 1, 255, 255), (17, 0, 255), (3, 255, 0)]
    for o, y, x in pts:
        v, s = OK.conv3x3_entry_f64(X, W, 0, o, y, x)
        assert abs(Y[0, o, y, x] - v) <= TOL * s


# ------------------------------------------------------------------- rowsum
@pytest.mark.parametrize("R,Cn", [(1024, 64), (7, 5), (3, 5000), (300, 2048), (2, 16384),
                                  (4096, 1)])
def test_rowsum_parity(R, Cn):
    r = rng(R * 3 + Cn)
    Z = r.uniform(-1, 1, (R, Cn)).astype(np.float32)
    z = dev(Z)
    out = torch.full((R,), float("nan"), device=DEV)
    launch({"op": "rowsum", "shape": (R, Cn), "in": (0,), "out": (1,)}, [z, out])
    s, a = OK.rowsum_f64(Z)
    assert np.all(np.abs(out.cpu().numpy() - s) <= TOL * a)


def test_rowsum_integer_exact():
    r = rng(9)
    Z = r.integers(-2, 3, (100, 3000)).astype(np.float32)
    z = dev(Z)
    out = torch.empty(100, device=DEV)
    launch({"op": "rowsum", "shape": (100, 3000), "in": (0,), "out": (1,)}, [z, out])
    assert np.array_equal(out.cpu().numpy(), Z.astype(np.int64).sum(1).astype(np.float32))


# ------------------------------------------------------------------ softmax
# (8193, 2048) and (4097, 4096) are over 64 MiB: the streaming (nontemporal) path
@pytest.mark.parametrize("R,L", [(256, 128), (5, 3), (64, 256), (33, 1000), (16, 1024),
                                 (9, 2048), (8, 4096), (3, 5000), (7, 1), (8193, 2048),
                                 (4097, 4096)])
def test_softmax_parity(R, L):
    r = rng(R + L)
    X = r.uniform(-8, 8, (R, L)).astype(np.float32)
    x = dev(X)
    y = torch.full_like(x, float("nan"))
    launch({"op": "softmax", "shape": (R, L), "in": (0,), "out": (1,)}, [x, y])
    ref = OK.softmax_f64(X)
    got = y.cpu().numpy()
    big = ref >= 1e-30
    assert np.all(np.abs(got[big] - ref[big]) <= TOL * ref[big])
    assert np.all(np.abs(got[~big]) <= 1e-37)


# -------------------------------------------------------------------- voxel
def run_voxel(P, nx=512, ny=512, fp=(-51.2, -51.2, 5.0)):
    n = len(P)
    p = dev(P.reshape(-1)) if n else torch.zeros(4, device=DEV)
    G = nx * ny
    vi = torch.full((max(n, 1),), 7, dtype=torch.int32, device=DEV)
    vc = torch.full((G,), 7, dtype=torch.int32, device=DEV)
    vz = torch.full((G,), 7.0, device=DEV)
    vf = torch.full((G,), 7, dtype=torch.int32, device=DEV)
    launch({"op": "voxel", "shape": (n, nx, ny), "in": (0,), "out": (1, 2, 3, 4), "fparam": fp},
           [p, vi, vc, vz, vf])
    return vi.cpu().numpy()[:n], vc.cpu().numpy(), vz.cpu().numpy(), vf.cpu().numpy()


@pytest.mark.parametrize("n", [1000, 120_000, 1])
def test_voxel_bit_exact(n):
    r = rng(n)
    P = np.concatenate([r.normal(0, 20, (n, 3)), r.uniform(0, 1, (n, 1))], axis=1).astype(np.float32)
    got = run_voxel(P)
    want = OK.voxel_scatter(P)
    for g, w in zip(got, want):
        assert np.array_equal(np.asarray(g).view(np.uint32), np.asarray(w).view(np.uint32))


def test_voxel_boundaries_and_empty():
    P = np.array([[-51.2, 0.1, 1.0, 0], [51.2, 0.1, 2.0, 0], [-51.2001, 0.1, 3, 0],
                  [51.19, 51.19, -4.0, 0], [np.nan, 0, 0, 0], [0.1, 0.1, -0.0, 0],
                  [0.1, 0.1, 0.0, 0], [0.1, 0.15, -7.0, 0], [np.inf, 1, 1, 0]], np.float32)
    got = run_voxel(P)
    want = OK.voxel_scatter(P)
    for g, w in zip(got, want):
        assert np.array_equal(np.asarray(g).view(np.uint32), np.asarray(w).view(np.uint32))
    vi, vc, vz, vf = run_voxel(np.zeros((0, 4), np.float32))
    assert vc.sum() == 0 and np.all(vf == -1) and np.all(np.isneginf(vz))


def test_voxel_small_grid_ragged():
    r = rng(3)
    P = np.concatenate([r.normal(0, 1, (5000, 3)), r.uniform(0, 1, (5000, 1))], 1).astype(np.float32)
    fp = (-1.4, -1.0, 5.0)
    got = run_voxel(P, 7, 5, fp)
    want = OK.voxel_scatter(P, 7, 5, np.float32(fp[0]), np.float32(fp[1]), np.float32(fp[2]))
    for g, w in zip(got, want):
        assert np.array_equal(np.asarray(g).view(np.uint32), np.asarray(w).view(np.uint32))


def _same(got, want):
    for g, w in zip(got, want):
        assert np.array_equal(np.asarray(g).view(np.uint32), np.asarray(w).view(np.uint32))


def _cloud(seed, n, sigma=20.0):
    r = rng(seed)
    return np.concatenate([r.normal(0, sigma, (n, 3)), r.uniform(0, 1, (n, 1))],
                          axis=1).astype(np.float32)


# Large clouds take the binned path (tiles of 4096 cells, chunks of 8192
# points, reduce workgroups over groups of chunks): sizes that are ragged in
# all three (8 Mi + 5 points: 1025 chunks in 8 groups of up to 129).
@pytest.mark.parametrize("n", [1 << 20, 1_100_003, (8 << 20) + 5])
def test_voxel_binned_bit_exact(n):
    P = _cloud(n, n)
    assert capi.kernel_workspace({"op": "voxel", "shape": (n, 512, 512), "in": (0,),
                                  "out": (1, 2, 3, 4), "fparam": (-51.2, -51.2, 5.0)}) > 0
    _same(run_voxel(P), OK.voxel_scatter(P))


def test_voxel_binned_hot_cell_many_segments():
    # 1.2 M points in one cell (every chunk's whole run in one tile), signed zeros and
    # -inf among its z values, a few points elsewhere and outside
    n = 1_200_000
    r = rng(11)
    P = np.zeros((n, 4), np.float32)
    P[:, 0], P[:, 1] = 0.05, 0.05
    P[:, 2] = r.uniform(-5, 0, n).astype(np.float32)
    P[7, 2], P[8, 2], P[9, 2] = -0.0, 0.0, -np.inf
    P[::1000, 0] = r.uniform(-60, 60, len(P[::1000])).astype(np.float32)
    P[5, 2] = np.float32(-1e-30)
    got = run_voxel(P)
    want = OK.voxel_scatter(P)
    _same(got, want)
    assert got[1].max() > 1_000_000


def test_voxel_binned_odd_grid_and_workspace_api():
    # G = 30000 cells: 8 tiles, the last one partial; explicit workspace
    n, nx, ny = (1 << 20) + 5, 300, 100
    fp = (-30.0, -10.0, 5.0)
    r = rng(5)
    P = np.concatenate([r.uniform(-31, 31, (n, 1)), r.uniform(-11, 11, (n, 1)),
                        r.normal(0, 3, (n, 1)), r.uniform(0, 1, (n, 1))], 1).astype(np.float32)
    desc = {"op": "voxel", "shape": (n, nx, ny), "in": (0,), "out": (1, 2, 3, 4), "fparam": fp}
    need = capi.kernel_workspace(desc)
    assert need > 0
    p = dev(P.reshape(-1))
    G = nx * ny
    outs = [torch.full((n,), 7, dtype=torch.int32, device=DEV),
            torch.full((G,), 7, dtype=torch.int32, device=DEV), torch.full((G,), 7.0, device=DEV),
            torch.full((G,), 7, dtype=torch.int32, device=DEV)]
    ptrs = [int(t.data_ptr()) for t in [p] + outs]
    small = torch.empty(need // 2, dtype=torch.uint8, device=DEV)
    with pytest.raises(capi.UgError) as e:
        capi.kernel_launch_ws(desc, ptrs, int(small.data_ptr()), small.numel())
    assert e.value.status == capi.EINVAL
    ws = torch.full((need,), 0xA5, dtype=torch.uint8, device=DEV)   # stale contents
    for _ in range(2):                                               # reuse holds no state
        capi.kernel_launch_ws(desc, ptrs, int(ws.data_ptr()), need)
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in outs]
        _same(got, OK.voxel_scatter(P, nx, ny, np.float32(fp[0]), np.float32(fp[1]),
                                    np.float32(fp[2])))


def test_voxel_large_grid_takes_direct_path():
    # 4096 x 4096 cells exceed the binned path's 1024 tiles: no workspace
    n, nx, ny = 1 << 20, 4096, 4096
    fp = (-51.2, -51.2, 40.0)
    desc = {"op": "voxel", "shape": (n, nx, ny), "in": (0,), "out": (1, 2, 3, 4), "fparam": fp}
    assert capi.kernel_workspace(desc) == 0
    P = _cloud(2, n)
    _same(run_voxel(P, nx, ny, fp),
          OK.voxel_scatter(P, nx, ny, np.float32(fp[0]), np.float32(fp[1]), np.float32(fp[2])))


def test_voxel_binned_through_the_gate():
    # a registered kernel gets its workspace at registration
    n = 1_050_000
    P = _cloud(9, n)
    desc = {"op": "voxel", "shape": (n, 512, 512), "in": (0,), "out": (1, 2, 3, 4),
            "fparam": (-51.2, -51.2, 5.0)}
    G = 512 * 512
    p = dev(P.reshape(-1))
    outs = [torch.full((n,), 7, dtype=torch.int32, device=DEV),
            torch.full((G,), 7, dtype=torch.int32, device=DEV), torch.full((G,), 7.0, device=DEV),
            torch.full((G,), 7, dtype=torch.int32, device=DEV)]
    ptrs = [int(t.data_ptr()) for t in [p] + outs]
    g = capi.Gate("urgency")
    g.register_chain(100_000_000, 100_000_000, [{"kernels": [desc]}], 5)
    g.profile(0, ptrs, warmup=1, reps=2)
    g.start()
    g.submit(0, -1, ptrs)
    g.drain(30.0)
    comps = g.poll()
    g.stop()
    g.close()
    assert len(comps) == 1
    _same([t.cpu().numpy() for t in outs], OK.voxel_scatter(P))


def test_kernel_launch_rejects_bad_descriptors():
    a = torch.zeros(16, device=DEV)
    with pytest.raises(capi.UgError):
        capi.kernel_launch({"op": "gemm", "shape": (4, 4, 0), "in": (0, 0), "out": (0,)},
                           [a.data_ptr()])
    with pytest.raises(capi.UgError):
        capi.kernel_launch({"op": "rowsum", "shape": (4, 4), "in": (0,), "out": (3,)},
                           [a.data_ptr()])
    u = capi.kernel_util({"op": "gemm", "shape": (4096, 4096, 4096), "in": (0, 1), "out": (2,)})
    assert u == 1.0
    u = capi.kernel_util({"op": "rowsum", "shape": (8, 64), "in": (0,), "out": (1,)})
    assert u == 2 / 256          # 2 workgroups of 256 CUs
    u = capi.kernel_util({"op": "gemm", "shape": (256, 256, 256), "in": (0, 1), "out": (2,)})
    assert u == 64 / 256         # 32 x 32 tiles


# ----------------------------------------------------------------- FP8 GEMM
def _fp8_codes(r, shape, lo=4, hi=9):
    """Random finite E4M3 codes: random sign and mantissa, exponent field in
    [lo, hi] (magnitudes 2^-3 .. 7.5 for the defaults)."""
    s = r.integers(0, 2, shape) << 7
    e = r.integers(lo, hi + 1, shape) << 3
    m = r.integers(0, 8, shape)
    return (s | e | m).astype(np.uint8)


def fp8_bound(A8, Bt8):
    """Componentwise error bound of the FP8 product on the matrix cores.

    One instruction sums the 64 products of a K block in a fixed-point
    window whose lowest bit is 2^(e - 13), e = floor(log2) of the block's
    largest product magnitude (measured on gfx950: a product 2^13 times
    smaller than the largest is kept exactly, one 2^14 times smaller is
    dropped).  Each of the block's 64 products loses less than one such bit,
    so a block errs by less than 64 * 2^-13 * max|a_k b_k| (the largest
    product over the block, or the larger max|a| * max|b| for big inputs).
    The block sums are then accumulated in FP32: at most K/64 + 1 roundings
    of 2^-24 relative to the running |A||B|."""
    M, K = A8.shape
    N = Bt8.shape[0]
    nb = (K + 63) // 64
    pad = nb * 64 - K
    a = np.abs(OK.e4m3_decode(np.pad(A8, ((0, 0), (0, pad))))).reshape(M, nb, 64)
    b = np.abs(OK.e4m3_decode(np.pad(Bt8, ((0, 0), (0, pad))))).reshape(N, nb, 64)
    if M * N * K <= 1 << 27:
        pmax = np.zeros((M, N))
        for j in range(nb):
            pmax += (a[:, None, j, :] * b[None, :, j, :]).max(axis=2)
    else:
        pmax = a.max(axis=2) @ b.max(axis=2).T
    return 64 * 2.0 ** -13 * pmax + (nb + 1) * 2.0 ** -24 * OK.gemm_fp8_abs_f64(A8, Bt8)


def run_gemm_fp8(A8, Bt8):
    M, K = A8.shape
    N = Bt8.shape[0]
    a, b = dev(A8), dev(Bt8)
    c = torch.full((M, N), float("nan"), device=DEV)
    launch({"op": "gemm_fp8", "shape": (M, N, K), "in": (0, 1), "out": (2,)}, [a, b, c])
    return c.cpu().numpy()


def test_gemm_fp8_integer_codes_bit_exact():
    # codes of 0, +-1, +-2: every partial sum is a small integer, exact in
    # any order; two tiles by two, ragged M and N, K tail not a multiple of
    # the 128-byte step
    r = rng(21)
    table = np.array([0x00, 0x38, 0xB8, 0x40, 0xC0], np.uint8)
    M, N, K = 300, 270, 208
    A8, B8 = table[r.integers(0, 5, (M, K))], table[r.integers(0, 5, (N, K))]
    C = run_gemm_fp8(A8, B8)
    assert np.array_equal(C, OK.gemm_fp8_f64(A8, B8).astype(np.float32))


def test_gemm_fp8_integer_codes_bit_exact_ring():
    # the same integer codes through the K-multiple-of-64 kernel: one, two,
    # three (odd) and five K steps, ragged M and N below and above one tile
    r = rng(22)
    table = np.array([0x00, 0x38, 0xB8, 0x40, 0xC0], np.uint8)
    for M, N, K in [(300, 270, 64), (33, 257, 128), (256, 256, 192), (513, 100, 320)]:
        A8, B8 = table[r.integers(0, 5, (M, K))], table[r.integers(0, 5, (N, K))]
        C = run_gemm_fp8(A8, B8)
        assert np.array_equal(C, OK.gemm_fp8_f64(A8, B8).astype(np.float32)), (M, N, K)


# K a multiple of 64 takes the direct-to-LDS ring kernel, other multiples of
# 16 the register-staged one
@pytest.mark.parametrize("M,N,K", [(256, 256, 128), (512, 768, 1024), (77, 513, 16),
                                   (1, 1, 16), (1000, 300, 4096), (1, 1, 64), (700, 900, 448),
                                   (300, 257, 1088), (64, 1000, 208)])
def test_gemm_fp8_parity(M, N, K):
    r = rng(M + 3 * N + 7 * K)
    A8, B8 = _fp8_codes(r, (M, K)), _fp8_codes(r, (N, K))
    C = run_gemm_fp8(A8, B8)
    ref = OK.gemm_fp8_f64(A8, B8)
    bound = fp8_bound(A8, B8)
    assert np.all(np.abs(C - ref) <= bound), np.max(np.abs(C - ref) / bound)


@pytest.mark.parametrize("small", [0x38, 0x30, 0x20, 0x18, 0x04, 0x02, 0x01])
def test_gemm_fp8_wide_range_block(small):
    # one large product (256) and 63 small ones in a K block of row 0 and
    # column 0; the other rows and columns random
    r = rng(small)
    M = N = 32
    K = 128
    A8, B8 = _fp8_codes(r, (M, K)), _fp8_codes(r, (N, K))
    A8[0, :64] = small
    A8[0, 0] = 0x78
    B8[0, :] = 0x38
    C = run_gemm_fp8(A8, B8)
    ref = OK.gemm_fp8_f64(A8, B8)
    bound = fp8_bound(A8, B8)
    assert np.isfinite(C).all()
    assert np.all(np.abs(C - ref) <= bound), (C[0, 0], ref[0, 0], bound[0, 0])


def test_gemm_fp8_full_size_sampled():
    # the 8192^3 product of the overload workload, checked on sampled entries
    M = N = K = 8192
    r = rng(8)
    A8, B8 = _fp8_codes(r, (M, K)), _fp8_codes(r, (N, K))
    C = run_gemm_fp8(A8, B8)
    assert not np.isnan(C).any()
    pts = list(zip(r.integers(0, M, 64), r.integers(0, N, 64)))
    pts += [(0, 0), (M - 1, N - 1), (255, 256), (4095, 8191)]
    for m, n in pts:
        v, _ = OK.gemm_fp8_entry_f64(A8, B8, m, n)
        bound = fp8_bound(A8[m:m + 1], B8[n:n + 1])[0, 0]
        assert abs(C[m, n] - v) <= bound, (m, n, C[m, n], v)


def test_gemm_fp8_rejects_bad_k_and_alignment():
    a = torch.zeros(4096, dtype=torch.uint8, device=DEV)
    c = torch.zeros(64, device=DEV)
    with pytest.raises(capi.UgError):
        capi.kernel_launch({"op": "gemm_fp8", "shape": (8, 8, 24), "in": (0, 1), "out": (2,)},
                           [a.data_ptr(), a.data_ptr(), c.data_ptr()])
    with pytest.raises(capi.UgError):
        capi.kernel_launch({"op": "gemm_fp8", "shape": (8, 8, 32), "in": (0, 1), "out": (2,)},
                           [a.data_ptr() + 1, a.data_ptr(), c.data_ptr()])


# ---------------------------------------------------------------- BF16 GEMM
def _bf16_codes(r, shape, lo=124, hi=129):
    """Random finite bfloat16 codes: random sign and mantissa, exponent field
    in [lo, hi] (magnitudes 2^-3 .. 4 for the defaults)."""
    s = r.integers(0, 2, shape) << 15
    e = r.integers(lo, hi + 1, shape) << 7
    m = r.integers(0, 128, shape)
    return (s | e | m).astype(np.uint16)


def bf16_bound(A16, Bt16):
    """Componentwise error bound of the BF16 product with FP32 accumulation.

    Every product of two bfloat16 values is exact in FP32 (16 significant
    bits); the K products are then summed in FP32 in some order, each of the
    at most K additions erring by less than one unit in the last place
    (2^-23 relative, which covers truncation as well as rounding to
    nearest), so |C - C64| <= gamma_K |A| |B| with gamma_K = K u / (1 - K u),
    u = 2^-23."""
    K = A16.shape[1]
    u = 2.0 ** -23
    return K * u / (1 - K * u) * OK.gemm_bf16_abs_f64(A16, Bt16)


def run_gemm_bf16(A16, Bt16):
    M, K = A16.shape
    N = Bt16.shape[0]
    a = torch.from_numpy(A16.view(np.int16).copy()).to(DEV)
    b = torch.from_numpy(Bt16.view(np.int16).copy()).to(DEV)
    c = torch.full((M, N), float("nan"), device=DEV)
    launch({"op": "gemm_bf16", "shape": (M, N, K), "in": (0, 1), "out": (2,)}, [a, b, c])
    return c.cpu().numpy()


def test_gemm_bf16_integer_codes_bit_exact():
    # codes of 0, +-1, +-2, +-3: every partial sum is a small integer, exact
    # in any order; one, two, three (odd) and five K steps, ragged M and N
    r = rng(31)
    table = np.array([0x0000, 0x3F80, 0xBF80, 0x4000, 0xC000, 0x4040, 0xC040], np.uint16)
    for M, N, K in [(300, 270, 32), (33, 257, 64), (256, 256, 96), (513, 100, 160)]:
        A16, B16 = table[r.integers(0, 7, (M, K))], table[r.integers(0, 7, (N, K))]
        C = run_gemm_bf16(A16, B16)
        assert np.array_equal(C, OK.gemm_bf16_f64(A16, B16).astype(np.float32)), (M, N, K)


@pytest.mark.parametrize("M,N,K", [(256, 256, 64), (512, 768, 1024), (77, 513, 32), (1, 1, 32),
                                   (1000, 300, 4096), (700, 900, 224)])
def test_gemm_bf16_parity(M, N, K):
    r = rng(M + 5 * N + 11 * K)
    A16, B16 = _bf16_codes(r, (M, K)), _bf16_codes(r, (N, K))
    C = run_gemm_bf16(A16, B16)
    ref = OK.gemm_bf16_f64(A16, B16)
    bound = bf16_bound(A16, B16)
    assert np.all(np.abs(C - ref) <= bound), np.max(np.abs(C - ref) / bound)
    # and the componentwise criterion of the FP32 kernels
    assert np.all(np.abs(C - ref) <= TOL * OK.gemm_bf16_abs_f64(A16, B16))


def test_gemm_bf16_full_size_sampled():
    # the 4096^3 roofline shape, checked on sampled entries
    M = N = K = 4096
    r = rng(9)
    A16, B16 = _bf16_codes(r, (M, K)), _bf16_codes(r, (N, K))
    C = run_gemm_bf16(A16, B16)
    assert not np.isnan(C).any()
    pts = list(zip(r.integers(0, M, 64), r.integers(0, N, 64)))
    pts += [(0, 0), (M - 1, N - 1), (255, 256), (4095, 0)]
    u = 2.0 ** -23
    for m, n in pts:
        v, sc = OK.gemm_bf16_entry_f64(A16, B16, m, n)
        assert abs(C[m, n] - v) <= K * u / (1 - K * u) * sc, (m, n, C[m, n], v)


def test_gemm_bf16_rejects_bad_k_and_alignment():
    a = torch.zeros(4096, dtype=torch.int16, device=DEV)
    c = torch.zeros(64, device=DEV)
    with pytest.raises(capi.UgError):
        capi.kernel_launch({"op": "gemm_bf16", "shape": (8, 8, 48), "in": (0, 1), "out": (2,)},
                           [a.data_ptr(), a.data_ptr(), c.data_ptr()])
    with pytest.raises(capi.UgError):
        capi.kernel_launch({"op": "gemm_bf16", "shape": (8, 8, 32), "in": (0, 1), "out": (2,)},
                           [a.data_ptr() + 2, a.data_ptr(), c.data_ptr()])


# --------------------------------------------------------------- vector add
@pytest.mark.parametrize("n,w,r,off", [(1, 1, 1, 0), (1000003, 256, 1, 0), (4099, 3, 2, 0),
                                       (65536, 64, 0, 1), (777, 1024, 3, 3)])
def test_vecadd_bit_exact(n, w, r, off):
    # off > 0 shifts every array by `off` floats: misaligned, scalar path
    g = rng(n + w)
    A = (g.standard_normal(n + off) * 1e3).astype(np.float32)
    B = (g.standard_normal(n + off) * 1e-3).astype(np.float32)
    a, b = dev(A), dev(B)
    c = torch.full((n + off,), float("nan"), device=DEV)
    ptrs = [int(a.data_ptr()) + 4 * off, int(b.data_ptr()) + 4 * off, int(c.data_ptr()) + 4 * off]
    capi.kernel_launch({"op": "vecadd", "shape": (n, w, r), "in": (0, 1), "out": (2,)}, ptrs)
    torch.cuda.synchronize()
    got = c.cpu().numpy()[off:]
    assert np.array_equal(got.view(np.uint32), OK.vecadd_f32(A[off:], B[off:]).view(np.uint32))
    assert capi.kernel_util({"op": "vecadd", "shape": (n, w, r), "in": (0, 1), "out": (2,)}) == \
        min(1.0, w / 256)


# ---------------------------------------------------------------- BF16 conv
def run_conv_bf16(X16, W16):
    H, W, C = X16.shape
    x = torch.from_numpy(X16.view(np.int16).copy()).to(DEV)
    w = torch.from_numpy(W16.view(np.int16).copy()).to(DEV)
    y = torch.full((C * H * W,), float("nan"), device=DEV)
    launch({"op": "conv3x3_bf16", "shape": (1, C, H, W), "in": (0, 1), "out": (2,)}, [x, w, y])
    return y.cpu().numpy().reshape(1, C, H, W)


def test_conv3x3_bf16_integer_codes_bit_exact():
    r = rng(51)
    table = np.array([0x0000, 0x3F80, 0xBF80, 0x4000, 0xC000], np.uint16)
    for C, H, W in [(32, 5, 7), (64, 17, 23), (32, 1, 1)]:
        X16 = table[r.integers(0, 5, (H, W, C))]
        W16 = table[r.integers(0, 5, (C, 3, 3, C))]
        got = run_conv_bf16(X16, W16)
        assert np.array_equal(got, OK.conv3x3_bf16_f64(X16, W16).astype(np.float32)), (C, H, W)


@pytest.mark.parametrize("C,H,W", [(32, 8, 8), (96, 33, 30), (256, 16, 20), (128, 3, 300)])
def test_conv3x3_bf16_parity(C, H, W):
    r = rng(C + 7 * H + 13 * W)
    X16, W16 = _bf16_codes(r, (H, W, C)), _bf16_codes(r, (C, 3, 3, C))
    got = run_conv_bf16(X16, W16)
    ref = OK.conv3x3_bf16_f64(X16, W16)
    scale = OK.conv3x3_bf16_abs_f64(X16, W16)
    K = 9 * C
    u = 2.0 ** -23
    assert np.all(np.abs(got - ref) <= K * u / (1 - K * u) * scale)
    assert np.all(np.abs(got - ref) <= TOL * scale)


def test_conv3x3_bf16_full_size_sampled():
    # the roofline shape, C = 256 at 256 x 256, on sampled outputs
    C, H, W = 256, 256, 256
    r = rng(52)
    X16, W16 = _bf16_codes(r, (H, W, C)), _bf16_codes(r, (C, 3, 3, C))
    got = run_conv_bf16(X16, W16)
    assert not np.isnan(got).any()
    x, w = OK.bf16_decode(X16), OK.bf16_decode(W16)
    K = 9 * C
    u = 2.0 ** -23
    pts = [(int(o), int(y), int(xx)) for o, y, xx in zip(r.integers(0, C, 48), r.integers(0, H, 48),
                                                          r.integers(0, W, 48))]
    pts += [(0, 0, 0), (C - 1, H - 1, W - 1), (5, 0, W - 1), (200, H - 1, 0)]
    for o, y, xx in pts:
        v = sc = 0.0
        for dy in range(3):
            for dx in range(3):
                yy, xc = y + dy - 1, xx + dx - 1
                if 0 <= yy < H and 0 <= xc < W:
                    p = w[o, dy, dx, :] * x[yy, xc, :]
                    v += float(p.sum())
                    sc += float(np.abs(p).sum())
        assert abs(got[0, o, y, xx] - v) <= K * u / (1 - K * u) * sc, (o, y, xx)


def test_conv3x3_bf16_rejects_bad_shapes():
    a = torch.zeros(4096, dtype=torch.int16, device=DEV)
    c = torch.zeros(4096, device=DEV)
    for shape in [(1, 48, 4, 4), (2, 32, 4, 4), (1, 32, 0, 4)]:
        with pytest.raises(capi.UgError):
            capi.kernel_launch({"op": "conv3x3_bf16", "shape": shape, "in": (0, 1), "out": (2,)},
                               [a.data_ptr(), a.data_ptr(), c.data_ptr()])
