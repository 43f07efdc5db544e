"""ug_kernel_launch_noalloc (no allocation: a static device workspace)
against ug_kernel_launch (a stream-ordered allocation per call) on the same
inputs: bit-identical outputs for the binned voxel scatter, the one kernel
with a workspace, on two calls in a row (the second on a smaller cloud, over
the first call's leftovers), and for a kernel without one; sizes beyond the
static workspace are refused before any device call."""

import numpy as np
import pytest

from paper_2509_12207_amd import capi

MS = 1_000_000


def _voxel(n):
    return {"op": "voxel", "shape": (n, 512, 512), "in": (0,), "out": (1, 2, 3, 4),
            "fparam": (-51.2, -51.2, 5.0)}


def test_noalloc_refuses_a_workspace_above_the_static_size():
    n = 1 << 24                  # 16 Mi points: far above the static workspace
    assert capi.kernel_workspace(_voxel(n)) > capi.STATIC_SCRATCH_BYTES
    fake = [0x10000 * (i + 1) for i in range(5)]   # never dereferenced
    with pytest.raises(capi.UgError) as e:
        capi.kernel_launch_noalloc(_voxel(n), fake)
    assert e.value.status == capi.EINVAL


@pytest.mark.gpu
def test_noalloc_matches_the_allocating_entry_point():
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(11)
    s = torch.cuda.Stream()
    for n in (3_000_000, (1 << 20) + 12_345):       # both binned; the second smaller
        assert 0 < capi.kernel_workspace(_voxel(n)) <= capi.STATIC_SCRATCH_BYTES
        pts = np.empty((n, 4), np.float32)
        pts[:, :3] = rng.normal(0.0, 20.0, (n, 3))
        pts[:, 3] = rng.uniform(0.0, 1.0, n)
        p = torch.from_numpy(pts).to(dev)
        outs = []
        for launch in (capi.kernel_launch, capi.kernel_launch_noalloc):
            o = [torch.full((n,), 7, dtype=torch.int32, device=dev),
                 torch.full((512 * 512,), 7, dtype=torch.int32, device=dev),
                 torch.full((512 * 512,), 7.0, dtype=torch.float32, device=dev),
                 torch.full((512 * 512,), 7, dtype=torch.int32, device=dev)]
            torch.cuda.synchronize()
            launch(_voxel(n), [p.data_ptr()] + [t.data_ptr() for t in o], s.cuda_stream)
            s.synchronize()
            outs.append([t.cpu().numpy() for t in o])
        for a, b in zip(*outs):
            assert a.dtype == b.dtype and np.array_equal(a.view(np.uint32), b.view(np.uint32))
        assert int(outs[1][1].sum()) == int((outs[1][0] >= 0).sum())
    # a kernel with no workspace goes through unchanged
    A = torch.from_numpy(rng.uniform(-1, 1, (256, 384)).astype(np.float32)).to(dev)
    B = torch.from_numpy(rng.uniform(-1, 1, (384, 128)).astype(np.float32)).to(dev)
    C1 = torch.zeros(256, 128, device=dev)
    C2 = torch.zeros(256, 128, device=dev)
    k = {"op": "gemm", "shape": (256, 128, 384), "in": (0, 1), "out": (2,)}
    capi.kernel_launch(k, [A.data_ptr(), B.data_ptr(), C1.data_ptr()], s.cuda_stream)
    capi.kernel_launch_noalloc(k, [A.data_ptr(), B.data_ptr(), C2.data_ptr()], s.cuda_stream)
    s.synchronize()
    assert torch.equal(C1, C2)
