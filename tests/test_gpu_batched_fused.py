"""GPU parity of the fused batched kernel: one workgroup per (ROI, block of 16 y-slices)
projects the block's slices into LDS and takes their matrix-core power sums there.

Every batch below is one the planner gives to the fused kernel (its workspace has no row
buffer, so it is smaller than with DPM_BATCH_FUSED=0).  Each ROI's moments must equal the
exact direct sums of eq. (2) (the C oracle), and the whole output must equal, bit for
bit, the same call through the separate projection and power-sum kernels.
"""
import sys

import numpy as np
import pytest

import oracle.native as onative
import synth
from gpu_util import assert_moments_equal

pytestmark = pytest.mark.gpu

# (N, M, L) numpy shapes, i.e. z, y, x: one slice (M = 1), fewer slices than waves,
# exactly one block of 16, a ragged block (17), several blocks, both dtypes.
SMALL = [((9, 1, 7), np.uint8), ((13, 3, 11), np.uint8), ((20, 16, 21), np.uint8), ((17, 17, 30), np.uint8),
         ((40, 33, 45), np.uint16), ((5, 70, 3), np.uint16), ((31, 48, 64), np.uint8), ((1, 2, 1), np.uint16)]
# uint8 rows wider than 257 voxels: line sums can pass 2^16, rows held as 32-bit values
WIDE8 = [((2, 35, 260), np.uint8), ((3, 20, 9), np.uint8)]


@pytest.fixture(scope="module")
def dpm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2012_08099_amd as m
    m.lib()
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(spec, seed):
    out = []
    for i, (shape, dt) in enumerate(spec):
        if dt == np.uint8 and min(shape) >= 8:
            out.append(synth.sphere_mask(shape, np.random.default_rng(seed + i)))
        else:
            out.append(synth.uniform_volume(shape, dt, seed=seed + i))
    return out


def run(dpm, rois, K, monkeypatch, fused):
    import torch
    monkeypatch.setenv("DPM_BATCH_FUSED", "1" if fused else "0")
    packed, desc = dpm.pack_rois(rois, "cuda:0")
    n, nm, nm4 = len(rois), dpm.num_moments(K), dpm.num_moments(min(K, 4))
    ex = torch.zeros((n * nm4, 2), dtype=torch.int64, device="cuda:0")
    fp = torch.zeros(n * nm, dtype=torch.float64, device="cuda:0")
    wsb = dpm.batched_workspace_bytes(desc, K)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda:0")
    dpm.moments_batched(packed, desc, K, ex, fp, ws)
    torch.cuda.synchronize()
    return wsb, ex.cpu(), fp.cpu().numpy()


def check(dpm, rois, K, monkeypatch, what):
    say(what, "K", K, [r.shape for r in rois][:4])
    ws_f, ex_f, fp_f = run(dpm, rois, K, monkeypatch, True)
    ws_s, ex_s, fp_s = run(dpm, rois, K, monkeypatch, False)
    assert ws_f < ws_s, "the planner did not take the fused kernel"
    nm, nm4 = dpm.num_moments(K), dpm.num_moments(min(K, 4))
    exact = dpm._exact_from_tensor(ex_f)
    for i, V in enumerate(rois):
        got = dpm.Moments(K, exact[i * nm4:(i + 1) * nm4], fp_f[i * nm:(i + 1) * nm])
        assert_moments_equal(got, onative.moments_hoisted(V, K), K, f"{what} roi {i} {V.shape}")
    assert np.array_equal(ex_f.numpy(), ex_s.numpy()), f"{what}: exact moments differ from the separate kernels"
    assert np.array_equal(fp_f.view(np.uint64), fp_s.view(np.uint64)), f"{what}: FP64 differs"


@pytest.mark.parametrize("K", [0, 1, 2, 3, 4, 5, 6])
def test_fused_small_mix_every_order(dpm, monkeypatch, K):
    check(dpm, make(SMALL, 10 * K), K, monkeypatch, "small mix")


@pytest.mark.parametrize("K", [2, 3])
def test_fused_wide_uint8_rows_as_32bit(dpm, monkeypatch, K):
    check(dpm, make(WIDE8, 7), K, monkeypatch, "wide uint8")


def test_fused_sphere_cube_order6(dpm, monkeypatch):
    rois = [synth.sphere_mask((96, 96, 96), np.random.default_rng(3)), synth.sphere_mask((50, 61, 77),
                                                                                           np.random.default_rng(4))]
    check(dpm, rois, 6, monkeypatch, "sphere 96^3")


def test_fused_uint16_order4(dpm, monkeypatch):
    rois = [synth.mri_phantom((64, 20, 96), seed=1), synth.uniform_volume((33, 47, 29), np.uint16, seed=2)]
    check(dpm, rois, 4, monkeypatch, "uint16")


def test_fused_roi_batch_1000(dpm, monkeypatch):
    """The bench's batch: 1000 uint8 sphere ROIs U{8..96}^3 at order 4."""
    check(dpm, synth.roi_batch(1000, seed=1), 4, monkeypatch, "1000 ROIs")


def test_fused_and_separate_rois_in_one_batch(dpm, monkeypatch):
    """ROIs whose block fits the fused kernel take it, the others (a 128^3 sphere and a
    long uint16 column at order 6) the separate kernels, in one call."""
    rng = np.random.default_rng(12)
    rois = [synth.sphere_mask((128, 128, 128), rng), synth.sphere_mask((40, 33, 50), rng),
            synth.uniform_volume((3, 70, 2), np.uint16, seed=4), synth.uniform_volume((900, 2, 3), np.uint16, seed=5),
            synth.sphere_mask((20, 17, 90), rng)]
    check(dpm, rois, 6, monkeypatch, "mixed fused / separate")


@pytest.mark.parametrize("K", [0, 2, 4, 5, 6])
def test_fused_random_shapes(dpm, monkeypatch, K):
    """60 seeded random ROIs per order: dims 1-130 (rows of 1-8, 9-32, 33-64 and wider
    voxels, single slices, ragged blocks), both voxel types, uniform random or sphere
    contents; some blocks fit the fused kernel and some (large ones) do not."""
    rng = np.random.default_rng(100 + K)
    rois = []
    for i in range(60):
        dims = tuple(int(v) for v in rng.integers(1, 131, size=3))
        if rng.random() < 0.3:
            dims = (dims[0], dims[1], int(rng.integers(1, 9)))  # very short rows
        dt = np.uint8 if rng.random() < 0.7 else np.uint16
        if dt == np.uint8 and min(dims) >= 8 and rng.random() < 0.5:
            rois.append(synth.sphere_mask(dims, rng))
        else:
            rois.append(synth.uniform_volume(dims, dt, seed=int(rng.integers(1 << 30))))
    check(dpm, rois, K, monkeypatch, f"random shapes K={K}")
