"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Projection images (step 1, Section 3.1) must equal the oracle's line sums bit for bit;
moments of orders <= 4 must equal the exact integers of eq. (2) bit for bit; every
order's FP64 value must be the double nearest to the exact integer (so the relative
error is <= 2^-53, inside the 1e-12 budget for orders 5-16).
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import oracle.native as onative
import synth
from gpu_util import assert_moments_equal, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2012_08099_amd as m
    m.lib()  # raises if the HIP library is missing
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


IMAGE_CASES = [
    ((16, 8, 64), np.uint16, 6),     # fast path, 8-lane sub-rows
    ((32, 5, 512), np.uint16, 6),    # fast path, full 64-lane rows
    ((29, 7, 13), np.uint8, 6),      # generic: ragged x and z
    ((20, 3, 1100), np.uint16, 4),   # generic: 3 column tiles, ragged
    ((16, 4, 1024), np.uint8, 3),    # fast: 2 column tiles
    ((24, 3, 40), np.uint16, 16),    # all three direction groups, generic
    ((32, 2, 128), np.uint16, 16),   # all three direction groups, fast
    ((1, 1, 1), np.uint8, 2),
    ((5, 2, 8), np.uint8, 0),
]


@pytest.mark.parametrize("shape,dt,K", IMAGE_CASES)
def test_projection_images_bit_exact(dpm, shape, dt, K):
    say("images", shape, dt.__name__, K)
    V = synth.uniform_volume(shape, dt, seed=hash((shape, K)) % 1000)
    imgs = dpm.project_images(to_dev(V), K)
    for d in range(K + 1):
        a, b = dpm.direction(d)
        ref = oracle.projection_image(V, a, b)
        got = imgs[d].cpu().numpy().astype(np.int64)
        assert got.shape == ref.shape, (d, got.shape, ref.shape)
        assert np.array_equal(got, ref), f"image {d} ({a},{b}) differs"


MOMENT_CASES = [
    ((64, 64, 64), np.uint8, 3),     # the 64^3 uint8 order-3 configuration
    ((29, 7, 13), np.uint8, 6),
    ((33, 9, 70), np.uint16, 6),
    ((48, 16, 64), np.uint16, 6),
    ((16, 16, 16), np.uint16, 16),
    ((40, 12, 24), np.uint8, 16),
    ((1, 1, 1), np.uint16, 4),
    ((1, 50, 1), np.uint8, 5),
    ((17, 1, 3), np.uint16, 7),
    ((3, 2, 600), np.uint16, 5),
    ((32, 8, 128), np.uint16, 12),
    ((16, 8, 64), np.uint16, 0),
    ((16, 8, 64), np.uint8, 1),
    ((32, 3, 512), np.uint16, 6),
    ((96, 2, 1024), np.uint16, 5),
    # size limits of the matrix-core power sums: row values reach 2^28 (L = 4100 at
    # uint16), coordinates a reach 8192 (L = 4096): both take the VALU power sums
    ((16, 2, 4100), np.uint16, 6),
    ((16, 2, 4096), np.uint16, 6),
    ((4100, 3, 2), np.uint16, 5),     # N = 4100: many z-splits per slice
    # orders 7-16 on whole-row loads: all direction groups in one launch
    ((48, 9, 64), np.uint8, 7),
    ((32, 5, 128), np.uint16, 11),
    ((64, 3, 256), np.uint16, 13),
    ((48, 7, 512), np.uint8, 16),
]


@pytest.mark.parametrize("shape,dt,K", MOMENT_CASES)
def test_moments_random(dpm, shape, dt, K):
    say("moments", shape, dt.__name__, K)
    V = synth.uniform_volume(shape, dt, seed=(shape[0] * 7 + K) % 997)
    res = dpm.moments(to_dev(V), K)
    assert_moments_equal(res, oracle.moments_exact(V, K), K, f"{shape} K={K}")


PATH_OVERRIDES = [
    ({"DPM_NO_MFMA": "1"}, (33, 9, 70), np.uint16, 6),      # VALU power sums
    ({"DPM_NO_MFMA": "1"}, (20, 6, 24), np.uint8, 16),      # VALU, every direction group
    ({"DPM_ZSPLITS": "3"}, (48, 10, 64), np.uint16, 7),     # z-split work items
    ({"DPM_ZSPLITS": "4", "DPM_NO_MFMA": "1"}, (70, 5, 64), np.uint8, 5),
    ({"DPM_FORCE_GENERIC": "1"}, (32, 8, 128), np.uint16, 6),
    ({"DPM_GROUP_LAUNCHES": "1"}, (32, 8, 128), np.uint16, 16),  # one launch per direction group
    ({"DPM_SLICE_WAVES": "4"}, (32, 5, 512), np.uint16, 6),      # 4 waves per projection workgroup
    ({"DPM_SLICE_WAVES": "4"}, (48, 6, 256), np.uint8, 4),
    ({"DPM_SLICE_WAVES": "4", "DPM_ZSPLITS": "2"}, (64, 3, 128), np.uint16, 5),
    ({"DPM_SLICE_WAVES": "8", "DPM_ZSPLITS": "2"}, (64, 3, 128), np.uint16, 5),
    ({"DPM_GROUP_LAUNCHES": "1"}, (48, 5, 64), np.uint8, 9),
    # chained-window projection (opt-in): rows of whole 64-lane tiles, 32-row units
    ({"DPM_CHAIN": "1"}, (32, 3, 512), np.uint16, 6),
    ({"DPM_CHAIN": "1"}, (96, 2, 1024), np.uint16, 5),
    ({"DPM_CHAIN": "1"}, (64, 5, 512), np.uint16, 3),
    ({"DPM_CHAIN": "1"}, (32, 4, 512), np.uint16, 1),
    ({"DPM_CHAIN": "1"}, (64, 16, 512), np.uint16, 0),
]


@pytest.mark.parametrize("env,shape,dt,K", PATH_OVERRIDES)
def test_moments_forced_paths(dpm, monkeypatch, env, shape, dt, K):
    """The planner's alternative paths, forced through its environment overrides."""
    say("forced", env, shape, dt.__name__, K)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    V = synth.uniform_volume(shape, dt, seed=K * 31 + shape[0])
    res = dpm.moments(to_dev(V), K)
    assert_moments_equal(res, oracle.moments_exact(V, K), K, f"{env} {shape} K={K}")


@pytest.mark.parametrize("dt", [np.uint8, np.uint16])
@pytest.mark.parametrize("shift", [1, 2, 3])
def test_unaligned_volume_at_buffer_end(dpm, dt, shift):
    """A volume whose first voxel is not 4-byte aligned and whose last voxel is the last
    element of its buffer: the generic lane loads read only aligned dwords that hold
    voxels of the row and shift them into place."""
    import torch
    say("unaligned", dt.__name__, shift)
    V = synth.uniform_volume((11, 5, 37), dt, seed=shift)
    src = to_dev(V).reshape(-1)
    flat = torch.empty(shift + src.numel(), dtype=src.dtype, device=src.device)
    flat[shift:] = src
    vol = flat[shift:].view(V.shape)
    assert vol.data_ptr() % 4 != 0 or dt is np.uint16
    res = dpm.moments(vol, 6)
    assert_moments_equal(res, oracle.moments_exact(V, 6), 6, f"unaligned {dt.__name__} +{shift}")


def test_all_zero_volume(dpm):
    V = np.zeros((48, 16, 64), dtype=np.uint16)
    res = dpm.moments(to_dev(V), 6)
    assert all(v == 0 for v in res.exact) and not res.fp64.any()


def test_saturated_volume(dpm):
    V = np.full((64, 32, 128), 65535, dtype=np.uint16)
    res = dpm.moments(to_dev(V), 8)
    assert_moments_equal(res, oracle.moments_exact(V, 8), 8, "saturated")


@pytest.mark.parametrize("corner", [(0, 0, 0), (31, 15, 63), (0, 15, 0), (31, 0, 63), (7, 3, 40)])
def test_impulse(dpm, corner):
    V = np.zeros((32, 16, 64), dtype=np.uint16)
    V[corner] = 65535
    res = dpm.moments(to_dev(V), 10)
    assert_moments_equal(res, oracle.moments_exact(V, 10), 10, f"impulse {corner}")


def test_mri_phantom_256_order6(dpm):
    say("mri 256^3 K=6")
    V = synth.mri_phantom((256, 256, 256), seed=0)
    res = dpm.moments(to_dev(V), 6)
    assert_moments_equal(res, onative.moments_hoisted(V, 6), 6, "mri256")


def test_ct_512_order6_full(dpm, monkeypatch):
    say("ct 512^3 K=6")
    V = synth.ct_phantom((512, 512, 512), seed=0)
    ref = onative.moments_hoisted(V, 6)
    res = dpm.moments(to_dev(V), 6)
    assert_moments_equal(res, ref, 6, "ct512")
    monkeypatch.setenv("DPM_CHAIN", "1")
    res = dpm.moments(to_dev(V), 6)
    assert_moments_equal(res, ref, 6, "ct512 chained windows")


def test_ct_128_order16_full(dpm):
    say("ct 128^3 K=16")
    V = synth.ct_phantom((128, 128, 128), seed=1)
    res = dpm.moments(to_dev(V), 16)
    assert_moments_equal(res, oracle.moments_exact(V, 16), 16, "ct128 K=16")


def test_deterministic(dpm):
    V = synth.mri_phantom((64, 64, 64), seed=3)
    a = dpm.moments(to_dev(V), 9)
    b = dpm.moments(to_dev(V), 9)
    assert a.exact == b.exact and np.array_equal(a.fp64.view(np.uint64), b.fp64.view(np.uint64))


def test_async_on_side_stream(dpm):
    import torch
    V = synth.uniform_volume((48, 24, 96), np.uint16, seed=5)
    vol = to_dev(V)
    K = 6
    nm, nm4 = dpm.num_moments(K), dpm.num_moments(4)
    ex = torch.zeros((nm4, 2), dtype=torch.int64, device="cuda:0")
    fp = torch.zeros(nm, dtype=torch.float64, device="cuda:0")
    ws = torch.empty(dpm.workspace_bytes(vol.shape, 2, K), dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    dpm.moments_async(vol, K, ex, fp, ws, stream=s)
    s.synchronize()
    got = dpm.Moments(K, dpm._exact_from_tensor(ex), fp.cpu().numpy())
    assert_moments_equal(got, oracle.moments_exact(V, K), K, "async")


def test_invalid_arguments(dpm):
    import torch
    lib = dpm.lib()
    vol = torch.zeros((4, 4, 8), dtype=torch.uint8, device="cuda:0")
    with pytest.raises((ValueError, dpm.DpmError)):
        dpm.moments(vol, 17)
    out = dpm._lib.Out(None, None)
    bad = dpm._lib.Dims(0, 4, 4)
    assert lib.dpm_moments_async(ctypes.c_void_p(vol.data_ptr()), bad, 1, 3, ctypes.byref(out), None, 0, None) == -1
    good = dpm._lib.Dims(8, 4, 4)
    assert lib.dpm_moments_async(ctypes.c_void_p(vol.data_ptr()), good, 9, 3, ctypes.byref(out), None, 0, None) == -1
    # workspace smaller than required
    ws = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    ex = torch.zeros((20, 2), dtype=torch.int64, device="cuda:0")
    out = dpm._lib.Out(ex.data_ptr(), None)
    rc = lib.dpm_moments_async(ctypes.c_void_p(vol.data_ptr()), good, 1, 3, ctypes.byref(out),
                               ctypes.c_void_p(ws.data_ptr()), 16, None)
    assert rc == -3


@pytest.mark.parametrize("n,seed", [(40, 0), (1000, 1)])
def test_batched_matches_single_and_oracle(dpm, n, seed):
    import torch
    say("batched", n)
    rois = synth.roi_batch(n, seed=seed)
    K = 4
    packed, desc = dpm.pack_rois(rois, "cuda:0")
    nm = dpm.num_moments(K)
    ex = torch.zeros((n * nm, 2), dtype=torch.int64, device="cuda:0")
    fp = torch.zeros(n * nm, dtype=torch.float64, device="cuda:0")
    ws = torch.empty(dpm.batched_workspace_bytes(desc, K), dtype=torch.uint8, device="cuda:0")
    dpm.moments_batched(packed, desc, K, ex, fp, ws)
    torch.cuda.synchronize()
    exact = dpm._exact_from_tensor(ex)
    fpn = fp.cpu().numpy()
    for i, V in enumerate(rois):
        ref = onative.moments_hoisted(V, K)
        got = dpm.Moments(K, exact[i * nm:(i + 1) * nm], fpn[i * nm:(i + 1) * nm])
        assert_moments_equal(got, ref, K, f"roi {i} {V.shape}")
        if i < 25:
            single = dpm.moments(to_dev(V), K)
            assert single.exact == got.exact


def test_batched_graph_replays(dpm, monkeypatch):
    """A batched call repeated with the same descriptors and buffers is captured into a
    graph on its second sighting and replayed from then on.  Every call -- first
    (eager), second (capture + launch), later replays -- matches the oracle, with new
    voxel contents written into the packed buffer between calls and other library work
    and host synchronisations in between."""
    import torch
    monkeypatch.delenv("DPM_NO_GRAPH", raising=False)
    say("batched graph replays")
    dpm.release()
    K = 4
    n = 48
    rois = synth.roi_batch(n, seed=5)
    packed, desc = dpm.pack_rois(rois, "cuda:0")
    nm = dpm.num_moments(K)
    ex = torch.zeros((n * nm, 2), dtype=torch.int64, device="cuda:0")
    fp = torch.zeros(n * nm, dtype=torch.float64, device="cuda:0")
    ws = torch.empty(dpm.batched_workspace_bytes(desc, K), dtype=torch.uint8, device="cuda:0")
    other = synth.uniform_volume((20, 9, 33), np.uint16, seed=3)
    for call in range(5):
        # new contents in place (same shapes, same buffer)
        vols = [synth.uniform_volume(V.shape, V.dtype, seed=100 * call + i) if call % 2 else
                (V if call == 0 else np.ascontiguousarray(V[::-1])) for i, V in enumerate(rois)]
        newp, _ = dpm.pack_rois(vols, "cuda:0")
        packed.copy_(newp)
        ex.zero_()
        fp.zero_()
        dpm.moments_batched(packed, desc, K, ex, fp, ws)
        torch.cuda.synchronize()
        assert dpm.batched_graph_count() == (0 if call == 0 else 1), call
        exact = dpm._exact_from_tensor(ex)
        fpn = fp.cpu().numpy()
        for i, V in enumerate(vols):
            got = dpm.Moments(K, exact[i * nm:(i + 1) * nm], fpn[i * nm:(i + 1) * nm])
            assert_moments_equal(got, onative.moments_hoisted(V, K), K, f"call {call} roi {i} {V.shape}")
        # eager work of the library between replays
        res = dpm.moments(to_dev(other), 3)
        assert_moments_equal(res, oracle.moments_exact(other, 3), 3, "eager call between replays")
    # a different output buffer is a different call: no replay of the cached graph
    fp2 = torch.zeros_like(fp)
    dpm.moments_batched(packed, desc, K, ex, fp2, ws)
    torch.cuda.synchronize()
    assert torch.equal(fp2, fp)
    assert dpm.batched_graph_count() == 1
    dpm.release()
    assert dpm.batched_graph_count() == 0


def test_large_planes_order3(dpm):
    """A 3000 x 2 x 3000 uint16 volume (wide rows and many z rows at once)."""
    say("3000x2x3000 u16 K=3")
    V = synth.uniform_volume((3000, 2, 3000), np.uint16, seed=9)
    res = dpm.moments(to_dev(V), 3)
    assert_moments_equal(res, onative.moments_hoisted(V, 3), 3, "3000x2x3000")


def test_batched_extreme_roi_shapes(dpm):
    """Batched ROIs at the batched path's size limit (4096 along one axis), single voxels,
    and both dtypes in one batch: each equals its single call and the oracle."""
    import torch
    say("batched extreme shapes")
    shapes = [((1, 1, 1), np.uint8), ((3, 2, 4096), np.uint16), ((2048, 1, 1), np.uint8),
              ((1, 4096, 1), np.uint16), ((2, 3, 4096), np.uint8), ((5, 7, 9), np.uint16),
              ((64, 1, 64), np.uint8)]
    rois = [synth.uniform_volume(sh, dt, seed=i) for i, (sh, dt) in enumerate(shapes)]
    K = 6
    packed, desc = dpm.pack_rois(rois, "cuda:0")
    n, nm, nm4 = len(rois), dpm.num_moments(K), dpm.num_moments(4)
    ex = torch.zeros((n * nm4, 2), dtype=torch.int64, device="cuda:0")
    fp = torch.zeros(n * nm, dtype=torch.float64, device="cuda:0")
    ws = torch.empty(dpm.batched_workspace_bytes(desc, K), dtype=torch.uint8, device="cuda:0")
    dpm.moments_batched(packed, desc, K, ex, fp, ws)
    torch.cuda.synchronize()
    exact = dpm._exact_from_tensor(ex)
    fpn = fp.cpu().numpy()
    for i, V in enumerate(rois):
        got = dpm.Moments(K, exact[i * nm4:(i + 1) * nm4], fpn[i * nm:(i + 1) * nm])
        assert_moments_equal(got, oracle.moments_exact(V, K), K, f"roi {i} {V.shape}")
        single = dpm.moments(to_dev(V), K)
        assert single.exact == got.exact


def test_batched_refuses_rows_beyond_lds(dpm):
    """A 4096-deep column at order 6 needs more LDS for its full-z image rows than one
    workgroup has: the batched planner refuses it (workspace size 0, DPM_ERANGE), and the
    single-volume path, which splits z, computes it."""
    import ctypes
    import torch
    from paper_2012_08099_amd import _lib
    V = synth.uniform_volume((4096, 1, 1), np.uint8, seed=4)
    packed, desc = dpm.pack_rois([V], "cuda:0")
    assert dpm.batched_workspace_bytes(desc, 6) == 0
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    out = _lib.Out(None, torch.zeros(84, dtype=torch.float64, device="cuda:0").data_ptr())
    rc = dpm.lib().dpm_moments_batched(ctypes.c_void_p(packed.data_ptr()), desc, 1, 6, ctypes.byref(out),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert rc == -2
    assert_moments_equal(dpm.moments(to_dev(V), 6), oracle.moments_exact(V, 6), 6, "4096 column")


def test_moments_async_replayed_from_a_captured_graph(dpm):
    """A caller may capture dpm_moments_async (caller-owned workspace and outputs, its
    tables built by an earlier eager call) into a HIP graph: every replay, with eager
    library work and synchronisations between replays, equals the eager result, and new
    voxels written in place give the new volume's moments."""
    import torch
    say("graph capture of dpm_moments_async")
    K = 6
    V = synth.ct_phantom((48, 40, 128), seed=4)
    W = synth.mri_phantom((32, 24, 64), seed=6)
    vol = to_dev(V)
    nm, nm4 = dpm.num_moments(K), dpm.num_moments(4)
    ex = torch.zeros((nm4, 2), dtype=torch.int64, device="cuda:0")
    fp = torch.zeros(nm, dtype=torch.float64, device="cuda:0")
    ws = torch.empty(dpm.workspace_bytes(V.shape, 2, K), dtype=torch.uint8, device="cuda:0")
    dpm.moments_async(vol, K, ex, fp, ws)  # eager: builds the device tables
    torch.cuda.synchronize()
    ref_ex, ref_fp = ex.clone(), fp.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        dpm.moments_async(vol, K, ex, fp, ws, stream=torch.cuda.current_stream())
    for i in range(4):
        ex.zero_()
        fp.zero_()
        torch.cuda.synchronize()
        other = dpm.moments(to_dev(W), 3)  # eager library work between replays
        assert_moments_equal(other, oracle.moments_exact(W, 3), 3, f"eager between replays {i}")
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ex, ref_ex) and torch.equal(fp.view(torch.int64), ref_fp.view(torch.int64)), i
    V2 = synth.uniform_volume(V.shape, np.uint16, seed=8, hi=4095)
    vol.copy_(to_dev(V2))
    g.replay()
    torch.cuda.synchronize()
    got = dpm.Moments(K, dpm._exact_from_tensor(ex), fp.cpu().numpy())
    assert_moments_equal(got, oracle.moments_exact(V2, K), K, "replay on new voxels")
