"""GPU parity of the paper's own route (five images of Section 3.1, 1D integrals of
Section 5, eqs. 10-16) and of the 1D-integral route for the default images, through the
C ABI, against the oracle: images bit for bit, moments of orders <= 4 bit for bit as
int128 and every FP64 the nearest double."""
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
    m.lib()
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    ((29, 7, 13), np.uint8, 4),      # ragged everything, one tile, generic loads
    ((16, 9, 64), np.uint16, 3),     # aligned rows: fast loads, four images
    ((70, 20, 600), np.uint16, 4),   # two x-tiles, two z-blocks, three y-blocks
    ((130, 17, 1030), np.uint8, 4),  # three x-tiles, generic loads, ragged z-block
    ((64, 64, 64), np.uint8, 3),     # the 64^3 uint8 order-3 configuration
    ((5, 3, 8), np.uint16, 2),       # three images
    ((1, 1, 1), np.uint8, 4),
    ((3, 1, 200), np.uint16, 1),
    ((9, 40, 1), np.uint8, 0),
]


@pytest.mark.parametrize("shape,dt,K", CASES)
def test_paper_images_bit_exact(dpm, shape, dt, K):
    say("paper images", shape, dt.__name__, K)
    V = synth.uniform_volume(shape, dt, seed=sum(shape) + K)
    got = dpm.paper_images(to_dev(V), K)
    ref = oracle.paper_images(V, K)
    assert len(got) == len(ref)
    for e, (g, r) in enumerate(zip(got, ref)):
        g = g.cpu().numpy().astype(np.int64)
        assert g.shape == r.shape, (e, g.shape, r.shape)
        assert np.array_equal(g, r), f"image {e} differs"


@pytest.mark.parametrize("shape,dt,K", CASES)
def test_paper_moments_exact(dpm, shape, dt, K):
    say("paper moments", shape, dt.__name__, K)
    V = synth.uniform_volume(shape, dt, seed=3 * sum(shape) + K)
    assert_moments_equal(dpm.moments_paper(to_dev(V), K), oracle.moments_exact(V, K), K, f"paper {shape} K={K}")


@pytest.mark.parametrize("shape,dt,K", CASES)
def test_drt_route_moments_exact(dpm, shape, dt, K):
    say("drt moments", shape, dt.__name__, K)
    V = synth.uniform_volume(shape, dt, seed=5 * sum(shape) + K)
    assert_moments_equal(dpm.moments_drt(to_dev(V), K), oracle.moments_exact(V, K), K, f"drt {shape} K={K}")


def test_paper_and_drt_on_saturated_and_impulse_volumes(dpm):
    V = np.full((40, 24, 72), 65535, dtype=np.uint16)
    ref = oracle.moments_exact(V, 4)
    assert_moments_equal(dpm.moments_paper(to_dev(V), 4), ref, 4, "paper saturated")
    assert_moments_equal(dpm.moments_drt(to_dev(V), 4), ref, 4, "drt saturated")
    for corner in [(0, 0, 0), (39, 23, 71), (0, 23, 71), (39, 0, 0)]:
        V = np.zeros((40, 24, 72), dtype=np.uint16)
        V[corner] = 65535
        ref = oracle.moments_exact(V, 4)
        assert_moments_equal(dpm.moments_paper(to_dev(V), 4), ref, 4, f"paper impulse {corner}")
        assert_moments_equal(dpm.moments_drt(to_dev(V), 4), ref, 4, f"drt impulse {corner}")


def test_paper_route_unaligned_volume(dpm):
    """A volume starting 2 bytes into its buffer: the generic loads."""
    import torch
    V = synth.uniform_volume((12, 5, 64), np.uint16, seed=8)
    src = to_dev(V).reshape(-1)
    flat = torch.empty(1 + src.numel(), dtype=src.dtype, device=src.device)
    flat[1:] = src
    vol = flat[1:].view(V.shape)
    assert_moments_equal(dpm.moments_paper(vol, 4), oracle.moments_exact(V, 4), 4, "paper unaligned")


def test_paper_and_drt_at_bench_sizes(dpm):
    """256^3 MRI-like and 512^3 CT-like uint16 volumes at order 4 against the exact
    direct sums."""
    for shape, gen in [((256, 256, 256), synth.mri_phantom), ((512, 512, 512), synth.ct_phantom)]:
        say("paper/drt", shape)
        V = gen(shape, seed=0)
        ref = onative.moments_hoisted(V, 4)
        vol = to_dev(V)
        assert_moments_equal(dpm.moments_paper(vol, 4), ref, 4, f"paper {shape}")
        assert_moments_equal(dpm.moments_drt(vol, 4), ref, 4, f"drt {shape}")
        assert_moments_equal(dpm.moments(vol, 4), ref, 4, f"default {shape}")


def test_paper_route_errors(dpm):
    import torch
    lib = dpm.lib()
    vol = torch.zeros((4, 4, 8), dtype=torch.uint8, device="cuda:0")
    assert lib.dpm_paper_workspace_bytes(dpm._lib.Dims(8, 4, 4), 1, 5) == 0
    assert lib.dpm_drt_workspace_bytes(dpm._lib.Dims(8, 4, 4), 1, 5) == 0
    out = dpm._lib.Out(None, None)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    args = (ctypes.c_void_p(vol.data_ptr()), dpm._lib.Dims(8, 4, 4), 1)
    assert lib.dpm_moments_paper(*args, 5, ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()), ws.numel(), None) == -5
    assert lib.dpm_moments_drt(*args, 5, ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()), ws.numel(), None) == -5
    assert lib.dpm_moments_paper(*args, 4, ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()), 16, None) == -3
    assert lib.dpm_moments_drt(*args, 4, ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()), 16, None) == -3
    # an image too wide for the 1D-integral coordinates
    assert lib.dpm_paper_workspace_bytes(dpm._lib.Dims(40000, 1, 1), 1, 4) == 0
    assert lib.dpm_moments_paper(ctypes.c_void_p(vol.data_ptr()), dpm._lib.Dims(40000, 1, 1), 1, 4, ctypes.byref(out),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), None) == -2
