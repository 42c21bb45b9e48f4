"""GPU parity of moments from supplied projection images (dpm_moments_from_images, the
tomography use noted in Section 3.2): images computed by the oracle on the CPU (the line
sums of eq. 4, with the offset of the beta < 0 images) give the oracle's moments bit for
bit, as do the library's own projection images; out-of-range entries are refused."""
import sys

import numpy as np
import pytest

import oracle
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


def oracle_images(dpm, V, K):
    import torch
    parts = []
    for d in range(K + 1):
        a, b = dpm.direction(d)
        parts.append(oracle.projection_image(V, a, b).astype(np.int32).reshape(-1))
    return torch.from_numpy(np.concatenate(parts)).to("cuda:0")


@pytest.mark.parametrize("shape,dt,K", [((9, 5, 13), np.uint8, 4), ((20, 7, 24), np.uint16, 6),
                                        ((16, 4, 64), np.uint16, 10), ((6, 3, 11), np.uint8, 16),
                                        ((1, 1, 1), np.uint16, 3)])
def test_moments_from_oracle_images(dpm, shape, dt, K):
    say("from images", shape, dt.__name__, K)
    V = synth.uniform_volume(shape, dt, seed=K)
    code = 1 if dt == np.uint8 else 2
    res = dpm.moments_from_images(oracle_images(dpm, V, K), V.shape, code, K)
    assert_moments_equal(res, oracle.moments_exact(V, K), K, f"{shape} K={K}")


def test_moments_from_own_images_equal_volume_path(dpm):
    import torch
    V = synth.mri_phantom((48, 40, 64), seed=2)
    K = 6
    imgs = dpm.project_images(to_dev(V), K)
    flat = torch.cat([im.reshape(-1) for im in imgs]).contiguous()
    a = dpm.moments_from_images(flat, V.shape, 2, K)
    b = dpm.moments(to_dev(V), K)
    assert a.exact == b.exact
    assert np.array_equal(a.fp64.view(np.uint64), b.fp64.view(np.uint64))


def test_out_of_range_images_refused(dpm):
    V = synth.uniform_volume((8, 4, 10), np.uint8, seed=1)
    imgs = oracle_images(dpm, V, 3)
    bad = imgs.clone()
    bad[5] = -1
    with pytest.raises(dpm.DpmError) as e:
        dpm.moments_from_images(bad, V.shape, 1, 3)
    assert e.value.status == -2
    bad = imgs.clone()
    bad[7] = 255 * 10 + 1  # above vmax * max(L, N)
    with pytest.raises(dpm.DpmError):
        dpm.moments_from_images(bad, V.shape, 1, 3)
    # the good images still work afterwards
    assert_moments_equal(dpm.moments_from_images(imgs, V.shape, 1, 3), oracle.moments_exact(V, 3), 3, "after")
