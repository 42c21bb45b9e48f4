"""Pins of the oracle's paper-route pieces (CPU): the five images of Section 3.1, the 1D
integrals of Section 5 and their combination into 2D moments, and eqs. 10-16 -- each
against what mathematics fixes (mass, marginals, impulses, the direct 2D moment sum, the
definition of eq. 2), not against a retyped copy of itself."""
import numpy as np
import pytest

import oracle
import synth


def test_paper_images_impulse_positions():
    """One voxel v at (x0, y0, z0) lands on exactly one pixel of each image, at the index
    maps of eqs. 5-9 (X-Z at column x0 - z0 + N - 1)."""
    N, M, L = 5, 4, 6
    for (z0, y0, x0) in [(0, 0, 0), (4, 3, 5), (0, 3, 5), (4, 0, 0), (2, 1, 3)]:
        V = np.zeros((N, M, L), dtype=np.uint16)
        V[z0, y0, x0] = 65535
        XY, YZ, ZX, XPZ, XMZ = oracle.paper_images(V, 4)
        for img, (j, i) in [(XY, (y0, x0)), (YZ, (z0, y0)), (ZX, (x0, z0)), (XPZ, (y0, x0 + z0)),
                            (XMZ, (y0, x0 - z0 + N - 1))]:
            nz = np.argwhere(img)
            assert nz.tolist() == [[j, i]] and img[j, i] == 65535


@pytest.mark.parametrize("seed", range(3))
def test_paper_images_marginals(seed):
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in rng.integers(1, 9, size=3))
    V = rng.integers(0, 256, size=shape).astype(np.uint8)
    XY, YZ, ZX, XPZ, XMZ = oracle.paper_images(V, 4)
    W = V.astype(np.int64)
    mass = int(W.sum())
    assert all(int(im.sum()) == mass for im in (XY, YZ, ZX, XPZ, XMZ))
    ym, xm, zm = W.sum(axis=(0, 2)), W.sum(axis=(0, 1)), W.sum(axis=(1, 2))
    assert np.array_equal(XY.sum(axis=1), ym) and np.array_equal(YZ.sum(axis=0), ym)
    assert np.array_equal(XPZ.sum(axis=1), ym) and np.array_equal(XMZ.sum(axis=1), ym)
    assert np.array_equal(XY.sum(axis=0), xm) and np.array_equal(ZX.sum(axis=1), xm)
    assert np.array_equal(YZ.sum(axis=1), zm) and np.array_equal(ZX.sum(axis=0), zm)
    # the diagonal images are the (1, +-1) projections of eq. 4
    assert np.array_equal(XPZ, oracle.projection_image(V, 1, 1))
    assert np.array_equal(XMZ, oracle.projection_image(V, 1, -1))
    assert len(oracle.paper_images(V, 3)) == 4 and len(oracle.paper_images(V, 2)) == 3


def test_drt_integrals_impulse_and_axis_sums():
    img = np.zeros((5, 7), dtype=np.int64)
    img[3, 4] = 9  # j = 3, i = 4
    for g, (tmin, P) in enumerate(oracle.drt_integrals(img, 5)):
        a, b = oracle.DRT_DIRS[g]
        nz = [k + tmin for k, v in enumerate(P) if v]
        assert nz == [a * 4 + b * 3] and sum(P) == 9
    img = np.random.default_rng(1).integers(0, 100, size=(6, 9))
    ints = oracle.drt_integrals(img, 5)
    assert ints[0] == (0, img.sum(axis=0).tolist())          # onto the x axis: column sums
    assert ints[1] == (0, img.sum(axis=1).tolist())          # onto the y axis: row sums
    assert ints[3][0] == -(img.shape[0] - 1)                 # i - j runs negative
    assert all(sum(P) == int(img.sum()) for _, P in ints)


@pytest.mark.parametrize("K", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("origin", [0, 3])
def test_moments_2d_from_integrals_equal_the_direct_sum(K, origin):
    """The 1D-integral route gives the 2D moments of eq. 1 exactly (also about a shifted
    column origin)."""
    img = np.random.default_rng(K * 10 + origin).integers(0, 1000, size=(7, 11))
    got = oracle.moments_2d_from_integrals(oracle.drt_integrals(img, K + 1), K, origin=origin)
    assert got == oracle.image_moments_2d(img, K, origin=origin)


@pytest.mark.parametrize("seed", range(4))
def test_paper_moments_equal_the_definition(seed):
    rng = np.random.default_rng(50 + seed)
    shape = tuple(int(s) for s in rng.integers(1, 8, size=3))
    V = rng.integers(0, 65536, size=shape).astype(np.uint16)
    for K in range(5):
        assert oracle.paper_moments(V, K) == oracle.moments_exact(V, K), (shape, K)
    tiny = synth.uniform_volume((2, 3, 2), np.uint8, seed=seed)
    assert oracle.paper_moments(tiny, 4) == oracle.moments_bruteforce(tiny, 4)
