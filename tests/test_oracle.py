"""Pins for the CPU oracle against facts the paper and mathematics fix.

The paper prints no moment values for a worked example (the MRI example of Section 4
reports timings only), so the oracle is pinned by: brute force on tiny volumes,
closed forms (impulses; uniform boxes via Faulhaber sums), invariants (mass, axis
permutation, reflection, translation of central moments, slab additivity), the
projection definitions of Section 3.1 and the moment identities eqs. (10)-(16) of
Section 3.2 -- with the left-hand sides of eqs. (15)/(16) exchanged, which is the
only reading under which the binomial expansion of (x +- z)^3 y holds.
"""
import itertools
from fractions import Fraction
from math import comb

import numpy as np
import pytest
import sympy

import oracle
import oracle.native as onative
import synth
from oracle import moment_list, moments_bruteforce, moments_exact, moment_single

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def as_dict(vals, K):
    return dict(zip(moment_list(K), vals))


# ----------------------------------------------------------------- graded order
def test_graded_order_and_index():
    ml = moment_list(3)
    assert ml[:10] == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0),
                       (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]
    for K in (0, 4, 16):
        assert len(moment_list(K)) == comb(K + 3, 3)
    assert len(moment_list(16)) == 969
    for i, t in enumerate(moment_list(5)):
        assert oracle.moment_index(*t) == i


# ----------------------------------------------------------------- brute force
@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 3, 2), (4, 1, 3), (2, 5, 1), (5, 4, 6), (7, 3, 8)])
@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_exact_equals_bruteforce(shape, dtype):
    V = synth.uniform_volume(shape, dtype, seed=sum(shape))
    for K in (0, 3, 5):
        assert moments_exact(V, K) == moments_bruteforce(V, K)


def test_all_binary_2x2x2_volumes():
    for bits in range(256):
        V = np.array([(bits >> i) & 1 for i in range(8)], dtype=np.uint8).reshape(2, 2, 2)
        bf = moments_bruteforce(V, 3)
        assert moments_exact(V, 3) == bf
        assert onative.moments_hoisted(V, 3) == bf
        assert onative.moments_direct(V, 3) == bf


# ----------------------------------------------------------------- closed forms
@pytest.mark.parametrize("v", [1, 200, 65535])
def test_impulse(v):
    N, M, L = 6, 5, 7
    for (z0, y0, x0) in [(0, 0, 0), (N - 1, M - 1, L - 1), (0, M - 1, 3), (N - 1, 0, 0), (2, 3, 4)]:
        V = np.zeros((N, M, L), dtype=np.uint16)
        V[z0, y0, x0] = v
        got = as_dict(moments_exact(V, 6), 6)
        for (p, q, r), m in got.items():
            assert m == v * x0**p * y0**q * z0**r, ((p, q, r), (z0, y0, x0))
        assert onative.moments_hoisted(V, 6) == list(got.values())


def faulhaber(p, n):
    """sum_{x=0}^{n-1} x^p by Faulhaber's formula with Bernoulli numbers (B_1 = -1/2)."""
    if p == 0:
        return n
    s = Fraction(0)
    for j in range(p + 1):
        b = Fraction(str(sympy.bernoulli(j)))
        if j == 1:
            b = Fraction(-1, 2)
        s += comb(p + 1, j) * b * Fraction(n) ** (p + 1 - j)
    s /= p + 1
    assert s.denominator == 1
    return int(s)


def test_faulhaber_helper_small():
    # independent spot values: 0+1+4+9 = 14, 0+1+8+27+64 = 100
    assert faulhaber(2, 4) == 14 and faulhaber(3, 5) == 100 and faulhaber(0, 7) == 7


@pytest.mark.parametrize("c", [1, 4095])
def test_uniform_box_closed_form(c):
    N, M, L = 5, 7, 6
    V = np.full((N, M, L), c, dtype=np.uint16)
    got = as_dict(moments_exact(V, 8), 8)
    for (p, q, r), m in got.items():
        assert m == c * faulhaber(p, L) * faulhaber(q, M) * faulhaber(r, N)


def test_sub_box_closed_form():
    N, M, L = 9, 8, 10
    (z0, z1), (y0, y1), (x0, x1) = (2, 7), (1, 5), (3, 10)
    V = np.zeros((N, M, L), dtype=np.uint8)
    V[z0:z1, y0:y1, x0:x1] = 7
    got = as_dict(moments_exact(V, 7), 7)
    for (p, q, r), m in got.items():
        ex = 7 * (faulhaber(p, x1) - faulhaber(p, x0)) * (faulhaber(q, y1) - faulhaber(q, y0)) \
            * (faulhaber(r, z1) - faulhaber(r, z0))
        assert m == ex


def test_box_order16_large():
    # 512^3 box at order 16 exercises the limb-split summation at full size on x.
    N, M, L = 3, 4, 512
    V = np.full((N, M, L), 65535, dtype=np.uint16)
    got = as_dict(moments_exact(V, 16), 16)
    for (p, q, r), m in list(got.items())[::7]:
        assert m == 65535 * faulhaber(p, L) * faulhaber(q, M) * faulhaber(r, N)
    assert moment_single(V, 16, 0, 0) == 65535 * faulhaber(16, L) * M * N


# ----------------------------------------------------------------- invariants
def test_mass_and_linearity():
    A = synth.uniform_volume((6, 5, 7), np.uint8, seed=3)
    B = synth.uniform_volume((6, 5, 7), np.uint8, seed=4)
    ma, mb = moments_exact(A, 5), moments_exact(B, 5)
    assert ma[0] == int(A.sum(dtype=np.int64))
    mab = moments_exact(A.astype(np.uint16) + B.astype(np.uint16), 5)
    assert mab == [a + b for a, b in zip(ma, mb)]


def test_axis_permutation_permutes_indices():
    V = synth.uniform_volume((4, 5, 6), np.uint16, seed=5)
    m = as_dict(moments_exact(V, 6), 6)
    # swap x and z: V'[z'][y][x'] = V[x'][y][z'] -> M'_pqr = M_rqp
    Vxz = np.ascontiguousarray(V.transpose(2, 1, 0))
    mxz = as_dict(moments_exact(Vxz, 6), 6)
    # swap x and y: M'_pqr = M_qpr
    Vxy = np.ascontiguousarray(V.transpose(0, 2, 1))
    mxy = as_dict(moments_exact(Vxy, 6), 6)
    for (p, q, r) in moment_list(6):
        assert mxz[(p, q, r)] == m[(r, q, p)]
        assert mxy[(p, q, r)] == m[(q, p, r)]


def test_reflection_binomial():
    V = synth.uniform_volume((4, 3, 7), np.uint8, seed=6)
    L = V.shape[2]
    m = as_dict(moments_exact(V, 5), 5)
    mr = as_dict(moments_exact(np.ascontiguousarray(V[:, :, ::-1]), 5), 5)
    for (p, q, r) in moment_list(5):
        ex = sum(comb(p, t) * (L - 1) ** (p - t) * (-1) ** t * m[(t, q, r)] for t in range(p + 1))
        assert mr[(p, q, r)] == ex


def test_translation_shifts_raw_and_keeps_central():
    V = synth.uniform_volume((3, 4, 3), np.uint8, seed=7)
    a, b, c = 2, 1, 3  # offsets along x, y, z
    big = np.zeros((3 + c + 1, 4 + b + 2, 3 + a), dtype=np.uint8)
    big[c:c + 3, b:b + 4, a:a + 3] = V
    m = as_dict(moments_exact(V, 4), 4)
    mb = as_dict(moments_exact(big, 4), 4)
    for (p, q, r) in moment_list(4):
        ex = 0
        for i in range(p + 1):
            for j in range(q + 1):
                for k in range(r + 1):
                    ex += comb(p, i) * comb(q, j) * comb(r, k) * a ** (p - i) * b ** (q - j) \
                        * c ** (r - k) * m[(i, j, k)]
        assert mb[(p, q, r)] == ex
    assert oracle.central_moments(V, 4) == oracle.central_moments(big, 4)


def test_slab_additivity():
    V = synth.uniform_volume((9, 4, 5), np.uint16, seed=8)
    h = 4
    m = as_dict(moments_exact(V, 6), 6)
    lo = as_dict(moments_exact(V[:h], 6), 6)
    hi = as_dict(moments_exact(np.ascontiguousarray(V[h:]), 6), 6)
    for (p, q, r) in moment_list(6):
        shifted = sum(comb(r, t) * h ** (r - t) * hi[(p, q, t)] for t in range(r + 1))
        assert m[(p, q, r)] == lo[(p, q, r)] + shifted


# ----------------------------------------------------------------- C oracle
@pytest.mark.parametrize("dtype,shape,K", [(np.uint8, (9, 7, 11), 6), (np.uint16, (5, 8, 6), 4),
                                           (np.uint16, (1, 1, 1), 0), (np.uint8, (3, 1, 17), 3)])
def test_c_oracle_matches_python(dtype, shape, K):
    V = synth.uniform_volume(shape, dtype, seed=11)
    ex = moments_exact(V, K)
    assert onative.moments_direct(V, K) == ex
    assert onative.moments_hoisted(V, K) == ex


def test_c_oracle_refuses_overflow():
    V = np.full((64, 64, 64), 65535, dtype=np.uint16)
    with pytest.raises(OverflowError):
        onative.moments_hoisted(V, 16)


# ----------------------------------------------------------------- projections
DIRS = [(1, 0), (0, 1), (1, 1), (1, -1), (2, 1), (2, -1), (1, 2), (1, -2), (3, 1), (3, -2), (2, 3), (1, 4)]


def projection_loop(V, a, b):
    """Independent re-statement of eq. (4): visit each voxel, add it to its pixel."""
    N, M, L = V.shape
    o = -b * (N - 1) if b < 0 else 0
    W = a * (L - 1) + abs(b) * (N - 1) + 1
    img = [[0] * W for _ in range(M)]
    for z in range(N):
        for y in range(M):
            for x in range(L):
                img[y][a * x + b * z + o] += int(V[z, y, x])
    return np.array(img, dtype=np.int64)


@pytest.mark.parametrize("d", DIRS)
def test_projection_definition(d):
    V = synth.uniform_volume((5, 4, 6), np.uint16, seed=12)
    img = oracle.projection_image(V, *d)
    assert np.array_equal(img, projection_loop(V, *d))
    # every row holds the whole xz-slice mass
    assert np.array_equal(img.sum(axis=1), V.sum(axis=(0, 2), dtype=np.int64))


@pytest.mark.parametrize("d", DIRS[:8])
def test_projection_moments_are_binomial_3d_moments(d):
    """Image moments about the true origin = sum_p C(k,p) a^p b^(k-p) M_{p,q,k-p}."""
    a, b = d
    V = synth.uniform_volume((4, 3, 5), np.uint8, seed=13)
    N = V.shape[0]
    K = 5
    m = as_dict(moments_exact(V, K), K)
    img = oracle.projection_image(V, a, b)
    o = -b * (N - 1) if b < 0 else 0
    im = oracle.image_moments_2d(img, K, origin=o)
    for (k, q), val in im.items():
        ex = sum(comb(k, p) * a**p * b ** (k - p) * m[(p, q, k - p)] for p in range(k + 1))
        assert val == ex


def paper_images(V):
    """The five projections of Section 4 (Listing 1), as (row j, column i) arrays."""
    N, M, L = V.shape
    XY = oracle.projection_image(V, 1, 0)                 # i = x, j = y        eq. (5)
    YZ = oracle.projection_image(V, 0, 1)                 # stored [y][z]; eq. (6) has i = y, j = z
    ZX = np.zeros((L, N), dtype=np.int64)                 # eq. (7): i = z, j = x -> stored [x][z]
    for z in range(N):
        ZX[:, z] = V[z].sum(axis=0, dtype=np.int64)
    XPZ = oracle.projection_image(V, 1, 1)                # i = x + z, j = y      eq. (8)
    XMZ = oracle.projection_image(V, 1, -1)               # i = x - z (+ N - 1)   eq. (9)
    return XY, YZ, ZX, XPZ, XMZ


def test_paper_equations_10_to_16():
    V = synth.uniform_volume((6, 5, 7), np.uint16, seed=14)
    N = V.shape[0]
    m = as_dict(moments_exact(V, 4), 4)
    XY, YZ, ZX, XPZ, XMZ = paper_images(V)
    mxy = oracle.image_moments_2d(XY, 4)
    # eq. (6) puts i = y on the first index: transpose the [y][z] storage to [z][y]
    myz = oracle.image_moments_2d(np.ascontiguousarray(YZ.T), 4)
    mzx = oracle.image_moments_2d(ZX, 4)
    mp = oracle.image_moments_2d(XPZ, 4)
    mm = oracle.image_moments_2d(XMZ, 4, origin=N - 1)
    for p in range(5):
        for q in range(5 - p):
            assert m[(p, q, 0)] == mxy[(p, q)]          # eq. (10)
            assert m[(0, p, q)] == myz[(p, q)]          # eq. (11)
            assert m[(q, 0, p)] == mzx[(p, q)]          # eq. (12)
    assert 2 * m[(1, 1, 1)] == mp[(2, 1)] - m[(2, 1, 0)] - m[(0, 1, 2)]     # eq. (13)
    assert 2 * m[(1, 2, 1)] == mp[(2, 2)] - m[(2, 2, 0)] - m[(0, 2, 2)]     # eq. (14)
    # eqs. (15)/(16) with their left-hand sides exchanged
    assert 6 * m[(2, 1, 1)] == mp[(3, 1)] - mm[(3, 1)] - 2 * m[(0, 1, 3)]
    assert 6 * m[(1, 1, 2)] == mp[(3, 1)] + mm[(3, 1)] - 2 * m[(3, 1, 0)]
    # the printed assignment does not hold on a generic volume
    assert 6 * m[(1, 1, 2)] != mp[(3, 1)] - mm[(3, 1)] - 2 * m[(0, 1, 3)]


def test_paper_negative_index_offset_correction():
    """Section 5: moments of the x - z image taken at its stored column index, then
    shifted to the origin x-hat = N - 1 with the printed M31 and M13 formulas."""
    V = synth.uniform_volume((5, 4, 6), np.uint8, seed=15)
    N = V.shape[0]
    XMZ = oracle.projection_image(V, 1, -1)
    raw = oracle.image_moments_2d(XMZ, 4, origin=0)        # stored column index
    true = oracle.image_moments_2d(XMZ, 4, origin=N - 1)
    xh = N - 1
    assert true[(3, 1)] == raw[(3, 1)] - 3 * raw[(2, 1)] * xh + 3 * raw[(1, 1)] * xh**2 - raw[(0, 1)] * xh**3
    assert true[(1, 3)] == raw[(1, 3)] - raw[(0, 3)] * xh
    # the general binomial shift the printed cases instantiate
    for (k, q), v in true.items():
        assert v == sum(comb(k, t) * (-xh) ** (k - t) * raw[(t, q)] for t in range(k + 1))


def test_moment_single_matches():
    V = synth.uniform_volume((6, 7, 5), np.uint16, seed=16)
    m = as_dict(moments_exact(V, 6), 6)
    for t in [(0, 0, 0), (6, 0, 0), (0, 6, 0), (0, 0, 6), (2, 2, 2), (1, 3, 2)]:
        assert moment_single(V, *t) == m[t]


# ---- features of Section 4 (centroid, central, normalised, physical-spacing moments)

@pytest.mark.parametrize("seed", range(4))
def test_central_from_raw_equals_definition(seed):
    """The binomial expansion from raw moments equals the direct translated sum."""
    rng = np.random.default_rng(seed)
    V = rng.integers(0, 9, size=tuple(int(s) for s in rng.integers(1, 6, size=3))).astype(np.uint8)
    V[0, 0, 0] += 1  # non-zero mass
    K = 5
    assert oracle.central_from_raw(oracle.moments_exact(V, K), K) == oracle.central_moments(V, K)


def test_central_moments_of_a_box_closed_form():
    """A uniform box: mu_pqr = c * S_p(L) S_q(M) S_r(N), S_k(n) = sum_{x<n} (x - (n-1)/2)^k
    (zero for odd k)."""
    from fractions import Fraction
    N, M, L, c = 5, 4, 7, 3
    V = np.full((N, M, L), c, dtype=np.uint8)
    K = 6

    def S(k, n):
        return sum((Fraction(x) - Fraction(n - 1, 2)) ** k for x in range(n))

    mu = oracle.central_from_raw(oracle.moments_exact(V, K), K)
    for (p, q, r), v in mu.items():
        assert v == c * S(p, L) * S(q, M) * S(r, N), (p, q, r)
        if p % 2 or q % 2 or r % 2:
            assert v == 0


def test_features_eta_and_spacing_definitions():
    from fractions import Fraction
    V = np.random.default_rng(3).integers(0, 50, size=(6, 5, 7)).astype(np.uint8)
    K = 4
    raw = oracle.moments_exact(V, K)
    f = oracle.features(raw, K, spacing=(2.0, 3.0, 0.5))
    idx = {pqr: i for i, pqr in enumerate(oracle.moment_list(K))}
    m000 = int(raw[0])
    assert f["eta"][idx[(0, 0, 0)]] == 1.0
    assert f["mu"][idx[(1, 0, 0)]] == f["mu"][idx[(0, 1, 0)]] == f["mu"][idx[(0, 0, 1)]] == 0.0
    assert f["centroid"][0] == float(Fraction(int(raw[idx[(1, 0, 0)]]), m000))
    for (p, q, r), i in idx.items():
        mu = f["mu_exact"][(p, q, r)]
        assert f["mu_phys"][i] == float(Fraction(2) ** (1 + p) * Fraction(3) ** (1 + q) * Fraction(1, 2) ** (1 + r) * mu)
        n = p + q + r
        assert abs(f["eta"][i] - float(mu) / m000 ** (n / 3 + 1)) <= 1e-12 * max(abs(f["eta"][i]), 1e-300)
    g = oracle.features(raw, K)
    assert g["mu_phys"] == g["mu"]


def test_features_order_zero_uses_first_order_raw_moments():
    V = np.random.default_rng(5).integers(0, 9, size=(3, 4, 5)).astype(np.uint8)
    V[1, 1, 1] += 1
    raw = oracle.moments_exact(V, 1)
    f = oracle.features(raw, 0)
    assert f["mu"] == [float(raw[0])] and f["eta"] == [1.0]
    with pytest.raises(ValueError):
        oracle.central_from_raw(raw[:1], 0)


@pytest.mark.parametrize("seed", range(3))
def test_features_mu_phys_is_the_physical_coordinate_sum(seed):
    """Section 4's spacing normalisation pinned to what it stands for: the central moment
    of the volume placed at physical positions (alpha x, beta y, delta z), every voxel
    weighing its physical volume alpha beta delta -- a direct exact-rational sum over the
    voxels, with anisotropic spacing."""
    from fractions import Fraction
    rng = np.random.default_rng(100 + seed)
    V = rng.integers(0, 30, size=(4, 3, 5)).astype(np.uint8)
    V[1, 1, 1] += 1
    K = 4
    spacing = (0.5, 0.75, 2.5)  # exactly representable
    al, be, de = (Fraction(s) for s in spacing)
    f = oracle.features(oracle.moments_exact(V, K), K, spacing=spacing)
    zz, yy, xx = np.nonzero(V)
    vals = [int(V[a, b, c]) for a, b, c in zip(zz, yy, xx)]
    mass = sum(vals) * al * be * de
    X = [al * int(c) for c in xx]
    Y = [be * int(b) for b in yy]
    Z = [de * int(a) for a in zz]
    w = [v * al * be * de for v in vals]
    xb = sum(wi * xi for wi, xi in zip(w, X)) / mass
    yb = sum(wi * yi for wi, yi in zip(w, Y)) / mass
    zb = sum(wi * zi for wi, zi in zip(w, Z)) / mass
    for i, (p, q, r) in enumerate(oracle.moment_list(K)):
        direct = sum(wi * (xi - xb) ** p * (yi - yb) ** q * (zi - zb) ** r for wi, xi, yi, zi in zip(w, X, Y, Z))
        assert f["mu_phys"][i] == float(direct), (p, q, r)


@pytest.mark.parametrize("seed", range(3))
def test_features_eta_exact_where_the_exponent_is_an_integer(seed):
    """eta = mu / mu000^(n/3 + 1) is an exact rational when n/3 + 1 is an integer
    (n = 0, 3, 6): there the oracle's value is the nearest double of mu / mu000^(n/3 + 1)
    with mu the direct translated sum.  At every other order, eta^3 mu000^(n+3) = mu^3
    (which fixes the exponent) to the working precision."""
    from fractions import Fraction
    rng = np.random.default_rng(200 + seed)
    V = rng.integers(0, 12, size=(5, 4, 6)).astype(np.uint8)
    V[2, 1, 3] += 1
    K = 6
    f = oracle.features(oracle.moments_exact(V, K), K)
    mu = oracle.central_moments(V, K)
    m000 = mu[(0, 0, 0)]
    assert m000 == int(V.sum())
    for i, (p, q, r) in enumerate(oracle.moment_list(K)):
        n = p + q + r
        if n % 3 == 0:
            assert f["eta"][i] == float(mu[(p, q, r)] / Fraction(m000) ** (n // 3 + 1)), (p, q, r)
        else:
            lhs = Fraction(f["eta"][i]) ** 3 * Fraction(m000) ** (n + 3)
            rhs = mu[(p, q, r)] ** 3
            assert abs(lhs - rhs) <= Fraction(1, 10 ** 13) * abs(rhs) + Fraction(1, 10 ** 300), (p, q, r)
