"""Exact CPU definitions of the quantities the DPM method computes.

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Every function here is a
plain definition from Diggin & Diggin, "Fast 3D Image Moments" (arXiv 2012.08099),
written out in exact integer (or exact rational) arithmetic:

* ``moments_bruteforce`` / ``moments_exact`` / ``moment_single``: the 3D moment
  generating sum of Section 1, eq. (2), over 0 <= x < L, 0 <= y < M, 0 <= z < N.
* ``projection_image``: the discrete projection of Section 3.1, eq. (4), for an
  aligned direction; eqs. (5), (6), (8) and (9) are the directions (1,0), (0,1),
  (1,1) and (1,-1); the further projections listed after eq. (9) (arctan(1/2),
  arctan(2), ...) are the other integer directions.
* ``image_moments_2d``: the 2D moment sum of Section 1, eq. (1).
* ``central_moments``: the central moments of Section 4 (centroid, then the
  translated sum), in exact rationals.
* ``central_from_raw``: the same central moments from exact raw moments, by expanding
  the three binomials of that sum (checked against ``central_moments``).
* ``features``: centroid, central moments, the scale-normalised moments and the
  physical-spacing moments of Section 4, from exact raw moments.

Volumes are numpy arrays of shape (N, M, L) indexed V[z][y][x] (x contiguous, the
memory order of the projection pseudo-code in Section 5).  Coordinates are 0-based as
in the bounds of eq. (2), and 0**0 == 1.

Moment vectors use the graded order: total order n = p+q+r ascending; within one n,
p descending, then q descending.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

__all__ = [
    "moment_list",
    "moment_index",
    "moments_bruteforce",
    "moments_exact",
    "moment_single",
    "projection_image",
    "image_moments_2d",
    "central_moments",
    "central_from_raw",
    "features",
]


def moment_list(K):
    """All (p, q, r) with p+q+r <= K in graded order."""
    out = []
    for n in range(K + 1):
        for p in range(n, -1, -1):
            for q in range(n - p, -1, -1):
                out.append((p, q, n - p - q))
    return out


def moment_index(p, q, r):
    """Position of (p, q, r) in the graded order (by enumeration)."""
    n = p + q + r
    for i, t in enumerate(moment_list(n)):
        if t == (p, q, r):
            return i
    raise ValueError((p, q, r))


def _as_int_array(V):
    V = np.asarray(V)
    if V.ndim != 3:
        raise ValueError("volume must be 3-D (N, M, L) = (z, y, x)")
    if V.dtype.kind not in "ui":
        raise ValueError("volume must hold integers")
    return V


def moments_bruteforce(V, K):
    """Eq. (2) literally: one pass over the voxels, every monomial per voxel.

    Pure Python; only for tiny volumes.  Returns a list in graded order.
    """
    V = _as_int_array(V)
    N, M, L = V.shape
    mons = moment_list(K)
    acc = [0] * len(mons)
    for z in range(N):
        for y in range(M):
            for x in range(L):
                v = int(V[z, y, x])
                if v == 0:
                    continue
                for i, (p, q, r) in enumerate(mons):
                    acc[i] += v * x**p * y**q * z**r
    return acc


def _x_power_sums(V, K):
    """A[z][y][p] = sum_x x**p V[z][y][x] as exact Python ints (object array).

    A float64 matrix product is used as the summation step.  It is exact because
    x**p is split into base-2**b limbs with vmax * (2**b - 1) * L < 2**53, so every
    product and every partial sum is an integer below 2**53.
    """
    N, M, L = V.shape
    vmax = int(V.max()) if V.size else 0
    if vmax == 0:
        return np.zeros((N, M, K + 1), dtype=object)
    b = 53 - vmax.bit_length() - max(1, (L - 1).bit_length() if L > 1 else 1) - 1
    b = max(1, min(b, 30))
    mask = (1 << b) - 1
    pows = [[x**p for p in range(K + 1)] for x in range(L)]
    maxbits = max(1, max(v.bit_length() for row in pows for v in row))
    nlimb = (maxbits + b - 1) // b
    Vf = V.reshape(N * M, L).astype(np.float64)
    A = np.zeros((N * M, K + 1), dtype=object)
    for l in range(nlimb):
        W = np.array([[(pows[x][p] >> (b * l)) & mask for p in range(K + 1)] for x in range(L)],
                     dtype=np.float64)
        if not W.any():
            continue
        R = Vf @ W
        assert R.max() < 2.0**53
        A += R.astype(np.int64).astype(object) * (1 << (b * l))
    return A.reshape(N, M, K + 1)


def moments_exact(V, K):
    """Eq. (2) with the loop-invariant powers hoisted; exact Python integers.

    M_pqr = sum_z z**r sum_y y**q sum_x x**p V(x, y, z).
    Returns a list in graded order.
    """
    V = _as_int_array(V)
    N, M, L = V.shape
    A = _x_power_sums(V, K)                       # [z][y][p]
    ypow = np.array([[y**q for q in range(K + 1)] for y in range(M)], dtype=object)  # [y][q]
    # B[z][p][q] = sum_y y**q A[z][y][p]
    B = np.zeros((N, K + 1, K + 1), dtype=object)
    for q in range(K + 1):
        B[:, :, q] = (A * ypow[None, :, q, None]).sum(axis=1)
    out = []
    for (p, q, r) in moment_list(K):
        out.append(sum(z**r * B[z, p, q] for z in range(N)))
    return [int(v) for v in out]


def moment_single(V, p, q, r):
    """One moment M_pqr by eq. (2), exact (same hoisting as ``moments_exact``)."""
    V = _as_int_array(V)
    N, M, L = V.shape
    K = p
    A = _x_power_sums(V, K)[:, :, p]              # [z][y]
    ypow = np.array([y**q for y in range(M)], dtype=object)
    B = (A * ypow[None, :]).sum(axis=1)           # [z]
    return int(sum(z**r * B[z] for z in range(N)))


def projection_image(V, alpha, beta):
    """Discrete projection of eq. (4) along the aligned direction (alpha, beta).

    I(i, y) = sum of V(x, y, z) over alpha*x + beta*z + o == i, where the offset
    o = |beta| (N - 1) when beta < 0 (the negative-index shift of eq. (9), stored at
    column x - z + N - 1 in the projection pseudo-code) and 0 otherwise.
    Returns an int64 array of shape (M, W), W = alpha (L-1) + |beta| (N-1) + 1.
    """
    V = _as_int_array(V)
    N, M, L = V.shape
    if alpha < 0 or (alpha == 0 and beta <= 0):
        raise ValueError("direction must have alpha > 0, or alpha == 0 and beta > 0")
    o = -beta * (N - 1) if beta < 0 else 0
    W = alpha * (L - 1) + abs(beta) * (N - 1) + 1
    img = np.zeros((M, W), dtype=np.int64)
    x = np.arange(L)
    for z in range(N):
        cols = alpha * x + beta * z + o
        for y in range(M):
            np.add.at(img[y], cols, V[z, y].astype(np.int64))
    return img


def image_moments_2d(img, K, origin=0):
    """2D moments of eq. (1) of an image stored as img[j][i] (row j, column i).

    M_pq = sum_{i,j} I(i, j) (i - origin)**p j**q for p+q <= K, returned as a dict.
    ``origin`` places the moment origin inside the image, as the offset correction
    for the negative-index projection in Section 5 does (origin = N - 1).
    """
    img = np.asarray(img)
    H, W = img.shape
    out = {}
    for p in range(K + 1):
        for q in range(K + 1 - p):
            s = 0
            for j in range(H):
                row = img[j]
                rs = 0
                for i in range(W):
                    v = int(row[i])
                    if v:
                        rs += v * (i - origin) ** p
                s += rs * j**q
            out[(p, q)] = s
    return out


def central_moments(V, K):
    """Central moments mu_pqr of Section 4, exact rationals, by definition.

    Centroid (x, y, z)-bar = (M100, M010, M001) / M000, then
    mu_pqr = sum V (x - xbar)**p (y - ybar)**q (z - zbar)**r.  Small volumes only.
    """
    V = _as_int_array(V)
    N, M, L = V.shape
    m000 = int(V.sum(dtype=np.int64))
    if m000 == 0:
        raise ValueError("empty volume has no centroid")
    zz, yy, xx = np.nonzero(V)
    vals = [int(V[a, b, c]) for a, b, c in zip(zz, yy, xx)]
    xbar = Fraction(sum(v * int(c) for v, c in zip(vals, xx)), m000)
    ybar = Fraction(sum(v * int(b) for v, b in zip(vals, yy)), m000)
    zbar = Fraction(sum(v * int(a) for v, a in zip(vals, zz)), m000)
    out = {}
    for (p, q, r) in moment_list(K):
        s = Fraction(0)
        for v, a, b, c in zip(vals, zz, yy, xx):
            s += v * (int(c) - xbar) ** p * (int(b) - ybar) ** q * (int(a) - zbar) ** r
        out[(p, q, r)] = s
    return out


def central_from_raw(raw, K):
    """Central moments of Section 4 from the exact raw moments ``raw`` (graded order, all
    orders up to some order >= max(K, 1)), exact rationals: expanding (x - xbar)^p (y - ybar)^q (z - zbar)^r binomially,
    mu_pqr = sum_{a<=p, b<=q, c<=r} C(p,a) C(q,b) C(r,c) (-xbar)^(p-a) (-ybar)^(q-b)
    (-zbar)^(r-c) M_abc."""
    from math import comb
    kr = 0
    while (kr + 1) * (kr + 2) * (kr + 3) // 6 < len(raw):
        kr += 1
    if (kr + 1) * (kr + 2) * (kr + 3) // 6 != len(raw) or kr < max(K, 1):
        raise ValueError("raw must hold every moment of some order >= max(K, 1)")
    M = {pqr: int(v) for pqr, v in zip(moment_list(kr), raw)}
    m000 = M[(0, 0, 0)]
    if m000 == 0:
        raise ValueError("empty volume has no centroid")
    xb, yb, zb = Fraction(M[(1, 0, 0)], m000), Fraction(M[(0, 1, 0)], m000), Fraction(M[(0, 0, 1)], m000)
    out = {}
    for (p, q, r) in moment_list(K):
        s = Fraction(0)
        for a in range(p + 1):
            for b in range(q + 1):
                for c in range(r + 1):
                    s += (comb(p, a) * comb(q, b) * comb(r, c) * (-xb) ** (p - a) * (-yb) ** (q - b)
                          * (-zb) ** (r - c) * M[(a, b, c)])
        out[(p, q, r)] = s
    return out


def features(raw, K, spacing=(1, 1, 1)):
    """The object features of Section 4 from exact raw moments (graded order):
    centroid = (M100, M010, M001) / M000; mu = central moments (exact rationals);
    eta_pqr = mu_pqr / mu_000^((p+q+r)/3 + 1), evaluated in 60-digit decimal arithmetic;
    mu_phys_pqr = alpha^(1+p) beta^(1+q) delta^(1+r) mu_pqr with (alpha, beta, delta) =
    spacing taken exactly.  Returns floats (nearest double of each quantity) and the
    exact mu."""
    from decimal import Decimal, localcontext
    mu = central_from_raw(raw, K)
    m000 = int(raw[0])
    al, be, de = (Fraction(s) for s in spacing)
    out = {"centroid": [float(Fraction(int(raw[i]), m000)) for i in (1, 2, 3)], "mu_exact": mu,
           "mu": [], "eta": [], "mu_phys": []}
    with localcontext() as ctx:
        ctx.prec = 60
        dm = Decimal(m000)
        for (p, q, r) in moment_list(K):
            v = mu[(p, q, r)]
            n = p + q + r
            out["mu"].append(float(v))
            e = (Decimal(v.numerator) / Decimal(v.denominator)) / dm ** (Decimal(n) / Decimal(3) + 1)
            out["eta"].append(float(e))
            out["mu_phys"].append(float(al ** (1 + p) * be ** (1 + q) * de ** (1 + r) * v))
    return out
