"""The paper's own five-image route and its 1D-integral step -- TEST INFRASTRUCTURE ONLY.

Plain CPU definitions, in exact integers and exact rationals, of the pieces of the DPM
method as Diggin & Diggin ("Fast 3D Image Moments", arXiv 2012.08099) print them for
orders <= 4:

* ``paper_images``: the projections of Section 3.1 -- I(x, y) (eq. 5), I(y, z) (eq. 6),
  I(z, x) (eq. 7), I(x + z, y) (eq. 8) and I(x - z, y) (eq. 9), the last stored at
  column x - z + N - 1 as in the projection listing of Section 5.  Order 3 needs the
  first four, orders <= 2 the first three, order 4 all five (Section 4).
* ``drt_integrals``: the five 1D integrals of a 2D image of Section 5 (onto the x axis,
  the y axis, the 45 and 135 degree axes and the arctan(1/2) axis), by definition.
* ``moments_2d_from_integrals``: the 2D moments of an image from the 1D moments of
  those integrals.  Expanding (a i + b j)^n binomially gives, for each order n, a
  linear system in the n + 1 moments M_{p, n-p}; it is solved here in exact rationals.
  (The paper takes this step from a companion paper that is not available; this is
  the binomial reading of it.)
* ``paper_moments``: the 3D moments from the five images' 2D moments by eqs. 10-16,
  with the left-hand sides of eqs. 15 and 16 exchanged (the printed assignment does
  not hold; see tests) and the X - Z image's moments shifted to the origin N - 1 by the
  binomial correction of Section 5.

Images are numpy arrays img[j][i] (row j, column i) of I(i, j) as the paper indexes it.
Only ``tests/`` uses this module.
"""
from __future__ import annotations

from fractions import Fraction
from math import comb

import numpy as np

from .moments import image_moments_2d, moment_list

# directions of the 1D integrals, t = a i + b j: Vert, Horiz, Diag, AntiDiag, X2Y
DRT_DIRS = ((1, 0), (0, 1), (1, 1), (1, -1), (1, 2))


def n_paper_images(K):
    """Images the paper's route needs for moments of order <= K (<= 4)."""
    if not 0 <= K <= 4:
        raise ValueError("the paper's route covers orders 0..4")
    return 3 if K <= 2 else K + 1


def paper_images(V, K):
    """[XY, YZ, ZX, X+Z, X-Z][:n_paper_images(K)], each an int64 array img[j][i].

    XY: i = x, j = y (M x L); YZ: i = y, j = z (N x M); ZX: i = z, j = x (L x N);
    X+Z: i = x + z, j = y (M x (L+N-1)); X-Z: i = x - z + N - 1, j = y (M x (L+N-1)).
    Built by accumulating every voxel into every image, as the projection listing of
    Section 5 does (pure additions)."""
    V = np.asarray(V)
    N, M, L = V.shape
    n = n_paper_images(K)
    W = L + N - 1
    XY = np.zeros((M, L), dtype=np.int64)
    YZ = np.zeros((N, M), dtype=np.int64)
    ZX = np.zeros((L, N), dtype=np.int64)
    XPZ = np.zeros((M, W), dtype=np.int64)
    XMZ = np.zeros((M, W), dtype=np.int64)
    x = np.arange(L)
    for z in range(N):
        for y in range(M):
            row = V[z, y].astype(np.int64)
            XY[y] += row                        # I(i = x, j = y)
            YZ[z, y] += int(row.sum())          # I(i = y, j = z)
            ZX[:, z] += row                     # I(i = z, j = x)
            np.add.at(XPZ[y], x + z, row)       # I(i = x + z, j = y)
            np.add.at(XMZ[y], x - z + N - 1, row)  # I(i = x - z + N - 1, j = y)
    return [XY, YZ, ZX, XPZ, XMZ][:n]


def drt_integrals(img, ndir):
    """The first ``ndir`` 1D integrals of Section 5 of img[j][i]:
    P_g(t) = sum of I(i, j) over a_g i + b_g j = t, (a_g, b_g) = DRT_DIRS[g].
    Returns [(tmin_g, P_g)] with P_g[t - tmin_g]."""
    img = np.asarray(img)
    H, W = img.shape
    out = []
    for a, b in DRT_DIRS[:ndir]:
        ts = [a * i + b * j for i in (0, W - 1) for j in (0, H - 1)]
        tmin, tmax = min(ts), max(ts)
        P = [0] * (tmax - tmin + 1)
        for j in range(H):
            for i in range(W):
                v = int(img[j, i])
                if v:
                    P[a * i + b * j - tmin] += v
        out.append((tmin, P))
    return out


def moments_2d_from_integrals(integrals, K, origin=0):
    """2D moments M_{p,q} = sum I(i, j) (i - origin)^p j^q, p + q <= K, of an image
    from its 1D integrals (``drt_integrals`` with ndir >= K + 1).

    The 1D moment of integral g about the image's moment origin is
    m_{g,n} = sum_t (t - a_g origin)^n P_g(t) = sum_p C(n,p) a_g^p b_g^(n-p) M_{p,n-p};
    the first n + 1 directions give an invertible system for each n."""
    if len(integrals) < K + 1:
        raise ValueError("need K + 1 integrals")
    out = {}
    for n in range(K + 1):
        m = []
        for g in range(n + 1):
            a, b = DRT_DIRS[g]
            tmin, P = integrals[g]
            m.append(sum((tmin + k - a * origin) ** n * v for k, v in enumerate(P) if v))
        A = [[Fraction(comb(n, p) * DRT_DIRS[g][0] ** p * DRT_DIRS[g][1] ** (n - p)) for p in range(n + 1)]
             for g in range(n + 1)]
        sol = _solve(A, [Fraction(v) for v in m])
        for p in range(n + 1):
            assert sol[p].denominator == 1, "the 2D moments of an integer image are integers"
            out[(p, n - p)] = int(sol[p])
    return out


def _solve(A, rhs):
    """Exact Gaussian elimination over the rationals."""
    n = len(A)
    A = [row[:] + [r] for row, r in zip(A, rhs)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    return [A[r][n] / A[r][r] for r in range(n)]


def paper_moments(V, K):
    """3D moments of order <= K (<= 4) by the paper's route: the images of Section 3.1,
    their 2D moments (eq. 1), eqs. 10-16 (15/16 with exchanged left-hand sides) and the
    Section 5 offset of the X - Z image.  Returns a list in graded order."""
    imgs = paper_images(V, K)
    N = np.asarray(V).shape[0]
    mom = [image_moments_2d(im, K) for im in imgs]
    XY, YZ, ZX = mom[0], mom[1], mom[2]
    out = []
    for (p, q, r) in moment_list(K):
        if r == 0:
            v = XY[(p, q)]                       # eq. 10
        elif p == 0:
            v = YZ[(q, r)]                       # eq. 11
        elif q == 0:
            v = ZX[(r, p)]                       # eq. 12
        elif (p, q, r) == (1, 1, 1):
            v = Fraction(mom[3][(2, 1)] - XY[(2, 1)] - YZ[(1, 2)], 2)  # eq. 13
        elif (p, q, r) == (1, 2, 1):
            v = Fraction(mom[3][(2, 2)] - XY[(2, 2)] - YZ[(2, 2)], 2)  # eq. 14
        else:
            xh = N - 1
            raw = mom[4]
            m31 = raw[(3, 1)] - 3 * raw[(2, 1)] * xh + 3 * raw[(1, 1)] * xh ** 2 - raw[(0, 1)] * xh ** 3
            if (p, q, r) == (1, 1, 2):
                v = Fraction(mom[3][(3, 1)] + m31 - 2 * XY[(3, 1)], 6)
            else:  # (2, 1, 1)
                v = Fraction(mom[3][(3, 1)] - m31 - 2 * YZ[(1, 3)], 6)
        assert Fraction(v).denominator == 1
        out.append(int(v))
    return out
