"""The stored 512^3 order-16 goldens (tests/golden, written by make_ct512_k16.py from
the oracle) re-checked on the CPU where an independent computation is cheap: the mass
and the first moments by plain numpy int64 sums (eq. 2 with p+q+r <= 1)."""
import json
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ct512_k16_seed0.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLD) as fh:
        return json.load(fh)


def test_golden_file_shape(golden):
    assert golden["max_order"] == 16
    ms = {(p, q, r): int(v) for p, q, r, v in golden["moments"]}
    assert len(ms) == len(golden["moments"]) >= 40
    assert (16, 0, 0) in ms and (0, 0, 16) in ms and (0, 0, 0) in ms
    assert all(v >= 0 for v in ms.values())  # non-negative voxels and coordinates


def test_golden_low_orders_independently(golden):
    N, M, L = golden["volume"]["shape_zyx"]
    V = synth.ct_phantom((N, M, L), seed=golden["volume"]["seed"]).astype(np.int64)
    ms = {(p, q, r): int(v) for p, q, r, v in golden["moments"]}
    assert ms[(0, 0, 0)] == int(V.sum())
    x = np.arange(L, dtype=np.int64)
    y = np.arange(M, dtype=np.int64)
    z = np.arange(N, dtype=np.int64)
    assert ms[(1, 0, 0)] == int((V.sum(axis=(0, 1)) * x).sum())
    assert ms[(0, 1, 0)] == int((V.sum(axis=(0, 2)) * y).sum())
    assert ms[(0, 0, 1)] == int((V.sum(axis=(1, 2)) * z).sum())


def test_golden_is_every_moment_to_order_16(golden):
    assert len(golden["moments"]) == 969
    assert sorted((p, q, r) for p, q, r, _ in golden["moments"]) == sorted(
        (p, q, n - p - q) for n in range(17) for p in range(n + 1) for q in range(n - p + 1))


def test_golden_moments_with_a_zero_index_from_the_marginals(golden):
    """Every stored moment with p, q or r = 0 recomputed from the volume's 2D marginal sums
    (eq. 2 summed over the missing axis first) with Python integers: a route that shares
    nothing with the oracle's limb-split products."""
    N, M, L = golden["volume"]["shape_zyx"]
    V = synth.ct_phantom((N, M, L), seed=golden["volume"]["seed"]).astype(np.int64)
    ms = {(p, q, r): int(v) for p, q, r, v in golden["moments"]}
    K = golden["max_order"]
    marg = {"xy": V.sum(axis=0), "xz": V.sum(axis=1), "yz": V.sum(axis=2)}  # [y][x], [z][x], [z][y]

    def pw(n):
        return np.array([[c ** k for k in range(K + 1)] for c in range(n)], dtype=object)

    px, py, pz = pw(L), pw(M), pw(N)
    # S[a][k] = sum_b marg[a][b] * b^k (inner axis first), then the outer powers
    Sxy = marg["xy"].astype(object) @ px   # [y][p]
    Sxz = marg["xz"].astype(object) @ px   # [z][p]
    Syz = marg["yz"].astype(object) @ py   # [z][q]
    Txy = py.T @ Sxy                       # [q][p]
    Txz = pz.T @ Sxz                       # [r][p]
    Tyz = pz.T @ Syz                       # [r][q]
    n_checked = 0
    for (p, q, r), v in ms.items():
        if r == 0:
            assert v == Txy[q][p], (p, q, r)
        elif q == 0:
            assert v == Txz[r][p], (p, q, r)
        elif p == 0:
            assert v == Tyz[r][q], (p, q, r)
        else:
            continue
        n_checked += 1
    assert n_checked == 969 - 560
