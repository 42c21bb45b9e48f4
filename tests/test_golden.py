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
