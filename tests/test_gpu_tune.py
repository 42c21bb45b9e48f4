"""GPU test of the autotuner: every candidate work split is timed through the C ABI,
must reproduce the default plan's moments bit for bit, and the installed fastest split
still matches the oracle."""
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_moments_equal, to_dev

pytestmark = pytest.mark.gpu


def test_autotune_installs_an_exact_split():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2012_08099_amd as dpm
    from paper_2012_08099_amd import autotune
    print("autotune 64x48x96 u16 K=6", flush=True)
    sys.stdout.flush()
    V = synth.uniform_volume((64, 48, 96), np.uint16, seed=2)
    vol = to_dev(V)
    try:
        r = autotune.tune(vol, 6, reps=3, warmup=1, z_splits=(0, 1, 2, 4), power_chunks=(0, 4, -1), waves=(0, 4),
                          objective="throughput")
        assert len(r["candidates"]) == 24 and all(c["ms"] > 0 for c in r["candidates"])
        best = r["best"]
        info = dpm.plan(V.shape, 2, 6)
        if best["z_splits"]:
            assert info["z_splits"] <= best["z_splits"]
        if best["power_chunk"] > 0:
            assert info["power_chunk"] == best["power_chunk"]
        res = dpm.moments(vol, 6)
        assert_moments_equal(res, oracle.moments_exact(V, 6), 6, f"tuned {best}")
        r2 = autotune.tune(vol, 6, reps=2, warmup=1, z_splits=(0, 2), power_chunks=(0,), waves=(0,))
        assert r2["objective"] == "latency" and len(r2["candidates"]) == 2
        assert_moments_equal(dpm.moments(vol, 6), oracle.moments_exact(V, 6), 6, f"tuned {r2['best']}")
        # no candidate beats the default by the whole default time: the default stays
        r3 = autotune.tune(vol, 6, reps=2, warmup=1, z_splits=(0, 2), power_chunks=(0, 4), waves=(0, 4), margin=1.0)
        assert (r3["best"]["z_splits"], r3["best"]["power_chunk"], r3["best"]["waves"]) == (0, 0, 0)
    finally:
        autotune.clear()
