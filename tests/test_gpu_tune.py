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


def test_batch_tuning_installs_an_exact_geometry():
    """autotune.tune_batched: every batch geometry (fused or separate kernels, units per
    sub-row, slices per wave) gives the default's moments bit for bit, and the installed
    one and the forced separate route still match the exact direct sums of eq. (2)."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import oracle.native as onative
    import paper_2012_08099_amd as dpm
    from paper_2012_08099_amd import autotune
    K = 4
    rng = np.random.default_rng(7)
    rois = [synth.uniform_volume((int(rng.integers(4, 40)), int(rng.integers(1, 40)), int(rng.integers(3, 60))),
                                 np.uint8 if i % 3 else np.uint16, seed=100 + i) for i in range(40)]
    print("tune_batched 40 ROIs K=4", flush=True)
    sys.stdout.flush()
    packed, desc = dpm.pack_rois(rois, "cuda:0")
    n, nm = len(rois), dpm.num_moments(K)

    def call():
        ex = torch.zeros((n * nm, 2), dtype=torch.int64, device="cuda:0")
        fp = torch.zeros(n * nm, dtype=torch.float64, device="cuda:0")
        ws = torch.empty(max(dpm.batched_workspace_bytes(desc, K), 1), dtype=torch.uint8, device="cuda:0")
        dpm.moments_batched(packed, desc, K, ex, fp, ws)
        torch.cuda.synchronize()
        exact = dpm._exact_from_tensor(ex.cpu())
        fpn = fp.cpu().numpy()
        for i, V in enumerate(rois):
            got = dpm.Moments(K, exact[i * nm:(i + 1) * nm], fpn[i * nm:(i + 1) * nm])
            assert_moments_equal(got, onative.moments_hoisted(V, K), K, f"roi {i} {V.shape}")

    try:
        r = autotune.tune_batched(packed, desc, K, reps=3, warmup=3, confirm_rounds=1)
        assert len(r["candidates"]) == 10 and all(c["ms"] > 0 for c in r["candidates"])
        call()
        autotune.set_batch_tuning(K, fused=-1)
        call()
        autotune.set_batch_tuning(K, fused=0, units=1, max_spw=1)
        call()
        # no candidate beats the default by the whole default time: the default stays
        r2 = autotune.tune_batched(packed, desc, K, reps=2, warmup=3, units=(0, 4), max_spw=(0,), confirm_rounds=1,
                                   margin=1.0)
        assert (r2["best"]["fused"], r2["best"]["units"], r2["best"]["max_spw"]) == (0, 0, 0)
    finally:
        autotune.unset_batch_tuning(K)
