"""GPU tests of the served loop (dpm_server_*): every request's result equals the same
volume's single-call result and the oracle; small requests are batched; admission
respects the device-memory budget; inputs may start on the host or on the device.
"""
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


def drain(srv, n, timeout_ms=60000):
    got = []
    t0 = srv.now_ms()
    while len(got) < n:
        got += srv.poll(256, wait_ms=50)
        assert srv.now_ms() - t0 < timeout_ms, f"only {len(got)} of {n} completions"
    return got


def mixed_requests(seed, n):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        u = rng.uniform()
        if u < 0.6:
            shape = tuple(int(s) for s in rng.integers(3, 40, size=3))
            V = synth.sphere_mask(shape, rng)
            K = int(rng.integers(0, 7))
        elif u < 0.9:
            shape = tuple(int(s) for s in rng.integers(16, 70, size=3))
            V = synth.uniform_volume(shape, np.uint16, seed=int(rng.integers(1 << 30)))
            K = int(rng.integers(2, 9))
        else:
            shape = (64, 64, 64)
            V = synth.mri_phantom(shape, seed=int(rng.integers(1 << 30)))
            K = int(rng.integers(5, 11))
        reqs.append((V, K, bool(rng.integers(0, 2))))
    return reqs


def test_server_matches_oracle_mixed(dpm):
    import torch
    say("server mixed")
    reqs = mixed_requests(7, 120)
    srv = dpm.Server(hbm_budget=1 << 30, n_streams=3, batch_voxels=40 ** 3, batch_max=64)
    try:
        tags = {}
        for V, K, on_dev in reqs:
            vol = to_dev(V) if on_dev else torch.from_numpy(V.view(np.int16) if V.dtype == np.uint16 else V)
            tags[srv.submit(vol, K)] = (V, K)
        done = drain(srv, len(reqs))
        stats = srv.stats()
    finally:
        srv.close()
    assert sorted(c["tag"] for c in done) == sorted(tags)
    assert stats["batched_jobs"] >= 1 and stats["single_jobs"] >= 1
    for c in done:
        V, K = tags[c["tag"]]
        assert c["status"] == 0
        assert c["t_arrival_ms"] <= c["t_start_ms"] <= c["t_done_ms"]
        small = V.size <= 40 ** 3 and K <= 6
        assert c["batched"] == small
        assert_moments_equal(c["moments"], oracle.moments_exact(V, K), K, f"tag {c['tag']} {V.shape} K={K}")


def test_server_admission_waits_for_budget(dpm):
    """A budget that holds about one medium job at a time: requests queue, still all
    complete, in full, and the arena's peak stays inside the budget."""
    say("server budget")
    shape = (64, 96, 80)
    vols = [synth.uniform_volume(shape, np.uint16, seed=s) for s in range(12)]
    ws = dpm.workspace_bytes(shape, 2, 5)
    budget = ws + ws // 2 + (64 << 10)  # one job's workspace and outputs, not two
    srv = dpm.Server(hbm_budget=budget, n_streams=2, batch_voxels=0, batch_max=1)
    try:
        tags = {srv.submit(to_dev(V), 5): V for V in vols}
        done = drain(srv, len(vols))
        stats = srv.stats()
    finally:
        srv.close()
    assert stats["arena_peak_used"] <= budget
    for c in done:
        assert c["status"] == 0
        assert_moments_equal(c["moments"], oracle.moments_exact(tags[c["tag"]], 5), 5, "budget")


def test_server_refuses_what_cannot_fit(dpm):
    srv = dpm.Server(hbm_budget=1 << 20, n_streams=1)
    try:
        with pytest.raises(dpm.DpmError):
            srv.submit(to_dev(np.zeros((128, 128, 128), np.uint16)), 6)
        with pytest.raises((dpm.DpmError, ValueError)):
            srv.submit(to_dev(np.zeros((4, 4, 4), np.uint16)), 17)
    finally:
        srv.close()


def test_server_same_volume_alone_and_in_a_mix(dpm):
    """One volume's result does not depend on what it was served with."""
    say("server alone vs mix")
    V = synth.mri_phantom((40, 36, 44), seed=5)
    alone = dpm.moments(to_dev(V), 6)
    srv = dpm.Server(hbm_budget=1 << 30, n_streams=2, batch_voxels=64 ** 3)
    try:
        others = [synth.uniform_volume((20, 24, 28), np.uint8, seed=s) for s in range(30)]
        for i, o in enumerate(others):
            srv.submit(to_dev(o), 6)
            if i == 15:
                t = srv.submit(to_dev(V), 6)
        done = drain(srv, 31)
    finally:
        srv.close()
    mine = [c for c in done if c["tag"] == t][0]
    assert mine["batched"]
    assert mine["moments"].exact == alone.exact
    assert np.array_equal(mine["moments"].fp64.view(np.uint64), alone.fp64.view(np.uint64))


def test_server_serves_unbatchable_small_request_alone(dpm):
    """A request that is small in voxels but whose full-z image rows exceed the batched
    path's LDS (a 4096-deep column at order 6) is served by the single-volume path."""
    say("server unbatchable")
    V = synth.uniform_volume((4096, 1, 1), np.uint8, seed=1)
    W = synth.uniform_volume((20, 20, 20), np.uint8, seed=2)
    srv = dpm.Server(hbm_budget=1 << 28, n_streams=1, batch_voxels=1 << 20)
    try:
        tv = srv.submit(to_dev(V), 6)
        tw = srv.submit(to_dev(W), 6)
        done = {c["tag"]: c for c in drain(srv, 2)}
    finally:
        srv.close()
    assert done[tv]["status"] == 0 and not done[tv]["batched"]
    assert done[tw]["status"] == 0 and done[tw]["batched"]
    assert_moments_equal(done[tv]["moments"], oracle.moments_exact(V, 6), 6, "column")
    assert_moments_equal(done[tw]["moments"], oracle.moments_exact(W, 6), 6, "cube")


def test_server_requery_from_resident_image_moments(dpm):
    """Requests kept resident answer later queries of any order up to theirs from their
    image moments on the device, equal to the oracle; batched and single requests."""
    say("server requery")
    small = synth.sphere_mask((30, 26, 34), np.random.default_rng(3))
    large = synth.mri_phantom((72, 64, 80), seed=4)
    srv = dpm.Server(hbm_budget=1 << 30, n_streams=2, batch_voxels=40 ** 3)
    try:
        ts = srv.submit(to_dev(small), 6, keep=True)
        tl = srv.submit(to_dev(large), 9, keep=True)
        tn = srv.submit(to_dev(small), 6)  # not kept
        done = {c["tag"]: c for c in drain(srv, 3)}
        assert done[ts]["batched"] and not done[tl]["batched"]
        st = srv.stats()
        assert st["resident"] == 2 and st["resident_bytes"] > 0
        for tag, V, K in [(ts, small, 6), (tl, large, 9)]:
            ref = oracle.moments_exact(V, K)
            for k in sorted({0, 1, 4, K // 2, K}):
                got = srv.requery(tag, k)
                assert_moments_equal(got, ref[:dpm.num_moments(k)], k, f"requery tag {tag} K={k}")
        with pytest.raises(dpm.DpmError):
            srv.requery(tn, 6)      # never kept
        with pytest.raises(dpm.DpmError):
            srv.requery(ts, 7)      # above the kept order
        srv.release_resident(ts)
        with pytest.raises(dpm.DpmError):
            srv.requery(ts, 2)
        assert srv.stats()["resident"] == 1
    finally:
        srv.close()


def test_server_evicts_resident_entries_under_budget_pressure(dpm):
    """A budget that holds one job and a few resident entries: later requests evict the
    least recently used entries; every request still completes exactly, the entries that
    remain still answer queries, and the evicted ones refuse them."""
    say("server eviction")
    shape = (48, 40, 56)
    vols = [synth.uniform_volume(shape, np.uint16, seed=10 + s) for s in range(10)]
    K = 6
    ws = dpm.workspace_bytes(shape, 2, K)
    # one job at a time (workspace, outputs, its resident block of about 11 KB) plus room
    # for a few more resident entries
    budget = ws + (64 << 10)
    srv = dpm.Server(hbm_budget=budget, n_streams=1, batch_voxels=0, batch_max=1)
    try:
        tags = []
        for V in vols:
            tags.append(srv.submit(to_dev(V), K, keep=True))
            drain(srv, 1)  # one after another: the oldest entries are the least recently used
        st = srv.stats()
        assert st["evictions"] > 0 and st["arena_peak_used"] <= budget
        alive = [t for t in tags if t in _resident_tags(srv, tags, K)]
        assert tags[-1] in alive and tags[0] not in alive
        for t in alive:
            V = vols[tags.index(t)]
            assert_moments_equal(srv.requery(t, K), oracle.moments_exact(V, K), K, f"resident {t}")
    finally:
        srv.close()


def _resident_tags(srv, tags, K):
    import paper_2012_08099_amd as dpm
    out = []
    for t in tags:
        try:
            srv.requery(t, 0)
            out.append(t)
        except dpm.DpmError:
            pass
    return out


def test_server_batches_only_requests_of_one_order(dpm):
    """Small requests of different orders, waiting together, are served in batches of one
    order each; every result is exact at its own order."""
    say("server equal-order batches")
    rng = np.random.default_rng(11)
    reqs = [(synth.sphere_mask(tuple(int(s) for s in rng.integers(8, 30, size=3)), rng), int(k))
            for k in rng.integers(0, 7, size=40)]
    srv = dpm.Server(hbm_budget=1 << 28, n_streams=1, batch_voxels=32 ** 3, batch_max=64)
    try:
        tags = {srv.submit(to_dev(V), K): (V, K) for V, K in reqs}
        done = drain(srv, len(reqs))
        st = srv.stats()
    finally:
        srv.close()
    assert st["batched_jobs"] >= len({K for _, K in reqs})
    for c in done:
        V, K = tags[c["tag"]]
        assert c["status"] == 0 and c["batched"]
        assert_moments_equal(c["moments"], oracle.moments_exact(V, K), K, f"order {K}")


def test_server_waits_for_the_kernel_that_writes_a_device_input(dpm):
    """A device volume written by a torch kernel just before submit (no synchronisation):
    the request carries an event of torch's stream, and the result is that of the
    written volume."""
    import torch
    say("server ready event")
    V = synth.uniform_volume((64, 64, 96), np.uint16, seed=21)
    src = to_dev(V)
    srv = dpm.Server(hbm_budget=1 << 30, n_streams=2, batch_voxels=0)
    try:
        tags = {}
        for i in range(4):
            dst = torch.flip(src, dims=[2]) if i % 2 else torch.roll(src, shifts=5 * i + 1, dims=0)
            ref = np.flip(V, axis=2) if i % 2 else np.roll(V, 5 * i + 1, axis=0)
            tags[srv.submit(dst, 6)] = np.ascontiguousarray(ref)
        done = drain(srv, 4)
    finally:
        srv.close()
    for c in done:
        assert_moments_equal(c["moments"], oracle.moments_exact(tags[c["tag"]], 6), 6, "flipped/rolled input")


def test_server_at_the_served_mix_sizes(dpm):
    """Requests of the served mix's own sizes: uint8 sphere ROIs of 32-128 per side,
    uint16 256 x 256 x Z slabs and the 512^3 uint16 CT-like volume, order 6, inputs on the
    device and in host memory, all in one server: every result equals the exact direct
    sums of eq. (2) (the C oracle)."""
    import torch
    import oracle.native as onative
    say("server at mix sizes")
    rng = np.random.default_rng(31)
    vols = [synth.sphere_mask((128, 96, 120), rng), synth.sphere_mask((32, 40, 64), rng),
            synth.mri_phantom((160, 256, 256), seed=2), synth.mri_phantom((300, 256, 256), seed=3),
            synth.ct_phantom((512, 512, 512), seed=1)]
    refs = [onative.moments_hoisted(V, 6) for V in vols]
    srv = dpm.Server(hbm_budget=4 << 30, n_streams=3, batch_voxels=128 ** 3)
    try:
        tags = {}
        for i, V in enumerate(vols):
            host = torch.from_numpy(V.view(np.int16) if V.dtype == np.uint16 else V)
            for on_dev in (True, False):
                tags[srv.submit(to_dev(V) if on_dev else host, 6)] = i
        done = drain(srv, len(tags), timeout_ms=120000)
    finally:
        srv.close()
    for c in done:
        i = tags[c["tag"]]
        assert c["status"] == 0
        assert_moments_equal(c["moments"], refs[i], 6, f"mix size {vols[i].shape}")
