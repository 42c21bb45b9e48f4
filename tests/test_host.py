"""Host-side checks of the C ABI (no GPU needed): the library loads and exports every
function that include/dpm.h declares, and its host logic -- direction family, graded
moment index, image widths, exact recombination weights, planning and argument
checks -- matches the mathematics of Section 3.
"""
import ctypes
import os
import re
from fractions import Fraction
from math import comb

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpm.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2012_08099_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libdpm.so not built (run __graft_entry__.build())")
    return _lib.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_functions()
    for must in ("dpm_moments", "dpm_moments_async", "dpm_moments_batched", "dpm_project_images",
                 "dpm_workspace_bytes", "dpm_batched_workspace_bytes", "dpm_recomb_weight", "dpm_plan"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared in dpm.h but not exported: {missing}"


# The projection family (Section 3.1, eq. 4 and the aligned projections after eq. 9):
# (1,0), (0,1), (1,1), (1,-1), then directions with small integer slopes.
FAMILY = [(1, 0), (0, 1), (1, 1), (1, -1), (2, 1), (2, -1), (1, 2), (1, -2), (3, 1), (3, -1),
          (1, 3), (1, -3), (3, 2), (3, -2), (2, 3), (2, -3), (1, 4)]


def test_direction_family(lib):
    a, b = ctypes.c_int(), ctypes.c_int()
    got = []
    for d in range(17):
        assert lib.dpm_direction(d, ctypes.byref(a), ctypes.byref(b)) == 0
        got.append((a.value, b.value))
    assert got == FAMILY
    assert lib.dpm_direction(17, ctypes.byref(a), ctypes.byref(b)) < 0
    # every k+1 leading directions are pairwise non-parallel, so each degree-k system
    # below is invertible
    for i in range(17):
        for j in range(i):
            assert FAMILY[i][0] * FAMILY[j][1] != FAMILY[i][1] * FAMILY[j][0]


def test_moment_count_and_graded_index(lib):
    for K in range(17):
        assert lib.dpm_num_moments(K) == (K + 1) * (K + 2) * (K + 3) // 6
        for i, (p, q, r) in enumerate(oracle.moment_list(K)):
            assert lib.dpm_moment_index(p, q, r) == i == oracle.moment_index(p, q, r)
    assert lib.dpm_num_moments(17) < 0 and lib.dpm_moment_index(17, 0, 0) < 0


@pytest.mark.parametrize("dims", [(1, 1, 1), (7, 3, 5), (64, 2, 31), (512, 512, 512)])
def test_image_width(lib, dims):
    d3 = (ctypes.c_int64 * 3)(*dims)
    L, M, N = dims
    for d, (a, b) in enumerate(FAMILY):
        # bins a x + b z for x < L, z < N span a (L-1) + |b| (N-1) + 1 values
        assert lib.dpm_image_width(d3, d) == a * (L - 1) + abs(b) * (N - 1) + 1


def weights(lib, k):
    num, den = ctypes.c_int64(), ctypes.c_uint64()
    W = []
    for p in range(k + 1):
        row = []
        for d in range(k + 1):
            assert lib.dpm_recomb_weight(k, p, d, ctypes.byref(num), ctypes.byref(den)) == 0
            assert den.value > 0
            row.append(Fraction(num.value, den.value))
        W.append(row)
    return W


@pytest.mark.parametrize("k", range(17))
def test_recomb_weights_invert_the_projection_system(lib, k):
    """The 2D moment of degree (k, q) of image d about its origin expands (binomial theorem
    on (alpha x + beta z)^k, as in the derivation of eq. 13) into
        m_d = sum_p C(k,p) alpha_d^p beta_d^(k-p) M_{p,q,k-p};
    the weights must be the exact inverse of that (k+1)x(k+1) system."""
    W = weights(lib, k)
    A = [[comb(k, p) * FAMILY[d][0] ** p * FAMILY[d][1] ** (k - p) for p in range(k + 1)] for d in range(k + 1)]
    for p in range(k + 1):
        for p2 in range(k + 1):
            s = sum(W[p][d] * A[d][p2] for d in range(k + 1))
            assert s == (1 if p == p2 else 0), (k, p, p2, s)


def test_recomb_weights_match_paper_equations(lib):
    """Eqs. (10)-(16) written as weights over images d = (1,0), (0,1), (1,1), (1,-1)."""
    # eq. (10): M_{p q 0} is the (1,0) image moment; eq. (11): M_{0 q r} the (0,1) one
    for k in range(5):
        W = weights(lib, k)
        assert W[k] == [1] + [0] * k
        if k >= 1:
            assert W[0] == [0, 1] + [0] * (k - 1)
    # eqs. (13) and (14): M_{1 q 1} = (M^{pi/4}_{2q} - M_{2q0} - M_{0q2}) / 2
    assert weights(lib, 2)[1] == [Fraction(-1, 2), Fraction(-1, 2), Fraction(1, 2)]
    # eqs. (15)/(16) with their left-hand sides exchanged (expanding (x +- z)^3 y):
    #   M_{211} = (M^{+}_{31} - M^{-}_{31} - 2 M_{013}) / 6
    #   M_{112} = (M^{+}_{31} + M^{-}_{31} - 2 M_{310}) / 6
    W3 = weights(lib, 3)
    assert W3[2] == [0, Fraction(-2, 6), Fraction(1, 6), Fraction(-1, 6)]
    assert W3[1] == [Fraction(-2, 6), 0, Fraction(1, 6), Fraction(1, 6)]


def plan(lib, dims, dtype, K):
    from paper_2012_08099_amd import _lib
    info = _lib.PlanInfo()
    rc = lib.dpm_plan((ctypes.c_int64 * 3)(*dims), dtype, K, ctypes.byref(info))
    return rc, info


def test_plan_headline_workload(lib):
    rc, info = plan(lib, (512, 512, 512), 2, 6)
    assert rc == 0
    assert info.n_dirs == 7 and info.n_groups == 1 and info.n_items == 512 and info.z_splits == 1
    assert info.limbs_slice == 4 and info.limbs_moment == 4
    assert 0 < info.lds_bytes <= 160 * 1024
    ws = lib.dpm_workspace_bytes((ctypes.c_int64 * 3)(512, 512, 512), 2, 6)
    assert ws == info.workspace > 0


def test_plan_groups_and_widths_grow_with_order(lib):
    prev_bits = 0
    for K in range(17):
        rc, info = plan(lib, (128, 128, 128), 2, K)
        assert rc == 0
        assert info.n_dirs == K + 1
        assert info.n_groups == (1 if K < 7 else 2 if K < 12 else 3)
        assert info.bits_moment >= prev_bits
        prev_bits = info.bits_moment
        assert 32 * info.limbs_moment >= info.bits_moment and 32 * info.limbs_slice >= info.bits_slice


def test_plan_bits_bound_a_saturated_volume(lib):
    """bits_moment must cover the largest exact numerator: every voxel 65535 maximises
    every 2D moment magnitude, and the numerator is sum_d |num| * |m_d|."""
    L = M = N = 40
    K = 8
    rc, info = plan(lib, (L, M, N), 2, K)
    assert rc == 0
    vmax = 65535
    worst = 0
    for k in range(K + 1):
        W = weights(lib, k)
        for q in range(K - k + 1):
            for p in range(k + 1):
                den = max(w.denominator for w in W[p])
                tot = 0
                for d in range(k + 1):
                    a, b = FAMILY[d]
                    m = sum(abs(a * x + b * z) ** k for x in range(L) for z in range(N)) * sum(y ** q for y in range(M))
                    tot += abs(W[p][d] * den) * m * vmax
                worst = max(worst, int(tot))
    assert worst.bit_length() + 1 <= info.bits_moment


def test_plan_rejects_bad_requests(lib):
    d3 = (ctypes.c_int64 * 3)
    assert plan(lib, (0, 4, 4), 2, 3)[0] == -1           # empty dimension
    assert plan(lib, (4, 4, 4), 3, 3)[0] == -1           # unknown dtype
    assert plan(lib, (4, 4, 4), 2, 17)[0] == -1          # order above 16
    assert plan(lib, (1 << 25, 4, 4), 2, 3)[0] == -2     # beyond the exact range
    assert lib.dpm_workspace_bytes(d3(4, 4, 4), 2, -1) == 0


def test_null_arguments_fail_before_device_work(lib):
    from paper_2012_08099_amd import _lib
    d3 = (ctypes.c_int64 * 3)(4, 4, 4)
    out = _lib.Out()
    assert lib.dpm_moments(None, d3, 2, 3, ctypes.byref(out)) == -1
    assert lib.dpm_moments_async(None, d3, 2, 3, ctypes.byref(out), None, 0, None) == -1
    assert lib.dpm_project_images(None, d3, 2, 3, None, None) == -1
    assert lib.dpm_profile_collect(None) == -1
    assert lib.dpm_recomb_weight(3, 4, 0, None, None) == -1
    assert lib.dpm_strerror(-2).decode().startswith("volume or order")


def test_batched_workspace_rejects_bad_rois(lib):
    from paper_2012_08099_amd import _lib
    rois = (_lib.Roi * 2)()
    rois[0].dims[:] = [8, 8, 8]
    rois[0].dtype = 2
    rois[1].dims[:] = [8, 0, 8]
    rois[1].dtype = 2
    assert lib.dpm_batched_workspace_bytes(rois, 2, 4) == 0
    rois[1].dims[:] = [8, 5, 8]
    assert lib.dpm_batched_workspace_bytes(rois, 2, 4) > 0
    assert lib.dpm_batched_workspace_bytes(rois, 2, 7) == 0   # batched path: orders <= 6


def _rois(shapes):
    """ROI descriptors for (L, M, N, dtype) tuples, packed one after the other."""
    from paper_2012_08099_amd import _lib
    rois = (_lib.Roi * len(shapes))()
    off = 0
    for i, (L, M, N, dt) in enumerate(shapes):
        rois[i].offset_bytes = off
        rois[i].dims[:] = [L, M, N]
        rois[i].dtype = dt
        off += L * M * N * dt
    return rois


def test_batched_plan_takes_the_fused_kernel_when_blocks_fit(lib, monkeypatch):
    """Small ROIs go to the fused kernel (rows kept in LDS: no row buffer in the
    workspace); DPM_BATCH_FUSED=0 restores the separate kernels and their row buffer; in a
    batch with a block beyond the fused kernel's LDS, only that ROI keeps the separate
    kernels and its rows."""
    small = _rois([(20, 33, 17, 1), (96, 96, 96, 1), (40, 5, 21, 2)])
    monkeypatch.setenv("DPM_BATCH_FUSED", "1")
    fused = lib.dpm_batched_workspace_bytes(small, 3, 4)
    monkeypatch.setenv("DPM_BATCH_FUSED", "0")
    separate = lib.dpm_batched_workspace_bytes(small, 3, 4)
    # the separate kernels' row buffer: at least one int32 per voxel row of every slice
    assert fused > 0 and separate - fused >= 4 * (33 * 17 + 96 * 96 + 5 * 21)
    wide = _rois([(20, 33, 17, 1), (4000, 3, 9, 1)])  # one 4000-voxel row side per slice
    alone = _rois([(4000, 3, 9, 1)])
    monkeypatch.setenv("DPM_BATCH_FUSED", "1")
    a, w1 = lib.dpm_batched_workspace_bytes(wide, 2, 6), lib.dpm_batched_workspace_bytes(alone, 1, 6)
    monkeypatch.setenv("DPM_BATCH_FUSED", "0")
    b, w0 = lib.dpm_batched_workspace_bytes(wide, 2, 6), lib.dpm_batched_workspace_bytes(alone, 1, 6)
    assert w1 == w0 > 0                       # the wide ROI alone: separate kernels either way
    assert 0 < a < b                           # the small one drops its rows in the mixed batch
    assert b - a >= 4 * 33 * 17                # at least one int32 per voxel row of its slices


def test_batch_tuning_routes_and_validates(lib, monkeypatch):
    """dpm_batch_tune_set: fused = -1 sends an order's batches to the separate kernels (their
    row buffer shows in the workspace, as with DPM_BATCH_FUSED=0), other orders keep the
    planner's routing, NULL restores it, and values outside the documented ranges are
    refused."""
    from paper_2012_08099_amd import _lib
    monkeypatch.delenv("DPM_BATCH_FUSED", raising=False)
    small = _rois([(20, 33, 17, 1), (96, 96, 96, 1), (40, 5, 21, 2)])
    fused4, fused3 = lib.dpm_batched_workspace_bytes(small, 3, 4), lib.dpm_batched_workspace_bytes(small, 3, 3)
    monkeypatch.setenv("DPM_BATCH_FUSED", "0")
    separate4 = lib.dpm_batched_workspace_bytes(small, 3, 4)
    monkeypatch.delenv("DPM_BATCH_FUSED")
    try:
        assert lib.dpm_batch_tune_set(4, ctypes.byref(_lib.BatchTuning(-1, 0, 0))) == 0
        assert lib.dpm_batched_workspace_bytes(small, 3, 4) == separate4 > fused4
        assert lib.dpm_batched_workspace_bytes(small, 3, 3) == fused3
        # the geometry knobs keep the fused routing (slices per wave live in LDS, not the workspace)
        assert lib.dpm_batch_tune_set(4, ctypes.byref(_lib.BatchTuning(0, 4, 2))) == 0
        assert lib.dpm_batched_workspace_bytes(small, 3, 4) == fused4
        assert lib.dpm_batch_tune_set(4, None) == 0
        assert lib.dpm_batched_workspace_bytes(small, 3, 4) == fused4
        for order, bad in ((7, _lib.BatchTuning(0, 0, 0)), (-1, _lib.BatchTuning(0, 0, 0)),
                           (4, _lib.BatchTuning(1, 0, 0)), (4, _lib.BatchTuning(-2, 0, 0)),
                           (4, _lib.BatchTuning(0, 17, 0)), (4, _lib.BatchTuning(0, -1, 0)),
                           (4, _lib.BatchTuning(0, 0, 3)), (4, _lib.BatchTuning(0, 0, 8))):
            assert lib.dpm_batch_tune_set(order, ctypes.byref(bad)) == -1
        for good in (_lib.BatchTuning(0, 1, 1), _lib.BatchTuning(0, 16, 4), _lib.BatchTuning(-1, 0, 2)):
            assert lib.dpm_batch_tune_set(6, ctypes.byref(good)) == 0
    finally:
        for k in range(7):
            lib.dpm_batch_tune_set(k, None)


def test_tuning_overrides_change_the_plan_only(lib):
    """dpm_tune_set: a per-shape override of the work split shows in dpm_plan (z-splits,
    power tiles) and is removed by t=NULL / dpm_tune_clear; bad values are refused."""
    from paper_2012_08099_amd import _lib
    d3 = (ctypes.c_int64 * 3)
    dims = (96, 64, 256)
    rc, base = plan(lib, dims, 2, 6)
    assert rc == 0
    t = _lib.Tuning(4, 4)
    assert lib.dpm_tune_set(d3(*dims), 2, 6, ctypes.byref(t)) == 0
    rc, tuned = plan(lib, dims, 2, 6)
    assert rc == 0 and tuned.z_splits == 4 and tuned.n_items == 64 * 4
    assert tuned.power_chunk == 4 and tuned.power_tiles > base.power_tiles
    assert lib.dpm_workspace_bytes(d3(*dims), 2, 6) == tuned.workspace
    # another order or dtype of the same dims is not affected
    assert plan(lib, dims, 2, 5)[1].z_splits == base.z_splits
    assert plan(lib, dims, 1, 6)[1].z_splits == base.z_splits
    t.power_chunk = -1  # whole rows: one tile per block of 16 items per slot
    assert lib.dpm_tune_set(d3(*dims), 2, 6, ctypes.byref(t)) == 0
    rc, whole = plan(lib, dims, 2, 6)
    assert whole.power_chunk == 0 and whole.power_tiles < tuned.power_tiles
    assert lib.dpm_tune_set(d3(*dims), 2, 6, None) == 0
    rc, again = plan(lib, dims, 2, 6)
    assert (again.z_splits, again.power_tiles, again.workspace) == (base.z_splits, base.power_tiles, base.workspace)
    assert lib.dpm_tune_set(d3(*dims), 2, 6, ctypes.byref(_lib.Tuning(2, 0))) == 0
    assert lib.dpm_tune_clear() == 0
    assert plan(lib, dims, 2, 6)[1].z_splits == base.z_splits
    # waves per projection workgroup: whole-row shapes only
    fast = (128, 64, 256)
    assert plan(lib, fast, 2, 6)[1].proj_waves == 8
    assert lib.dpm_tune_set(d3(*fast), 2, 6, ctypes.byref(_lib.Tuning(0, 0, 4))) == 0
    assert plan(lib, fast, 2, 6)[1].proj_waves == 4
    assert lib.dpm_tune_set(d3(*fast), 2, 6, ctypes.byref(_lib.Tuning(0, 0, 8))) == 0
    assert plan(lib, fast, 2, 6)[1].proj_waves == 8
    assert lib.dpm_tune_set(d3(*fast), 2, 6, None) == 0
    assert plan(lib, fast, 2, 6)[1].proj_waves == 8
    for bad in (_lib.Tuning(-1, 0), _lib.Tuning(5000, 0), _lib.Tuning(1, -2), _lib.Tuning(1, 5000),
                _lib.Tuning(1, 0, 5)):
        assert lib.dpm_tune_set(d3(*dims), 2, 6, ctypes.byref(bad)) == -1
    assert lib.dpm_tune_set(d3(0, 4, 4), 2, 6, ctypes.byref(t)) == -1
    assert lib.dpm_tune_set(d3(*dims), 2, 17, ctypes.byref(t)) == -1


def test_tuning_cache_round_trip(lib, tmp_path):
    """autotune.save / load: the JSON cache installs the stored overrides."""
    from paper_2012_08099_amd import autotune
    path = str(tmp_path / "tune.json")
    autotune.save([{"key": "96x64x256:2:6", "best": {"z_splits": 2, "power_chunk": 16, "ms": 0.1}}], path)
    autotune.save([{"key": "40x40x40:1:4", "best": {"z_splits": 1, "power_chunk": -1, "ms": 0.01}}], path)
    try:
        assert autotune.load(path) == 2
        rc, info = plan(lib, (96, 64, 256), 2, 6)
        assert info.z_splits == 2 and info.power_chunk == 16
        rc, info = plan(lib, (40, 40, 40), 1, 4)
        assert info.z_splits == 1 and info.power_chunk == 0
    finally:
        autotune.clear()
