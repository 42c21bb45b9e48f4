"""GPU parity at the sizes the benchmarks run: the 512^3 uint8 order-4 volume, the paper's
Table 1 volumes (128 MB - 1 GB of 1-byte voxels at orders 3 and 4, Section 6), all 969
moments of the 512^3 CT-like volume at order 16, the blocking entry point with host
outputs, and calls on two streams that share the library-owned workspace.

Every expected value comes from the oracle (the C direct sums of eq. 2 in int128, or the
stored golden written by tests/golden/make_ct512_k16.py from the oracle)."""
import ctypes
import json
import os
import sys

import numpy as np
import pytest

import oracle
import oracle.native as onative
import synth
from gpu_util import assert_moments_equal, to_dev

pytestmark = pytest.mark.gpu

# (MB, (N, M, L)): the sizes of the paper's Table 1 from 128 MB up (1-byte voxels),
# shaped as bench.py's table1_sweep shapes them
TABLE1_BIG = [(128, (512, 512, 512)), (256, (512, 512, 1024)), (512, (512, 1024, 1024)),
              (1024, (1024, 1024, 1024))]


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


def test_u8_512_order4_bench_input(dpm):
    """The u8_512_k4 bench volume (uniform random bytes, seed 0), every moment."""
    say("u8 512^3 K=4")
    V = synth.uniform_volume((512, 512, 512), np.uint8, seed=0)
    res = dpm.moments(to_dev(V), 4)
    assert_moments_equal(res, onative.moments_hoisted(V, 4), 4, "u8 512^3 K=4")


@pytest.mark.parametrize("mb,shape", TABLE1_BIG)
def test_table1_sizes_orders_3_and_4(dpm, mb, shape):
    """The paper's Table 1 volume sizes at both of its orders, against the exact direct
    sums (the volumes bench.py's table1_sweep times: uniform bytes seeded by the size)."""
    import torch
    say("table1", mb, "MB", shape)
    V = np.random.default_rng(mb).integers(0, 256, size=shape, dtype=np.uint8)
    vol = torch.from_numpy(V).to("cuda:0")
    for K in (3, 4):
        ref = onative.moments_hoisted(V, K)
        res = dpm.moments(vol, K)
        assert_moments_equal(res, ref, K, f"table1 {mb} MB K={K}")
        say("  K", K, "ok")
    del vol
    torch.cuda.empty_cache()


def test_ct_512_order16_golden_all(dpm):
    """All 969 moments of the 512^3 CT-like bench volume at order 16 (three direction
    groups in one launch) against the oracle's stored values."""
    say("ct 512^3 K=16 golden (all)")
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ct512_k16_seed0.json")) as fh:
        g = json.load(fh)
    assert len(g["moments"]) == 969
    V = synth.ct_phantom(tuple(g["volume"]["shape_zyx"]), seed=g["volume"]["seed"])
    res = dpm.moments(to_dev(V), 16)
    exact = [0] * 969
    for p, q, r, v in g["moments"]:
        exact[dpm.moment_index(p, q, r)] = int(v)
    assert_moments_equal(res, exact, 16, "ct512 K=16")


@pytest.mark.parametrize("shape,dt,K", [((40, 24, 72), np.uint16, 4), ((33, 17, 64), np.uint8, 16),
                                        ((64, 64, 64), np.uint8, 3)])
def test_blocking_dpm_moments_host_outputs(dpm, shape, dt, K):
    """dpm_moments: the blocking entry point, results in host memory, through the C ABI."""
    say("blocking dpm_moments", shape, dt.__name__, K)
    V = synth.uniform_volume(shape, dt, seed=K + shape[0])
    vol = to_dev(V)
    nm, nm4 = dpm.num_moments(K), dpm.num_moments(min(K, 4))
    ex = np.zeros((nm4, 2), dtype=np.int64)
    fp = np.zeros(nm, dtype=np.float64)
    out = dpm._lib.Out(ex.ctypes.data, fp.ctypes.data)
    code = 1 if dt == np.uint8 else 2
    rc = dpm.lib().dpm_moments(ctypes.c_void_p(vol.data_ptr()), dpm._lib.Dims(shape[2], shape[1], shape[0]),
                               code, K, ctypes.byref(out))
    assert rc == 0
    exact = [int(lo) & (2 ** 64 - 1) | (int(hi) << 64) for lo, hi in ex.tolist()]
    assert_moments_equal(dpm.Moments(K, exact, fp), oracle.moments_exact(V, K), K, "dpm_moments")
    # exact or fp64 alone
    fp2 = np.zeros(nm, dtype=np.float64)
    out = dpm._lib.Out(None, fp2.ctypes.data)
    assert dpm.lib().dpm_moments(ctypes.c_void_p(vol.data_ptr()), dpm._lib.Dims(shape[2], shape[1], shape[0]),
                                 code, K, ctypes.byref(out)) == 0
    assert np.array_equal(fp2, fp)


def test_shared_workspace_on_two_streams(dpm):
    """Calls without a workspace of their own on two non-blocking streams (and a blocking
    call on the default stream between them) share the library-owned workspace; the
    library orders them on the device, so every result is exact."""
    import torch
    say("shared workspace, two streams")
    K = 6
    vols = [synth.uniform_volume((96, 40, 160), np.uint16, seed=s) for s in range(4)]
    refs = [oracle.moments_exact(V, K) for V in vols]
    dev = [to_dev(V) for V in vols]
    nm, nm4 = dpm.num_moments(K), dpm.num_moments(4)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rnd in range(3):
        outs = []
        for i, v in enumerate(dev):
            ex = torch.zeros((nm4, 2), dtype=torch.int64, device="cuda:0")
            fp = torch.zeros(nm, dtype=torch.float64, device="cuda:0")
            s = streams[i % 2]
            s.wait_stream(torch.cuda.current_stream())
            dpm.moments_async(v, K, ex, fp, None, stream=s)
            outs.append((ex, fp))
            if i == 1:
                # a blocking call (library-owned workspace, default stream) in between
                hex_ = np.zeros((nm4, 2), dtype=np.int64)
                hfp = np.zeros(nm, dtype=np.float64)
                out = dpm._lib.Out(hex_.ctypes.data, hfp.ctypes.data)
                assert dpm.lib().dpm_moments(ctypes.c_void_p(dev[3].data_ptr()), dpm._lib.Dims(160, 40, 96), 2, K,
                                             ctypes.byref(out)) == 0
                exact = [int(lo) & (2 ** 64 - 1) | (int(hi) << 64) for lo, hi in hex_.tolist()]
                assert_moments_equal(dpm.Moments(K, exact, hfp), refs[3], K, "blocking in between")
        torch.cuda.synchronize()
        for i, (ex, fp) in enumerate(outs):
            got = dpm.Moments(K, dpm._exact_from_tensor(ex), fp.cpu().numpy())
            assert_moments_equal(got, refs[i], K, f"round {rnd} volume {i}")
    # images on a side stream, then features on the default stream
    s = streams[0]
    s.wait_stream(torch.cuda.current_stream())
    imgs = dpm.project_images(dev[0], K, stream=s)
    f = dpm.features(dev[1], K)
    torch.cuda.synchronize()
    a, b = dpm.direction(3)
    assert np.array_equal(imgs[3].cpu().numpy().astype(np.int64), oracle.projection_image(vols[0], a, b))
    ref_f = oracle.features(refs[1], K)
    assert np.allclose(f["mu"], ref_f["mu"], rtol=1e-13, atol=0)
