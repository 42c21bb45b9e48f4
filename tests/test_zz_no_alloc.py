"""The allocation-free entry point dpm_moments_noalloc, through the C ABI, against the
entry point it varies (dpm_moments_async with a caller workspace) and the oracle: two
calls in a row on the same fixed scratch array, the second with a smaller input, on
both power-sum paths; a request beyond the array is refused with the size it needs."""
import ctypes
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


def _outs(dpm, K):
    import torch
    nm, nm4 = dpm.num_moments(K), dpm.num_moments(min(K, 4))
    return (torch.full((nm4, 2), -7, dtype=torch.int64, device="cuda:0"),
            torch.full((nm,), -7.0, dtype=torch.float64, device="cuda:0"))


def _noalloc_vs_async(dpm, V, K):
    import torch
    vol = to_dev(V)
    code = 1 if V.dtype == np.uint8 else 2
    ws = torch.empty(dpm.workspace_bytes(vol.shape, code, K), dtype=torch.uint8, device="cuda:0")
    ex_a, fp_a = _outs(dpm, K)
    dpm.moments_async(vol, K, ex_a, fp_a, ws)
    ex_n, fp_n = _outs(dpm, K)
    need = dpm.moments_noalloc(vol, K, ex_n, fp_n)
    torch.cuda.synchronize()
    assert 0 < need <= dpm.lib().dpm_noalloc_scratch_bytes()
    assert torch.equal(ex_n, ex_a), "exact moments differ from dpm_moments_async"
    assert torch.equal(fp_n.view(torch.int64), fp_a.view(torch.int64)), "fp64 bits differ"
    got = dpm.Moments(K, dpm._exact_from_tensor(ex_n), fp_n.cpu().numpy())
    assert_moments_equal(got, oracle.moments_exact(V, K), K, f"noalloc {V.shape} K={K}")
    return need


@pytest.mark.parametrize("env", [{}, {"DPM_NO_MFMA": "1"}])
def test_noalloc_two_calls_second_smaller(dpm, monkeypatch, env):
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    big = synth.uniform_volume((80, 40, 136), np.uint16, seed=11)
    small = synth.uniform_volume((9, 7, 21), np.uint8, seed=12)
    say("noalloc", env, big.shape, "then", small.shape)
    n1 = _noalloc_vs_async(dpm, big, 6)
    n2 = _noalloc_vs_async(dpm, small, 4)
    assert n2 < n1


def test_noalloc_refuses_beyond_its_array(dpm):
    """512^3 uint16 at order 16 needs more than the fixed array: DPM_ENOMEM, nothing
    enqueued, and the size it would need is reported."""
    import torch
    say("noalloc too large")
    buf = torch.zeros(16, dtype=torch.uint8, device="cuda:0")  # never read: refused first
    ex, fp = _outs(dpm, 16)
    out = dpm._lib.Out(ex.data_ptr(), fp.data_ptr())
    need = ctypes.c_size_t(0)
    rc = dpm.lib().dpm_moments_noalloc(ctypes.c_void_p(buf.data_ptr()), dpm._lib.Dims(512, 512, 512), 2, 16,
                                       ctypes.byref(out), None, ctypes.byref(need))
    assert rc == -3
    assert need.value > dpm.lib().dpm_noalloc_scratch_bytes()
    torch.cuda.synchronize()
    assert (fp == -7.0).all(), "a refused call must not write its outputs"
    # the next call still works
    V = synth.uniform_volume((8, 8, 64), np.uint16, seed=3)
    _noalloc_vs_async(dpm, V, 5)
