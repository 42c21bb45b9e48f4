"""Helpers shared by the GPU tests (device upload, exact comparison)."""
import numpy as np


def to_dev(V):
    """numpy (N, M, L) uint8/uint16 -> contiguous device tensor (uint16 carried as int16 bits)."""
    import torch
    V = np.ascontiguousarray(V)
    if V.dtype == np.uint16:
        t = torch.from_numpy(V.view(np.int16))
    else:
        t = torch.from_numpy(V)
    return t.to("cuda:0")


def assert_moments_equal(res, exact_all, K, where=""):
    """GPU result vs exact oracle list (graded order).

    Orders <= 4: bit-exact 128-bit integers.  Every order: the FP64 value must be the
    nearest double to the exact integer (Python's float(int) rounds half to even), which
    implies a relative error <= 2**-53 (far inside 1e-12).
    """
    nm4 = len(res.exact)
    assert res.exact == exact_all[:nm4], f"{where}: exact orders <= 4 differ"
    fp = res.fp64
    bad = [i for i, (g, e) in enumerate(zip(fp.tolist(), exact_all)) if g != float(e)]
    assert not bad, f"{where}: fp64 mismatch at {bad[:8]} (got {[fp[i] for i in bad[:3]]}, " \
                    f"want {[exact_all[i] for i in bad[:3]]})"
