"""Seeded synthetic volumes shaped like the paper's workloads.

The paper measures on medical volumes (a 512x512x230 brain MRI, Section 4; CT/MRI
volumes of 1-1024 MB, Section 6, Table 1).  None of those datasets is available, so
these generators stand in for them.  Every generator takes an integer seed and is
deterministic for a given numpy version.

This module holds no moment arithmetic: it only produces voxel arrays.  Volumes are
numpy arrays of shape (N, M, L) = (z, y, x), x contiguous, i.e. ``V[z][y][x]``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_volume",
    "mri_phantom",
    "ct_phantom",
    "sphere_mask",
    "roi_batch",
    "request_mix",
]


def uniform_volume(shape, dtype=np.uint8, seed=0, lo=0, hi=None):
    """i.i.d. uniform voxels in [lo, hi] (hi defaults to the dtype maximum)."""
    rng = np.random.default_rng(seed)
    info = np.iinfo(dtype)
    hi = info.max if hi is None else hi
    return rng.integers(lo, hi + 1, size=tuple(shape), dtype=np.int64).astype(dtype)


def _ellipsoid_mask(zz, yy, xx, c, a):
    return (((zz - c[0]) / a[0]) ** 2 + ((yy - c[1]) / a[1]) ** 2 + ((xx - c[2]) / a[2]) ** 2) <= 1.0


def mri_phantom(shape=(256, 256, 256), seed=0, noise_sigma=40.0, vmax=4095):
    """MRI-like uint16 phantom: 6-10 nested ellipsoids painted outer to inner.

    The outer ellipsoid spans 0.35-0.45 of each dimension (semi-axis), each next one
    is shrunk by U[0.5, 0.9] and kept inside its parent; intensities U[200, 3000];
    background 0; additive Gaussian noise N(0, sigma^2) on every voxel; rounded and
    clamped to [0, vmax].
    """
    rng = np.random.default_rng(seed)
    N, M, L = shape
    dims = np.array([N, M, L], dtype=np.float64)
    n_ell = int(rng.integers(6, 11))
    ells = []
    semi = dims * rng.uniform(0.35, 0.45, size=3)
    centre = dims / 2.0 + rng.uniform(-0.03, 0.03, size=3) * dims
    for _ in range(n_ell):
        ells.append((centre.copy(), semi.copy(), float(rng.uniform(200, 3000))))
        shrink = rng.uniform(0.5, 0.9, size=3)
        new_semi = semi * shrink
        slack = semi - new_semi
        centre = centre + rng.uniform(-0.5, 0.5, size=3) * slack
        semi = new_semi
    out = np.empty(shape, dtype=np.uint16)
    yy, xx = np.meshgrid(np.arange(M, dtype=np.float64), np.arange(L, dtype=np.float64), indexing="ij")
    for z in range(N):
        plane = np.zeros((M, L), dtype=np.float64)
        for c, a, val in ells:
            m = _ellipsoid_mask(float(z), yy, xx, c, a)
            plane[m] = val
        plane += rng.normal(0.0, noise_sigma, size=(M, L))
        out[z] = np.clip(np.rint(plane), 0, vmax).astype(np.uint16)
    return out


def ct_phantom(shape=(512, 512, 512), seed=0, vmax=4095, slab=32):
    """CT-like uint16 volume with 12-bit values.

    Air U{0..50} outside a centred body ellipsoid (semi-axes 0.45/0.35/0.45 of the
    z/y/x dimensions), tissue N(1040, 30) inside, 10-30 bone blobs (ellipsoids inside
    the body) N(2000, 200); rounded and clamped to [0, vmax].  Generated per z-slab;
    each blob is evaluated only inside its bounding box.
    """
    rng = np.random.default_rng(seed)
    N, M, L = shape
    dims = np.array([N, M, L], dtype=np.float64)
    body_c = dims / 2.0
    body_a = dims * np.array([0.45, 0.35, 0.45])
    n_bone = int(rng.integers(10, 31))
    bones = []
    for _ in range(n_bone):
        while True:
            c = body_c + rng.uniform(-1, 1, size=3) * body_a * 0.8
            if (((c - body_c) / body_a) ** 2).sum() <= 0.64:
                break
        a = dims * rng.uniform(0.02, 0.08, size=3)
        bones.append((c, a))
    out = np.empty(shape, dtype=np.uint16)
    yy = np.arange(M, dtype=np.float64)[:, None]
    xx = np.arange(L, dtype=np.float64)[None, :]
    for z0 in range(0, N, slab):
        z1 = min(N, z0 + slab)
        nz = z1 - z0
        zz = np.arange(z0, z1, dtype=np.float64)[:, None, None]
        body = _ellipsoid_mask(zz, yy[None], xx[None], body_c, body_a)
        vol = rng.integers(0, 51, size=(nz, M, L)).astype(np.float32)
        tissue = rng.normal(1040.0, 30.0, size=(nz, M, L)).astype(np.float32)
        vol = np.where(body, tissue, vol)
        bone_mask = np.zeros((nz, M, L), dtype=bool)
        for c, a in bones:
            lo = np.maximum(np.floor(c - a), [z0, 0, 0]).astype(int)
            hi = np.minimum(np.ceil(c + a) + 1, [z1, M, L]).astype(int)
            if (hi <= lo).any():
                continue
            sub = _ellipsoid_mask(np.arange(lo[0], hi[0], dtype=np.float64)[:, None, None],
                                  np.arange(lo[1], hi[1], dtype=np.float64)[None, :, None],
                                  np.arange(lo[2], hi[2], dtype=np.float64)[None, None, :], c, a)
            bone_mask[lo[0] - z0:hi[0] - z0, lo[1]:hi[1], lo[2]:hi[2]] |= sub
        bone_mask &= body
        nb = int(bone_mask.sum())
        if nb:
            vol[bone_mask] = rng.normal(2000.0, 200.0, size=nb)
        out[z0:z1] = np.clip(np.rint(vol), 0, vmax).astype(np.uint16)
    return out


def sphere_mask(shape, rng, n_min=1, n_max=5):
    """uint8 binary mask of 1-5 random (overlapping) spheres inside a box."""
    N, M, L = shape
    mind = min(shape)
    zz, yy, xx = np.meshgrid(np.arange(N), np.arange(M), np.arange(L), indexing="ij")
    out = np.zeros(shape, dtype=np.uint8)
    for _ in range(int(rng.integers(n_min, n_max + 1))):
        c = rng.uniform(0, 1, size=3) * np.array([N, M, L])
        r = rng.uniform(2.0, max(2.0, mind / 2.0))
        out[((zz - c[0]) ** 2 + (yy - c[1]) ** 2 + (xx - c[2]) ** 2) <= r * r] = 1
    return out


def roi_batch(n=1000, seed=0, dmin=8, dmax=96):
    """A batch of uint8 sphere-mask ROIs with independent dims U{dmin..dmax}.

    Returns a list of (N, M, L) arrays.
    """
    rng = np.random.default_rng(seed)
    rois = []
    for _ in range(n):
        shape = tuple(int(s) for s in rng.integers(dmin, dmax + 1, size=3))
        rois.append(sphere_mask(shape, rng))
    return rois


def request_mix(n, seed=0, rate_hz=1000.0, ct_pool=None, small=False):
    """A Poisson request stream for the served workload.

    70 % uint8 sphere ROIs with sides U{32..128}, 25 % uint16 MRI-like slabs
    256x256xZ with Z U{100..300}, 5 % 512^3 uint16 CT-like volumes drawn from a pool.
    ``small=True`` shrinks every class (for quick tests).  Returns a list of
    (arrival_time_s, kind, volume).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n):
        t += float(rng.exponential(1.0 / rate_hz))
        u = rng.uniform()
        if u < 0.70:
            lo, hi = (8, 24) if small else (32, 128)
            shape = tuple(int(s) for s in rng.integers(lo, hi + 1, size=3))
            vol = sphere_mask(shape, rng)
            kind = "roi_u8"
        elif u < 0.95:
            z = int(rng.integers(10, 30)) if small else int(rng.integers(100, 301))
            side = 32 if small else 256
            vol = mri_phantom((z, side, side), seed=int(rng.integers(0, 2**31)))
            kind = "slab_u16"
        else:
            if ct_pool is not None and len(ct_pool):
                vol = ct_pool[int(rng.integers(0, len(ct_pool)))]
            else:
                side = 48 if small else 512
                vol = ct_phantom((side, side, side), seed=int(rng.integers(0, 2**31)))
            kind = "ct_u16"
        out.append((t, kind, vol))
    return out
