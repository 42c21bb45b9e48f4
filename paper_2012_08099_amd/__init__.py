"""3D geometric moments on MI355X with the Discrete Projection Moment method.

Diggin & Diggin, "Fast 3D Image Moments" (arXiv 2012.08099).  The moments
M_pqr = sum V(x,y,z) x^p y^q z^r (Section 1, eq. 2) of a uint8/uint16 volume are
computed by HIP kernels for gfx950 behind the C ABI of ``include/dpm.h``; this module
only marshals arguments (torch supplies device memory and streams).

Volumes are torch tensors of shape (N, M, L) = (z, y, x) on a ROCm device, dtype
torch.uint8 or torch.uint16, contiguous.  Moments come in graded order (p+q+r
ascending, then p descending, then q descending); see ``moment_list``.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import DpmError, Dims, I128, Out, PlanInfo, Roi, check, lib

__all__ = [
    "DpmError", "Moments", "moment_list", "num_moments", "moment_index", "direction", "image_width",
    "workspace_bytes", "plan", "moments", "moments_async", "project_images", "moments_batched",
    "batched_workspace_bytes", "pack_rois", "recomb_weight", "release", "profile_enable",
    "profile_collect",
]

KMAX = 16


def moment_list(K):
    """(p, q, r) in graded order for p+q+r <= K."""
    out = []
    for n in range(K + 1):
        for p in range(n, -1, -1):
            for q in range(n - p, -1, -1):
                out.append((p, q, n - p - q))
    return out


def num_moments(K):
    return int(lib().dpm_num_moments(int(K)))


def moment_index(p, q, r):
    return int(lib().dpm_moment_index(p, q, r))


def direction(d):
    a, b = ctypes.c_int(), ctypes.c_int()
    check(lib().dpm_direction(d, ctypes.byref(a), ctypes.byref(b)), "dpm_direction")
    return a.value, b.value


def _dims_of_shape(shape):
    N, M, L = (int(s) for s in shape)
    return Dims(L, M, N)


def image_width(shape, d):
    return int(lib().dpm_image_width(_dims_of_shape(shape), d))


def _dtype_code(t):
    import torch
    if t.dtype == torch.uint8:
        return _lib.DPM_U8
    if t.dtype in (torch.uint16, torch.int16):
        return _lib.DPM_U16
    raise TypeError(f"unsupported volume dtype {t.dtype}; use torch.uint8 or torch.uint16")


def _check_volume(vol):
    if not vol.is_cuda:
        raise ValueError("volume must be a device (ROCm) tensor")
    if vol.dim() != 3:
        raise ValueError("volume must have shape (N, M, L) = (z, y, x)")
    if not vol.is_contiguous():
        raise ValueError("volume must be contiguous")


def workspace_bytes(shape, dtype_code, K):
    return int(lib().dpm_workspace_bytes(_dims_of_shape(shape), dtype_code, K))


def plan(shape, dtype_code, K):
    info = PlanInfo()
    check(lib().dpm_plan(_dims_of_shape(shape), dtype_code, K, ctypes.byref(info)), "dpm_plan")
    return {f: getattr(info, f) for f, _ in PlanInfo._fields_}


def i128_to_int(lo, hi):
    return int(lo) | (int(hi) << 64)


@dataclass
class Moments:
    """Result of one volume: ``exact`` = orders <= min(K, 4) as Python ints; ``fp64`` =
    every order as float64 (nearest to the exact integer)."""
    K: int
    exact: list
    fp64: np.ndarray

    def as_dict(self):
        return dict(zip(moment_list(self.K), self.fp64.tolist()))


def _exact_from_tensor(ex):
    a = ex.view(-1, 2).cpu().numpy()
    return [int(lo) | (int(hi) << 64) for lo, hi in zip(a[:, 0].astype(np.uint64).tolist(),
                                                       a[:, 1].astype(np.int64).tolist())]


def moments(vol, K, stream=None):
    """Moments of one volume (blocking).  Returns ``Moments``."""
    import torch
    _check_volume(vol)
    nm, nm4 = num_moments(K), num_moments(min(K, 4))
    if nm < 0:
        raise ValueError("max_order must be in [0, 16]")
    dev = vol.device
    ex = torch.empty((nm4, 2), dtype=torch.int64, device=dev)
    fp = torch.empty(nm, dtype=torch.float64, device=dev)
    ws_n = workspace_bytes(vol.shape, _dtype_code(vol), K)
    if ws_n == 0:
        check(-2, "dpm_workspace_bytes")
    ws = torch.empty(ws_n, dtype=torch.uint8, device=dev)
    moments_async(vol, K, ex, fp, ws, stream)
    (stream or torch.cuda.current_stream(dev)).synchronize()
    return Moments(K, _exact_from_tensor(ex), fp.cpu().numpy())


def moments_async(vol, K, out_exact, out_fp64, workspace, stream=None):
    """Enqueue on ``stream`` (default: current).  Outputs/workspace are device tensors."""
    import torch
    _check_volume(vol)
    st = stream if stream is not None else torch.cuda.current_stream(vol.device)
    out = Out(out_exact.data_ptr() if out_exact is not None else None,
              out_fp64.data_ptr() if out_fp64 is not None else None)
    rc = lib().dpm_moments_async(ctypes.c_void_p(vol.data_ptr()), _dims_of_shape(vol.shape), _dtype_code(vol),
                                 int(K), ctypes.byref(out),
                                 ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None,
                                 workspace.numel() * workspace.element_size() if workspace is not None else 0,
                                 ctypes.c_void_p(st.cuda_stream))
    check(rc, "dpm_moments_async")


def moments_noalloc(vol, K, out_exact, out_fp64, stream=None):
    """``moments_async`` without a workspace and without any allocation: the library's
    fixed per-GPU scratch array holds the workspace (calls that overlap on one GPU race).
    Returns the scratch bytes the request used."""
    import torch
    _check_volume(vol)
    st = stream if stream is not None else torch.cuda.current_stream(vol.device)
    out = Out(out_exact.data_ptr() if out_exact is not None else None,
              out_fp64.data_ptr() if out_fp64 is not None else None)
    need = ctypes.c_size_t(0)
    rc = lib().dpm_moments_noalloc(ctypes.c_void_p(vol.data_ptr()), _dims_of_shape(vol.shape), _dtype_code(vol),
                                   int(K), ctypes.byref(out), ctypes.c_void_p(st.cuda_stream), ctypes.byref(need))
    check(rc, "dpm_moments_noalloc")
    return int(need.value)


def paper_workspace_bytes(shape, dtype_code, K):
    """Workspace of the paper's own route (five images, 1D integrals, eqs. 10-16)."""
    return int(lib().dpm_paper_workspace_bytes(_dims_of_shape(shape), int(dtype_code), int(K)))


def _paper_ws(vol, K):
    import torch
    n = paper_workspace_bytes(vol.shape, _dtype_code(vol), K)
    if n == 0:
        check(-5 if K > 4 else -2, "dpm_paper_workspace_bytes")
    return torch.empty(n, dtype=torch.uint8, device=vol.device)


def paper_image_shapes(shape, K):
    """(rows, columns) of the paper's images XY, YZ, ZX, X+Z, X-Z needed for order K."""
    N, M, L = (int(s) for s in shape)
    shapes = [(M, L), (N, M), (L, N), (M, L + N - 1), (M, L + N - 1)]
    return shapes[:3 if K <= 2 else K + 1]


def paper_images(vol, K, stream=None):
    """The paper's images (XY, YZ, ZX, X+Z, X-Z as needed for order K) as int32 device
    tensors img[j][i], formed by one pass over the volume."""
    import torch
    _check_volume(vol)
    shapes = paper_image_shapes(vol.shape, K)
    buf = torch.empty(sum(h * w for h, w in shapes), dtype=torch.int32, device=vol.device)
    ws = _paper_ws(vol, K)
    st = stream if stream is not None else torch.cuda.current_stream(vol.device)
    if stream is not None:
        stream.wait_stream(torch.cuda.current_stream(vol.device))
    rc = lib().dpm_paper_images(ctypes.c_void_p(vol.data_ptr()), _dims_of_shape(vol.shape), _dtype_code(vol), int(K),
                                ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                ctypes.c_void_p(st.cuda_stream))
    check(rc, "dpm_paper_images")
    out, off = [], 0
    for h, w in shapes:
        out.append(buf[off:off + h * w].view(h, w))
        off += h * w
    st.synchronize()
    return out


def moments_paper_async(vol, K, out_exact, out_fp64, workspace, stream=None):
    """The paper's route, enqueued on ``stream``; outputs and workspace are device tensors."""
    import torch
    _check_volume(vol)
    st = stream if stream is not None else torch.cuda.current_stream(vol.device)
    out = Out(out_exact.data_ptr() if out_exact is not None else None,
              out_fp64.data_ptr() if out_fp64 is not None else None)
    rc = lib().dpm_moments_paper(ctypes.c_void_p(vol.data_ptr()), _dims_of_shape(vol.shape), _dtype_code(vol), int(K),
                                 ctypes.byref(out), ctypes.c_void_p(workspace.data_ptr()),
                                 workspace.numel() * workspace.element_size(), ctypes.c_void_p(st.cuda_stream))
    check(rc, "dpm_moments_paper")


def moments_paper(vol, K):
    """Moments of order <= K (<= 4) by the paper's route (blocking).  Returns ``Moments``."""
    import torch
    nm = num_moments(K)
    ex = torch.empty((nm, 2), dtype=torch.int64, device=vol.device)
    fp = torch.empty(nm, dtype=torch.float64, device=vol.device)
    moments_paper_async(vol, K, ex, fp, _paper_ws(vol, K))
    torch.cuda.current_stream(vol.device).synchronize()
    return Moments(K, _exact_from_tensor(ex), fp.cpu().numpy())


def drt_workspace_bytes(shape, dtype_code, K):
    return int(lib().dpm_drt_workspace_bytes(_dims_of_shape(shape), int(dtype_code), int(K)))


def moments_drt_async(vol, K, out_exact, out_fp64, workspace, stream=None):
    """The default images with 2D moments by the 1D integrals of Section 5 (orders <= 4)."""
    import torch
    _check_volume(vol)
    st = stream if stream is not None else torch.cuda.current_stream(vol.device)
    out = Out(out_exact.data_ptr() if out_exact is not None else None,
              out_fp64.data_ptr() if out_fp64 is not None else None)
    rc = lib().dpm_moments_drt(ctypes.c_void_p(vol.data_ptr()), _dims_of_shape(vol.shape), _dtype_code(vol), int(K),
                               ctypes.byref(out), ctypes.c_void_p(workspace.data_ptr()),
                               workspace.numel() * workspace.element_size(), ctypes.c_void_p(st.cuda_stream))
    check(rc, "dpm_moments_drt")


def moments_drt(vol, K):
    import torch
    _check_volume(vol)
    n = drt_workspace_bytes(vol.shape, _dtype_code(vol), K)
    if n == 0:
        check(-5 if K > 4 else -2, "dpm_drt_workspace_bytes")
    ws = torch.empty(n, dtype=torch.uint8, device=vol.device)
    nm, nm4 = num_moments(K), num_moments(min(K, 4))
    ex = torch.empty((nm4, 2), dtype=torch.int64, device=vol.device)
    fp = torch.empty(nm, dtype=torch.float64, device=vol.device)
    moments_drt_async(vol, K, ex, fp, ws)
    torch.cuda.current_stream(vol.device).synchronize()
    return Moments(K, _exact_from_tensor(ex), fp.cpu().numpy())


def moments_from_images(images, shape, dtype_code, K):
    """Moments from the K+1 projection images of a (N, M, L) = ``shape`` volume (blocking).
    ``images``: one contiguous int32 device tensor in the layout of ``project_images``."""
    import torch
    if not images.is_cuda or images.dtype != torch.int32 or not images.is_contiguous():
        raise ValueError("images must be a contiguous int32 device tensor")
    nm, nm4 = num_moments(K), num_moments(min(K, 4))
    if nm < 0:
        raise ValueError("max_order must be in [0, 16]")
    ex = np.zeros((nm4, 2), dtype=np.int64)
    fp = np.zeros(nm, dtype=np.float64)
    out = Out(ex.ctypes.data, fp.ctypes.data)
    check(lib().dpm_moments_from_images(ctypes.c_void_p(images.data_ptr()), _dims_of_shape(shape), int(dtype_code),
                                        int(K), ctypes.byref(out)), "dpm_moments_from_images")
    exact = [int(lo) | (int(hi) << 64) for lo, hi in zip(ex[:, 0].astype(np.uint64).tolist(), ex[:, 1].tolist())]
    return Moments(K, exact, fp)


def features(vol, K, spacing=None):
    """Centroid, central moments mu, normalised eta and spacing-scaled mu' of a device
    volume for orders <= K (blocking).  Returns a dict of numpy arrays in graded order."""
    _check_volume(vol)
    nm = num_moments(K)
    if nm < 0:
        raise ValueError("max_order must be in [0, 16]")
    mu, eta, mup = (np.empty(nm, dtype=np.float64) for _ in range(3))
    out = _lib.FeaturesOut()
    out.mu, out.eta, out.mu_phys = mu.ctypes.data, eta.ctypes.data, mup.ctypes.data
    sp = (ctypes.c_double * 3)(*spacing) if spacing is not None else None
    check(lib().dpm_features(ctypes.c_void_p(vol.data_ptr()), _dims_of_shape(vol.shape), _dtype_code(vol), int(K),
                             sp, ctypes.byref(out)), "dpm_features")
    return {"centroid": np.array(out.centroid[:]), "mu": mu, "eta": eta, "mu_phys": mup}


def project_images(vol, K, stream=None):
    """The K+1 projection images as a list of int32 device tensors of shape (M, W_d)."""
    import torch
    _check_volume(vol)
    N, M, L = vol.shape
    widths = [image_width(vol.shape, d) for d in range(K + 1)]
    buf = torch.zeros(sum(w * M for w in widths), dtype=torch.int32, device=vol.device)
    st = stream if stream is not None else torch.cuda.current_stream(vol.device)
    if stream is not None:
        stream.wait_stream(torch.cuda.current_stream(vol.device))  # the zero fill above
    rc = lib().dpm_project_images(ctypes.c_void_p(vol.data_ptr()), _dims_of_shape(vol.shape), _dtype_code(vol),
                                  int(K), ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(st.cuda_stream))
    check(rc, "dpm_project_images")
    out, off = [], 0
    for w in widths:
        out.append(buf[off:off + w * M].view(M, w))
        off += w * M
    return out


def pack_rois(volumes, device, align=16):
    """Pack a list of numpy (N, M, L) uint8/uint16 arrays into one device buffer.

    Returns (packed uint8 tensor, ctypes array of Roi descriptors)."""
    import torch
    offs, total = [], 0
    for v in volumes:
        total = (total + align - 1) // align * align
        offs.append(total)
        total += v.nbytes
    host = np.zeros(max(total, 1), dtype=np.uint8)
    rois = (Roi * len(volumes))()
    for i, (v, o) in enumerate(zip(volumes, offs)):
        v = np.ascontiguousarray(v)
        host[o:o + v.nbytes] = v.view(np.uint8).reshape(-1)
        N, M, L = v.shape
        rois[i].offset_bytes = o
        rois[i].dims[0], rois[i].dims[1], rois[i].dims[2] = L, M, N
        rois[i].dtype = _lib.DPM_U8 if v.dtype == np.uint8 else _lib.DPM_U16
    return torch.from_numpy(host).to(device), rois


def batched_workspace_bytes(rois, K):
    return int(lib().dpm_batched_workspace_bytes(rois, len(rois), int(K)))


def moments_batched(packed, rois, K, out_exact, out_fp64, workspace, stream=None):
    """All ROIs in one launch sequence; outputs are device tensors of n_rois blocks."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(packed.device)
    out = Out(out_exact.data_ptr() if out_exact is not None else None,
              out_fp64.data_ptr() if out_fp64 is not None else None)
    rc = lib().dpm_moments_batched(ctypes.c_void_p(packed.data_ptr()), rois, len(rois), int(K),
                                   ctypes.byref(out), ctypes.c_void_p(workspace.data_ptr()),
                                   workspace.numel() * workspace.element_size(),
                                   ctypes.c_void_p(st.cuda_stream))
    check(rc, "dpm_moments_batched")


def batched_graph_count():
    """Graphs cached for repeated batched calls."""
    return int(lib().dpm_batched_graph_count())


def recomb_weight(k, p, d):
    n, den = ctypes.c_int64(), ctypes.c_uint64()
    check(lib().dpm_recomb_weight(k, p, d, ctypes.byref(n), ctypes.byref(den)), "dpm_recomb_weight")
    return n.value, den.value


def profile_enable(on=True):
    """Record HIP events around each stage of every following call (tracing)."""
    check(lib().dpm_profile_enable(1 if on else 0), "dpm_profile_enable")


def profile_collect():
    """Wait for the recorded events; return summed per-stage device milliseconds."""
    p = _lib.Profile()
    check(lib().dpm_profile_collect(ctypes.byref(p)), "dpm_profile_collect")
    return {"calls": p.calls, "ms_project": p.ms_project, "ms_power": p.ms_power,
            "ms_combine": p.ms_combine, "ms_total": p.ms_total}


def release():
    check(lib().dpm_release(), "dpm_release")


class Server:
    """The served loop of ``dpm_server_*`` (argument marshalling only).

    ``submit`` takes a contiguous uint8/uint16 array -- a device tensor (read in place,
    after the work queued so far on torch's current stream: an event recorded there is
    passed with the request) or a host tensor / numpy array (copied into the server's
    arena; pinned memory keeps that copy asynchronous) -- and returns a tag.  The input
    and the result arrays are kept alive here until ``poll`` has returned the request's
    completion.  ``keep=True`` keeps the request's image moments resident for
    ``requery``.
    """

    def __init__(self, hbm_budget=8 << 30, n_streams=4, batch_voxels=128 ** 3, batch_max=256,
                 max_inflight=16, device=0):
        cfg = _lib.ServerConfig(int(device), int(n_streams), int(hbm_budget), int(batch_voxels), int(batch_max),
                                int(max_inflight))
        h = ctypes.c_void_p()
        check(lib().dpm_server_create(ctypes.byref(cfg), ctypes.byref(h)), "dpm_server_create")
        self._h = h
        self._next = 1
        self._live = {}  # tag -> (input, exact, fp64, K)

    @staticmethod
    def now_ms():
        return lib().dpm_server_now_ms()

    def submit(self, vol, K, t_arrival_ms=0.0, keep=False):
        req = self._request(vol, K, t_arrival_ms, keep)
        rc = lib().dpm_server_submit(self._h, ctypes.byref(req))
        if rc:
            self._live.pop(req.tag, None)
            raise DpmError(rc, "dpm_server_submit")
        return req.tag

    def _request(self, vol, K, t_arrival_ms, keep=False):
        import numpy as np
        import torch
        if isinstance(vol, np.ndarray):
            vol = torch.from_numpy(np.ascontiguousarray(vol.view(np.int16) if vol.dtype == np.uint16 else vol))
        if not vol.is_contiguous() or vol.dim() != 3:
            raise ValueError("volume must be a contiguous 3D tensor (N, M, L)")
        exact = np.zeros((num_moments(min(K, 4)), 2), dtype=np.int64)
        fp = np.zeros(num_moments(K), dtype=np.float64)
        tag = self._next
        self._next += 1
        req = _lib.Request()
        req.data = vol.data_ptr()
        req.data_on_device = 1 if vol.is_cuda else 0
        req.dtype = _dtype_code(vol)
        req.dims[:] = [int(vol.shape[2]), int(vol.shape[1]), int(vol.shape[0])]
        req.max_order = int(K)
        req.tag = tag
        req.t_arrival_ms = float(t_arrival_ms)
        req.exact = exact.ctypes.data
        req.fp64 = fp.ctypes.data
        req.keep_resident = 1 if keep else 0
        ev = None
        if vol.is_cuda:
            # the server's stream waits for what torch has queued so far (e.g. the
            # kernel that wrote the volume)
            ev = torch.cuda.Event()
            ev.record(torch.cuda.current_stream(vol.device))
            req.ready_event = ev.cuda_event
        self._live[tag] = (vol, exact, fp, K, ev)
        return req

    def replay(self, items):
        """Submit [(vol, K, t_arrival_ms), ...] at their arrival times from a native loop
        (blocking; run it in a thread and poll meanwhile).  Returns the tags."""
        reqs = (_lib.Request * len(items))()
        tags = []
        for i, (vol, K, t) in enumerate(items):
            reqs[i] = self._request(vol, K, t)
            tags.append(reqs[i].tag)
        check(lib().dpm_server_replay(self._h, reqs, len(items)), "dpm_server_replay")
        return tags

    def poll(self, max_n=256, wait_ms=0):
        """Completed requests: list of dicts with tag, status, batched, times and the Moments."""
        buf = (_lib.Completion * max_n)()
        n = lib().dpm_server_poll(self._h, buf, max_n, int(wait_ms))
        if n < 0:
            raise DpmError(n, "dpm_server_poll")
        out = []
        for c in buf[:n]:
            vol, exact, fp, K, _ = self._live.pop(c.tag)
            ex = [i128_to_int(int(lo) & (2 ** 64 - 1), int(hi)) for lo, hi in exact.tolist()]
            out.append({"tag": c.tag, "status": c.status, "batched": bool(c.batched),
                        "t_arrival_ms": c.t_arrival_ms, "t_start_ms": c.t_start_ms, "t_done_ms": c.t_done_ms,
                        "moments": Moments(K, ex, fp)})
        return out

    def requery(self, tag, K):
        """Moments of order <= K of a completed request submitted with keep=True, from its
        resident image moments (no volume read).  Returns ``Moments``."""
        exact = np.zeros((num_moments(min(K, 4)), 2), dtype=np.int64)
        fp = np.zeros(num_moments(K), dtype=np.float64)
        check(lib().dpm_server_requery(self._h, int(tag), int(K), exact.ctypes.data, fp.ctypes.data),
              "dpm_server_requery")
        ex = [i128_to_int(int(lo) & (2 ** 64 - 1), int(hi)) for lo, hi in exact.tolist()]
        return Moments(K, ex, fp)

    def release_resident(self, tag):
        check(lib().dpm_server_release(self._h, int(tag)), "dpm_server_release")

    def stats(self):
        s = _lib.ServerStats()
        check(lib().dpm_server_stats_get(self._h, ctypes.byref(s)), "dpm_server_stats_get")
        return {f: getattr(s, f) for f, _ in s._fields_}

    def close(self):
        if self._h:
            check(lib().dpm_server_destroy(self._h), "dpm_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
