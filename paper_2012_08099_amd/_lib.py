"""ctypes binding of libdpm.so (argument marshalling only).

Every computation runs in the HIP kernels behind the C ABI of ``include/dpm.h``.
There is no CPU fallback: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpm.so")

DPM_U8 = 1
DPM_U16 = 2

STATUS = {0: "DPM_OK", -1: "DPM_EINVAL", -2: "DPM_ERANGE", -3: "DPM_ENOMEM", -4: "DPM_EDEVICE",
          -5: "DPM_ENOTSUP"}


class DpmError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = f"{where}: {STATUS.get(status, status)}"
        try:
            msg += f" ({lib().dpm_strerror(status).decode()})"
            if status == -4:
                msg += f" hipError={lib().dpm_last_device_error()}"
        except Exception:  # pragma: no cover - error while formatting an error
            pass
        super().__init__(msg)


class I128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_int64)]


class Out(ctypes.Structure):
    _fields_ = [("exact", ctypes.c_void_p), ("fp64", ctypes.c_void_p)]


class Roi(ctypes.Structure):
    _fields_ = [("offset_bytes", ctypes.c_uint64), ("dims", ctypes.c_int64 * 3),
                ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_dirs", ctypes.c_int32), ("n_groups", ctypes.c_int32), ("n_items", ctypes.c_int32),
                ("z_splits", ctypes.c_int32), ("limbs_slice", ctypes.c_int32),
                ("limbs_moment", ctypes.c_int32), ("bits_slice", ctypes.c_int32),
                ("bits_moment", ctypes.c_int32), ("lds_bytes", ctypes.c_int64),
                ("workspace", ctypes.c_int64), ("power_tiles", ctypes.c_int32),
                ("power_chunk", ctypes.c_int32), ("proj_waves", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class FeaturesOut(ctypes.Structure):
    _fields_ = [("centroid", ctypes.c_double * 3), ("mu", ctypes.c_void_p), ("eta", ctypes.c_void_p),
                ("mu_phys", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("z_splits", ctypes.c_int32), ("power_chunk", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("fused", ctypes.c_int32), ("units", ctypes.c_int32), ("max_spw", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int32), ("reserved", ctypes.c_int32), ("ms_project", ctypes.c_double),
                ("ms_power", ctypes.c_double), ("ms_combine", ctypes.c_double),
                ("ms_total", ctypes.c_double)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("n_streams", ctypes.c_int32), ("hbm_budget", ctypes.c_int64),
                ("batch_voxels", ctypes.c_int64), ("batch_max", ctypes.c_int32), ("max_inflight", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("data_on_device", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("dims", ctypes.c_int64 * 3), ("max_order", ctypes.c_int32), ("keep_resident", ctypes.c_int32),
                ("tag", ctypes.c_uint64), ("t_arrival_ms", ctypes.c_double), ("exact", ctypes.c_void_p),
                ("fp64", ctypes.c_void_p), ("ready_event", ctypes.c_void_p)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("batched", ctypes.c_int32),
                ("t_arrival_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("batched_jobs", ctypes.c_int64),
                ("single_jobs", ctypes.c_int64), ("arena_bytes", ctypes.c_int64), ("arena_peak_used", ctypes.c_int64),
                ("pending", ctypes.c_int32), ("inflight", ctypes.c_int32), ("resident", ctypes.c_int64),
                ("resident_bytes", ctypes.c_int64), ("evictions", ctypes.c_int64)]


Dims = ctypes.c_int64 * 3

# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "dpm_num_moments": (ctypes.c_int, [ctypes.c_int]),
    "dpm_moment_index": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "dpm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "dpm_last_device_error": (ctypes.c_int, []),
    "dpm_direction": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "dpm_image_width": (ctypes.c_int64, [ctypes.POINTER(ctypes.c_int64), ctypes.c_int]),
    "dpm_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int]),
    "dpm_moments": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                   ctypes.c_int, ctypes.POINTER(Out)]),
    "dpm_moments_async": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                         ctypes.c_int, ctypes.POINTER(Out), ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.c_void_p]),
    "dpm_moments_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                           ctypes.c_int, ctypes.POINTER(Out), ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "dpm_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "dpm_paper_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int]),
    "dpm_paper_images": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "dpm_moments_paper": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(Out), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "dpm_drt_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int]),
    "dpm_moments_drt": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(Out), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "dpm_project_images": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                          ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "dpm_batched_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Roi), ctypes.c_int, ctypes.c_int]),
    "dpm_moments_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Roi), ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(Out), ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_void_p]),
    "dpm_release": (ctypes.c_int, []),
    "dpm_batched_graph_count": (ctypes.c_int, []),
    "dpm_tune_set": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(Tuning)]),
    "dpm_tune_clear": (ctypes.c_int, []),
    "dpm_batch_tune_set": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(BatchTuning)]),
    "dpm_moments_from_images": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                                               ctypes.c_int, ctypes.POINTER(Out)]),
    "dpm_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.POINTER(FeaturesOut)]),
    "dpm_recomb_weight": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64)]),
    "dpm_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "dpm_profile_collect": (ctypes.c_int, [ctypes.POINTER(Profile)]),
    "dpm_plan": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(PlanInfo)]),
    "dpm_server_now_ms": (ctypes.c_double, []),
    "dpm_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]),
    "dpm_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Request)]),
    "dpm_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Completion), ctypes.c_int, ctypes.c_int]),
    "dpm_server_stats_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "dpm_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "dpm_server_replay": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Request), ctypes.c_int]),
    "dpm_server_requery": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "dpm_server_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
}

_lib = None


def lib():
    """Load libdpm.so (built in-tree by ``build.py``); raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2012_08099_amd.build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status, where):
    if status != 0:
        raise DpmError(status, where)
