"""ctypes declarations of the C ABI in include/raygs.h (argument marshalling only).

torch is imported first so that the HIP runtime it loads is the one the
library binds to (both use the soname libamdhip64.so.7).
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime before the library)

_HERE = os.path.dirname(os.path.abspath(__file__))
# RAYGS_LIBRARY may point at another build of the same ABI (e.g. for A/B timing)
LIB_PATH = os.environ.get("RAYGS_LIBRARY") or os.path.join(_HERE, "libraygs.so")

RGS_OK = 0
RGS_EINVAL = -1
RGS_EWORKSPACE = -2
RGS_EOVERFLOW = -3
RGS_EHIP = -4
RGS_ECAPTURE = -5
RGS_EUNSUPPORTED = -6
RGS_WS_BACKWARD = 1

STATUS_NAMES = {0: "RGS_OK", -1: "RGS_EINVAL", -2: "RGS_EWORKSPACE", -3: "RGS_EOVERFLOW", -4: "RGS_EHIP",
                -5: "RGS_ECAPTURE", -6: "RGS_EUNSUPPORTED"}


class Gaussians(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("n", C.c_int64), ("sh_degree", C.c_int32)]


class Camera(C.Structure):
    _fields_ = [("world_to_cam", C.c_double * 12), ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double),
                ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("p_min", C.c_double), ("alpha_max", C.c_double), ("t_eps", C.c_double), ("near_z", C.c_double),
                ("mip", C.c_int32), ("mip_sigma2_px", C.c_double), ("background", C.c_double * 3),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("divergence", C.c_int32)]


class ViewOut(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("final_T", C.c_void_p), ("n_contrib", C.c_void_p)]


class GaussianGrads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class Workspace(C.Structure):
    _fields_ = [("ptr", C.c_void_p), ("bytes", C.c_size_t), ("capacity", C.c_int64), ("flags", C.c_int32)]


class WorkspaceLayout(C.Structure):
    _fields_ = [(k, C.c_size_t) for k in ("counters", "views", "records", "depth_keys", "boxes", "bin_boxes", "conics",
                                          "tile_counts", "order", "offsets", "inst_tiles", "inst_ids", "tile_ranges",
                                          "record_grads", "total_bytes")] + [
        ("n_records", C.c_int64), ("capacity", C.c_int64), ("total_tiles", C.c_int64), ("tile_w", C.c_int32),
        ("tile_h", C.c_int32), ("tile_bits", C.c_int32), ("reserved", C.c_int32)]


EXPORTS = {
    # name: (restype, argtypes)
    "rgs_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    "rgs_destroy": (None, [C.c_void_p]),
    "rgs_last_error": (C.c_char_p, [C.c_void_p]),
    "rgs_workspace_size": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Camera), C.c_int32, C.POINTER(Options),
                                     C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]),
    "rgs_render": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.POINTER(Camera), C.c_int32, C.POINTER(Options),
                             C.POINTER(Workspace), C.POINTER(ViewOut), C.c_void_p]),
    "rgs_render_noalloc": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.POINTER(Camera), C.c_int32,
                                     C.POINTER(Options), C.POINTER(ViewOut), C.c_void_p, C.c_void_p]),
    "rgs_render_status": (C.c_int, [C.c_void_p, C.POINTER(Workspace), C.c_void_p, C.POINTER(C.c_int64)]),
    "rgs_render_backward": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.POINTER(Camera), C.c_int32,
                                      C.POINTER(Options), C.POINTER(Workspace), C.POINTER(ViewOut),
                                      C.POINTER(C.c_void_p), C.POINTER(GaussianGrads), C.c_void_p]),
    "rgs_batch_plan": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.POINTER(Camera), C.c_int32, C.POINTER(Options),
                                 C.c_int64, C.c_int32, C.POINTER(C.c_size_t), C.POINTER(C.c_void_p)]),
    "rgs_batch_launch": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.POINTER(Camera), C.POINTER(Workspace),
                                   C.POINTER(ViewOut), C.c_void_p]),
    "rgs_batch_status": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "rgs_plan_destroy": (None, [C.c_void_p]),
    "rgs_autotune": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.POINTER(Camera), C.c_int32, C.POINTER(Options),
                               C.POINTER(Workspace), C.POINTER(ViewOut), C.c_int32, C.c_void_p, C.POINTER(Options),
                               C.POINTER(C.c_double)]),
    "rgs_autotune_training": (C.c_int, [C.c_void_p, C.POINTER(Gaussians), C.POINTER(Camera), C.c_int32,
                                        C.POINTER(Options), C.POINTER(Workspace), C.POINTER(ViewOut),
                                        C.POINTER(C.c_void_p), C.POINTER(GaussianGrads), C.c_int32, C.c_void_p,
                                        C.POINTER(Options), C.POINTER(C.c_double)]),
    "rgs_get_workspace_layout": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Camera), C.c_int32, C.POINTER(Options),
                                           C.c_int64, C.c_int32, C.POINTER(WorkspaceLayout)]),
    "rgs_set_view_clocks": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32]),
    "rgs_wall_clock_hz": (C.c_double, [C.c_void_p]),
    "rgs_downsample_box": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_void_p, C.c_void_p]),
    "rgs_calibrate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rgs_set_stage_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "rgs_stage_times": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int64)]),
    "rgs_stage_names": (C.c_char_p, []),
}

_lib = None


def load(path: str = None):
    """Load libraygs.so; raises (never falls back) when it is missing."""
    global _lib
    if path is None:
        if _lib is not None:
            return _lib
        path = LIB_PATH
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_2503_18682_amd.build, or __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


class RayGSError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
