"""ctypes view of libdiffus.so (the C ABI of include/diffus.h).

Argument marshalling only: every step of the renderer runs in the HIP
kernels behind these entry points.  Importing this module never falls back
to anything else; if the library is missing, ``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdiffus.so")

c_i32, c_i64, c_f32, c_u64, c_sz, c_vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                           ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p)

DUS_OK, DUS_EINVAL, DUS_ESHAPE, DUS_EWORKSPACE, DUS_EHIP, DUS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
REFL_ABS, REFL_SIGNED = 0, 1
ATTEN_IN_SYSTEM, ATTEN_POST_HOC, ATTEN_OFF = 0, 1, 2
PLAN_POSE_ONLY, PLAN_ZERO_GRAD_Z, PLAN_NO_GRAPH, PLAN_DETERMINISTIC, PLAN_ONE_STREAM = 1, 2, 4, 8, 16
# phases of a plan step (DUS_PHASE_*), in launch order
PHASES = ("clear", "forward", "blur_loss", "adjoint", "scatter", "finish")
MAX_SAMPLES, MAX_RAYS, MAX_BLUR_RADIUS = 16384, 65536, 32
STATIC_SCRATCH_BYTES = 32 << 20


class DusVolume(ctypes.Structure):
    _fields_ = [("nx", c_i32), ("ny", c_i32), ("nz", c_i32),
                ("spacing_mm", c_f32 * 3), ("origin_mm", c_f32 * 3)]


class DusFan(ctypes.Structure):
    _fields_ = [("n_rays", c_i32), ("n_samples", c_i32), ("aperture_rad", c_f32),
                ("ds_mm", c_f32), ("r0_mm", c_f32), ("speckle_id", c_i32), ("out_offset", c_i64)]


class DusPhysics(ctypes.Structure):
    _fields_ = [("alpha_db_cm_mhz", c_f32), ("f_mhz", c_f32), ("refl_mode", c_i32),
                ("atten_mode", c_i32), ("speckle_on", c_i32), ("spk_cell", c_i32),
                ("spk_Ar", c_f32), ("spk_gamma", c_f32), ("spk_Ag0", c_f32), ("spk_Ag1", c_f32),
                ("blur_on", c_i32), ("blur_sigma0", c_f32), ("blur_sigma1", c_f32),
                ("reserved", c_i32), ("seed", c_u64)]


class DusSchedule(ctypes.Structure):
    _fields_ = [("fwd_chunk", c_i32), ("bwd_chunk", c_i32), ("xcd_group", c_i32), ("scatter_rays", c_i32),
                ("span_samples", c_i32)]


class DusGrid2d(ctypes.Structure):
    _fields_ = [("nx", c_i32), ("nz", c_i32), ("x0_mm", ctypes.c_float), ("z0_mm", ctypes.c_float),
                ("dx_mm", ctypes.c_float), ("dz_mm", ctypes.c_float), ("fill", ctypes.c_float)]


MAX_KNOTS = 64


class DusLut(ctypes.Structure):
    _fields_ = [("n", c_i32), ("x", ctypes.c_float * MAX_KNOTS), ("z", ctypes.c_float * MAX_KNOTS)]


# every symbol include/diffus.h declares, with (restype, argtypes)
SIGNATURES = {
    "dus_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "dus_last_error": (ctypes.c_char_p, []),
    "dus_version": (ctypes.c_int, []),
    "dus_workspace_bytes": (c_i64, [ctypes.POINTER(DusVolume), ctypes.POINTER(DusFan), c_i32,
                                    ctypes.POINTER(DusPhysics), c_i32]),
    "dus_render_bmode": (ctypes.c_int, [c_vp, ctypes.POINTER(DusVolume), c_vp, ctypes.POINTER(DusFan),
                                        c_i32, ctypes.POINTER(DusPhysics), c_vp, c_vp, c_vp, c_sz, c_vp]),
    "dus_render_bmode_backward": (ctypes.c_int, [c_vp, ctypes.POINTER(DusVolume), c_vp,
                                                 ctypes.POINTER(DusFan), c_i32, ctypes.POINTER(DusPhysics),
                                                 c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "dus_render_bmode_backward_static": (ctypes.c_int, [c_vp, ctypes.POINTER(DusVolume), c_vp,
                                                        ctypes.POINTER(DusFan), c_i32, ctypes.POINTER(DusPhysics),
                                                        c_vp, c_vp, c_vp, c_vp]),
    "dus_philox4x32_10": (ctypes.c_int, [c_vp, c_i64, c_u64, c_vp, c_vp]),
    "dus_pixel_gain": (ctypes.c_int, [ctypes.POINTER(DusFan), ctypes.POINTER(DusPhysics), c_vp, c_vp]),
    "dus_sample_volume": (ctypes.c_int, [c_vp, ctypes.POINTER(DusVolume), c_vp, ctypes.POINTER(DusFan), c_i32,
                                         c_vp, c_vp]),
    "dus_scan_convert": (ctypes.c_int, [c_vp, ctypes.POINTER(DusFan), ctypes.POINTER(DusGrid2d), c_vp, c_vp]),
    "dus_map_impedance": (ctypes.c_int, [c_vp, c_i64, ctypes.POINTER(DusLut), c_vp, c_vp]),
    "dus_map_impedance_backward": (ctypes.c_int, [c_vp, c_i64, ctypes.POINTER(DusLut), c_vp, c_vp, c_vp, c_vp]),
    "dus_smoothness_workspace_bytes": (ctypes.c_int64, [ctypes.POINTER(DusVolume)]),
    "dus_smoothness": (ctypes.c_int, [c_vp, ctypes.POINTER(DusVolume), ctypes.c_float, c_vp, c_vp, c_vp, c_sz,
                                      c_vp]),
    "dus_adam_step": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, c_i32, ctypes.c_float, ctypes.c_float, c_vp]),
    "dus_footprint_mask": (ctypes.c_int, [ctypes.POINTER(DusVolume), c_vp, ctypes.POINTER(DusFan), c_i32,
                                          c_vp, c_vp]),
    "dus_set_schedule": (ctypes.c_int, [ctypes.POINTER(DusSchedule)]),
    "dus_get_schedule": (ctypes.c_int, [ctypes.POINTER(DusSchedule)]),
    "dus_plan_create": (ctypes.c_int, [ctypes.POINTER(c_vp), ctypes.POINTER(DusVolume), ctypes.POINTER(DusFan),
                                       c_i32, ctypes.POINTER(DusPhysics), c_i32]),
    "dus_plan_workspace_bytes": (c_i64, [c_vp]),
    "dus_plan_set_schedule": (ctypes.c_int, [c_vp, ctypes.POINTER(DusSchedule)]),
    "dus_plan_get_schedule": (ctypes.c_int, [c_vp, ctypes.POINTER(DusSchedule)]),
    "dus_plan_step": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "dus_plan_step_timed": (ctypes.c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp,
                                           ctypes.POINTER(ctypes.c_float)]),
    "dus_plan_destroy": (None, [c_vp]),
}

_lib = None


def lib():
    """Load libdiffus.so (built in-tree by paper_2508_06768_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2508_06768_amd.build` "
                "(the renderer has no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class DusError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.dus_status_string(status).decode()
        detail = L.dus_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}): {detail}")
        self.status = status


def check(status: int, where: str) -> int:
    if status < 0:
        raise DusError(status, where)
    return status
