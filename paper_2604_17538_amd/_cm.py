"""ctypes binding of libcm.so (include/cm.h): same names, argument marshalling only.

Every step of the contact pipeline runs in the library's gfx950 kernels.  If the
library is missing this module raises at import; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libcm.so is not built; run `python -m paper_2604_17538_amd.build` "
                      "(hipcc for gfx950) first")

try:
    # torch's HIP code links the HIP runtime by its unversioned name from its own
    # lib directory; loading torch first makes this library bind to that same
    # runtime instead of bringing a second copy into the process
    import torch  # noqa: F401
except ImportError:
    pass

lib = ctypes.CDLL(LIB_PATH)

CM_OK, CM_E_INVALID, CM_E_OOM, CM_E_DEGENERATE, CM_E_HIP, CM_E_BUSY, CM_E_NOTFOUND = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "CM_OK", -1: "CM_E_INVALID", -2: "CM_E_OOM", -3: "CM_E_DEGENERATE", -4: "CM_E_HIP",
                -5: "CM_E_BUSY", -6: "CM_E_NOTFOUND"}


class cm_params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in
                ("tau_cap", "tau_cup", "tau_st", "tau_clip", "tau_blend", "d_max", "eps_t", "eps_n",
                 "grid_margin", "grid_margin_rel")] + \
               [(n, ctypes.c_int32) for n in ("st_iters", "grid_res", "curve", "broad_phase", "edge_bound", "prune_pieces",
                                              "sdf_kind", "edge_assign")] + \
               [(n, ctypes.c_float) for n in ("tau_t", "tau_disc")]


class cm_groups(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("p", "n", "d", "q", "W", "logZ")]


class cm_request(ctypes.Structure):
    _fields_ = [("q", ctypes.c_void_p), ("n", ctypes.c_int32), ("want_grad", ctypes.c_int32),
                ("cotangent", ctypes.c_void_p), ("out_groups", ctypes.c_void_p), ("out_grad", ctypes.c_void_p)]


# cm_query as a numpy structured dtype (64 bytes)
QUERY_DTYPE = np.dtype([("a", "<u4"), ("b", "<u4"), ("qa", "<f4", 4), ("ta", "<f4", 3),
                        ("qb", "<f4", 4), ("tb", "<f4", 3)])
assert QUERY_DTYPE.itemsize == 64

P = ctypes.c_void_p
I32, I64, U32, U64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
PP = ctypes.POINTER(ctypes.c_void_p)


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
    return f


cm_default_params = _sig("cm_default_params", I32, [ctypes.c_float, ctypes.POINTER(cm_params)])
cm_init = _sig("cm_init", I32, [I32, ctypes.POINTER(cm_params), ctypes.c_size_t, PP])
cm_shutdown = _sig("cm_shutdown", I32, [P])
cm_last_error = _sig("cm_last_error", ctypes.c_char_p, [P])
cm_build_pieces = _sig("cm_build_pieces", I32, [P, I32, P, P, ctypes.POINTER(U32)])
cm_build_objects = _sig("cm_build_objects", I32, [P, I32, P, P, P, P])
cm_build_pieces_raw = _sig("cm_build_pieces_raw", I32, [P, I32, P, P, P, P, P, P, ctypes.POINTER(U32)])
cm_release_object = _sig("cm_release_object", I32, [P, U32])
cm_object_info = _sig("cm_object_info", I32, [P, U32, ctypes.POINTER(I32), ctypes.POINTER(I64),
                                              ctypes.POINTER(I64), ctypes.POINTER(I64)])
cm_object_export = _sig("cm_object_export", I32, [P, U32, P, P, P, P, P, P])
cm_object_grid = _sig("cm_object_grid", I32, [P, U32, P, P])
cm_object_spline = _sig("cm_object_spline", I32, [P, U32, P, P])
cm_object_set_prims = _sig("cm_object_set_prims", I32, [P, U32, I32, P, P, P])
cm_plan_create = _sig("cm_plan_create", I32, [P, P, I32, PP])
cm_plan_destroy = _sig("cm_plan_destroy", I32, [P])
cm_plan_reserve = _sig("cm_plan_reserve", I32, [P, I32, I64, I64, PP])
cm_plan_refill = _sig("cm_plan_refill", I32, [P, P, P, I32, P])
cm_plan_capacity = _sig("cm_plan_capacity", I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I64), ctypes.POINTER(I64)])
cm_plan_info = _sig("cm_plan_info", I32, [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I32)])
cm_plan_offsets = _sig("cm_plan_offsets", I32, [P, P, P])
cm_plan_stats = _sig("cm_plan_stats", I32, [P, P])
cm_plan_work = _sig("cm_plan_work", I32, [P, P])
cm_plan_set_timing = _sig("cm_plan_set_timing", I32, [P, I32])
cm_plan_timing = _sig("cm_plan_timing", I32, [P, P])
cm_contacts_fwd = _sig("cm_contacts_fwd", I32, [P, P, P, cm_groups, P, P])
cm_contacts_fwd_noalloc = _sig("cm_contacts_fwd_noalloc", I32, [P, P, P, cm_groups, P])
cm_contacts_bwd = _sig("cm_contacts_bwd", I32, [P, P, P, cm_groups, P, P])
cm_hvp = _sig("cm_hvp", I32, [P, P, P, cm_groups, P, P, P, P])
cm_contacts_jvp = _sig("cm_contacts_jvp", I32, [P, P, P, cm_groups, cm_groups, P, P])
cm_project_points = _sig("cm_project_points", I32, [P, P, P, P, P, P])
cm_contacts_step = _sig("cm_contacts_step", I32, [P, P, P, cm_groups, cm_groups, P, P, P, P])
cm_graph_create = _sig("cm_graph_create", I32, [P, P, P, cm_groups, cm_groups, P, P, P, PP])
cm_graph_launch = _sig("cm_graph_launch", I32, [P, P])
cm_graph_destroy = _sig("cm_graph_destroy", I32, [P])
cm_plan_autotune = _sig("cm_plan_autotune", I32, [P, P, P, cm_groups, P, P, P, P, ctypes.POINTER(I32)])
cm_plan_set_launch_shape = _sig("cm_plan_set_launch_shape", I32, [P, I32, I32])
cm_plan_launch_shape = _sig("cm_plan_launch_shape", I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I32)])
cm_plan_set_wg_waves = _sig("cm_plan_set_wg_waves", I32, [P, I32, I32])
cm_plan_wg_waves = _sig("cm_plan_wg_waves", I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I32)])
cm_submit = _sig("cm_submit", I32, [P, ctypes.POINTER(cm_request), ctypes.POINTER(U64)])
cm_poll = _sig("cm_poll", I32, [P, U64, ctypes.POINTER(I32), ctypes.POINTER(I32)])
cm_wait = _sig("cm_wait", I32, [P, U64, I32, ctypes.POINTER(I32)])
cm_serve_stats = _sig("cm_serve_stats", I32, [P, P])
cm_serve_latencies = _sig("cm_serve_latencies", I32, [P, P, I64, ctypes.POINTER(I64)])

EXPORTED = ["cm_default_params", "cm_init", "cm_shutdown", "cm_last_error", "cm_build_pieces", "cm_build_objects",
            "cm_build_pieces_raw", "cm_release_object", "cm_object_info", "cm_object_export", "cm_object_grid", "cm_object_spline", "cm_object_set_prims",
            "cm_plan_create", "cm_plan_destroy", "cm_plan_reserve", "cm_plan_refill", "cm_plan_capacity", "cm_plan_info", "cm_plan_offsets", "cm_plan_stats", "cm_plan_work",
            "cm_plan_set_timing", "cm_plan_timing",
            "cm_contacts_fwd", "cm_contacts_fwd_noalloc", "cm_contacts_bwd", "cm_hvp", "cm_contacts_jvp", "cm_project_points",
            "cm_contacts_step", "cm_graph_create", "cm_graph_launch",
            "cm_graph_destroy", "cm_plan_autotune", "cm_plan_set_launch_shape", "cm_plan_launch_shape", "cm_plan_set_wg_waves", "cm_plan_wg_waves",
            "cm_submit", "cm_poll", "cm_wait", "cm_serve_stats",
            "cm_serve_latencies"]
