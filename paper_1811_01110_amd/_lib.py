"""ctypes declarations of libtsqbx.so (include/tsqbx.h).

Loading fails loudly if the library is not built: there is no fallback
implementation.  torch is imported first when it is installed so that the
library shares torch's HIP runtime (device pointers and streams of torch
tensors are then valid in the library).
"""
from __future__ import annotations

import ctypes
import os

LIBPATH = os.environ.get("TSQBX_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                       "libtsqbx.so")

c_int, c_uint, c_int64, c_uint64, c_size_t, c_double, c_void_p, c_char_p = (
    ctypes.c_int, ctypes.c_uint, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t,
    ctypes.c_double, ctypes.c_void_p, ctypes.c_char_p)

OK, E_INVALID, E_RANGE, E_NOMEM, E_DEVICE, E_BUDGET, E_STATE, E_TIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
E_CANCELED = -8
SLP, DLP, SPRIME = 1, 2, 4
HELMHOLTZ = 64
ACCUMULATE, NO_REORDER, PER_TARGET = 1, 2, 4
P_MAX = 32


class GeometryDesc(ctypes.Structure):
    _fields_ = [
        ("n_sources", c_int64), ("sources", c_void_p), ("weights", c_void_p), ("normals", c_void_p),
        ("n_centers", c_int64), ("centers", c_void_p), ("list_offsets", c_void_p),
        ("list_sources", c_void_p), ("n_targets", c_int64), ("targets", c_void_p),
        ("target_center", c_void_p), ("target_normals", c_void_p),
    ]


class GeometryInfo(ctypes.Structure):
    _fields_ = [("n_sources", c_int64), ("n_centers", c_int64), ("n_targets", c_int64),
                ("nnz", c_int64), ("pairs", c_int64), ("max_list", c_int64),
                ("device_bytes", c_size_t), ("has_normals", c_int),
                ("has_target_normals", c_int)]


class Tuning(ctypes.Structure):
    _fields_ = [("waves_per_block", c_int), ("group_lanes", c_int), ("unroll", c_int),
                ("xcd_remap", c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Item(ctypes.Structure):
    _fields_ = [("geom", c_void_p), ("p", c_int), ("layers", c_uint), ("d_sigma", c_void_p),
                ("d_out_slp", c_void_p), ("d_out_dlp", c_void_p), ("d_out_sprime", c_void_p)]


class HelmItem(ctypes.Structure):
    _fields_ = [("geom", c_void_p), ("p", c_int), ("layers", c_uint), ("k", c_double),
                ("d_sigma", c_void_p), ("d_out_slp", c_void_p), ("d_out_dlp", c_void_p),
                ("d_out_sprime", c_void_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_items", c_int64), ("n_units", c_int64), ("pairs", c_int64),
                ("pair_terms", c_int64), ("grid_blocks", c_int), ("waves_per_block", c_int),
                ("device_bytes", c_size_t)]


class LayoutInfo(ctypes.Structure):
    _fields_ = [("n_rows", c_int64), ("nnz", c_int64), ("pairs", c_int64), ("max_list", c_int64)]


class PlanTuning(ctypes.Structure):
    _fields_ = [("group_lanes", c_int), ("unroll", c_int), ("waves_per_block", c_int),
                ("oversubscription", c_int), ("step_cost", c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerTuning(ctypes.Structure):
    _fields_ = [("group_lanes", c_int), ("unroll", c_int), ("waves_per_block", c_int),
                ("unit_steps", c_int), ("step_requests", c_int), ("dma_min_sources", c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanTiming(ctypes.Structure):
    _fields_ = [("stage_ms", c_double), ("eval_ms", c_double), ("reps", c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_uint64), ("admitted", c_uint64), ("completed", c_uint64),
                ("failed", c_uint64), ("rejected", c_uint64), ("steps", c_uint64),
                ("bytes_in_flight", c_size_t), ("peak_bytes_in_flight", c_size_t),
                ("budget_bytes", c_size_t), ("pair_terms_completed", c_int64),
                ("latency_p50_ms", c_double), ("latency_p90_ms", c_double),
                ("latency_p99_ms", c_double), ("latency_max_ms", c_double),
                ("queue_p50_ms", c_double), ("queue_p99_ms", c_double), ("busy_s", c_double),
                ("host_launch_s", c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


P = ctypes.POINTER
_SIGNATURES = {
    "tsqbx_version": (c_int, []),
    "tsqbx_last_error": (c_char_p, []),
    "tsqbx_validate_geometry": (c_int, [P(GeometryDesc)]),
    "tsqbx_check_request": (c_int, [c_void_p, c_int, c_uint]),
    "tsqbx_ctx_create": (c_int, [c_int, P(c_void_p)]),
    "tsqbx_ctx_destroy": (c_int, [c_void_p]),
    "tsqbx_geometry_create": (c_int, [c_void_p, P(GeometryDesc), c_uint, P(c_void_p)]),
    "tsqbx_geometry_destroy": (c_int, [c_void_p]),
    "tsqbx_geometry_get_info": (c_int, [c_void_p, P(GeometryInfo)]),
    "tsqbx_eval": (c_int, [c_void_p, c_void_p, c_int, c_uint, c_void_p, c_void_p, c_void_p,
                           c_void_p, c_uint]),
    "tsqbx_eval_async": (c_int, [c_void_p, c_void_p, c_int, c_uint, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_uint, c_void_p]),
    "tsqbx_stage_async": (c_int, [c_void_p, c_void_p, c_uint, c_void_p, c_void_p]),
    "tsqbx_eval_staged_async": (c_int, [c_void_p, c_void_p, c_int, c_uint, c_void_p, c_void_p,
                                        c_void_p, c_uint, c_void_p]),
    "tsqbx_qbxl_form_async": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_uint,
                                      c_void_p]),
    "tsqbx_qbxl_eval_async": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_uint,
                                      c_void_p]),
    "tsqbx_eval_conventional_async": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p,
                                              c_uint, c_void_p]),
    "tsqbx_eval_helmholtz": (c_int, [c_void_p, c_void_p, c_int, c_uint, c_double, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_uint]),
    "tsqbx_eval_helmholtz_async": (c_int, [c_void_p, c_void_p, c_int, c_uint, c_double, c_void_p,
                                           c_void_p, c_void_p, c_void_p, c_uint, c_void_p]),
    "tsqbx_ball_lists": (c_int, [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_double,
                                 c_void_p, c_void_p, c_int64, P(c_int64), c_void_p]),
    "tsqbx_knn_lists": (c_int, [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p,
                                c_void_p, c_void_p, c_int64, P(c_int64), c_void_p]),
    "tsqbx_get_tuning": (c_int, [c_void_p, c_int, c_uint, c_int64, P(Tuning)]),
    "tsqbx_set_tuning": (c_int, [c_void_p, c_int, c_uint, c_int64, P(Tuning)]),
    "tsqbx_autotune": (c_int, [c_void_p, c_void_p, c_int, c_uint, P(Tuning), P(c_double)]),
    "tsqbx_schedule_preview": (c_int, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                       c_int, c_void_p, c_int64, P(c_int64), c_void_p,
                                       P(ctypes.c_int32)]),
    "tsqbx_plan_create": (c_int, [c_void_p, c_int64, P(Item), c_uint, P(c_void_p)]),
    "tsqbx_plan_create_helmholtz": (c_int, [c_void_p, c_int64, P(HelmItem), c_uint, P(c_void_p)]),
    "tsqbx_plan_execute": (c_int, [c_void_p, c_void_p]),
    "tsqbx_plan_get_info": (c_int, [c_void_p, P(PlanInfo)]),
    "tsqbx_plan_destroy": (c_int, [c_void_p]),
    "tsqbx_eval_async_noalloc": (c_int, [c_void_p, c_void_p, c_int, c_uint, c_void_p, c_void_p,
                                         c_void_p, c_void_p, c_uint, c_void_p]),
    "tsqbx_geometry_layout": (c_int, [P(GeometryDesc), c_uint, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_int64, c_void_p, c_int64, P(LayoutInfo)]),
    "tsqbx_geometry_create_device": (c_int, [c_void_p, P(GeometryDesc), c_uint, c_void_p,
                                             P(c_void_p)]),
    "tsqbx_geometry_read_layout": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                           c_int64, c_void_p, c_int64, P(LayoutInfo)]),
    "tsqbx_plan_get_tuning": (c_int, [c_void_p, P(PlanTuning)]),
    "tsqbx_plan_set_tuning": (c_int, [c_void_p, P(PlanTuning)]),
    "tsqbx_plan_profile": (c_int, [c_void_p, c_int, c_void_p, P(PlanTiming)]),
    "tsqbx_plan_autotune": (c_int, [c_void_p, c_void_p, P(PlanTuning), P(c_double)]),
    "tsqbx_tuning_save": (c_int, [c_void_p, ctypes.c_char_p]),
    "tsqbx_tuning_load": (c_int, [c_void_p, ctypes.c_char_p, P(c_int)]),
    "tsqbx_server_create": (c_int, [c_void_p, c_size_t, c_int, P(c_void_p)]),
    "tsqbx_server_request_bytes": (c_int, [c_void_p, c_uint, P(c_size_t)]),
    "tsqbx_server_submit": (c_int, [c_void_p, c_void_p, c_int, c_uint, c_void_p, c_void_p,
                                    c_void_p, c_void_p, P(c_uint64)]),
    "tsqbx_server_submit_pinned": (c_int, [c_void_p, c_void_p, c_int, c_uint, c_void_p, c_void_p,
                                           c_void_p, c_void_p, P(c_uint64)]),
    "tsqbx_server_submit_helmholtz": (c_int, [c_void_p, c_void_p, c_int, c_uint, c_double,
                                              c_void_p, c_void_p, c_void_p, c_void_p,
                                              P(c_uint64)]),
    "tsqbx_server_submit_helmholtz_pinned": (c_int, [c_void_p, c_void_p, c_int, c_uint, c_double,
                                                     c_void_p, c_void_p, c_void_p, c_void_p,
                                                     P(c_uint64)]),
    "tsqbx_server_request_bytes_helmholtz": (c_int, [c_void_p, c_int, c_uint, P(c_size_t)]),
    "tsqbx_server_poll": (c_int, [c_void_p, c_uint64, P(c_int)]),
    "tsqbx_server_wait": (c_int, [c_void_p, c_uint64, c_double]),
    "tsqbx_server_drain": (c_int, [c_void_p, c_double]),
    "tsqbx_server_cancel": (c_int, [c_void_p, c_uint64]),
    "tsqbx_server_get_tuning": (c_int, [c_void_p, P(ServerTuning)]),
    "tsqbx_server_set_tuning": (c_int, [c_void_p, P(ServerTuning)]),
    "tsqbx_server_autotune": (c_int, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_int, P(ServerTuning), P(c_double)]),
    "tsqbx_server_get_stats": (c_int, [c_void_p, P(ServerStats)]),
    "tsqbx_server_destroy": (c_int, [c_void_p]),
}

_lib = None


def exported_names():
    return list(_SIGNATURES)


def load():
    """Load libtsqbx.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    try:  # share torch's HIP runtime when torch is present
        import torch  # noqa: F401
    except Exception:
        pass
    if not os.path.exists(LIBPATH):
        raise ImportError(f"{LIBPATH} is not built: run `python -m paper_1811_01110_amd.build` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIBPATH)
    missing = [n for n in _SIGNATURES if not hasattr(lib, n)]
    if missing:
        raise ImportError(f"{LIBPATH} lacks exported symbols: {', '.join(missing)}")
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
