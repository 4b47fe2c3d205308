"""ctypes loader for libmx.so and the signatures of every C entry point.

The library must have been built (``python -m paper_2211_00621_amd.build``);
there is no fallback: loading fails with an ImportError naming what is missing.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmx.so")

c_status = ctypes.c_int
c_enum = ctypes.c_int
c_i64 = ctypes.c_int64
c_size = ctypes.c_size_t
c_p = ctypes.c_void_p
c_pp = ctypes.POINTER(ctypes.c_void_p)
c_f32 = ctypes.c_float
c_int = ctypes.c_int

# name -> (restype, argtypes); kept in the order of include/mx.h
SIGNATURES = {
    "mx_init": (c_status, [c_int]),
    "mx_last_error": (ctypes.c_char_p, []),
    "mx_version": (ctypes.c_char_p, []),
    "mx_set_debug": (c_status, [c_int]),
    "mx_get_debug": (c_int, []),
    "mx_workspace_bytes": (c_size, [c_enum, c_i64, c_i64]),
    "mx_copy32": (c_status, [c_p, c_p, c_i64, c_p]),
    "mx_stream_read": (c_status, [c_p, c_i64, c_p, c_p]),
    "mx_lengths_to_offsets": (c_status, [c_p, c_i64, c_p, c_p, c_size, c_p]),
    "mx_marshal_rows": (c_status, [c_pp, c_p, c_i64, c_size, c_p, c_size, c_p, c_p, c_p, c_p, c_size, c_p]),
    "mx_unmarshal_rows": (c_status, [c_p, c_p, c_i64, c_size, c_p, c_size, c_pp, c_p]),
    "mx_records_to_fields": (c_status, [c_p, c_i64, c_int, c_size, c_pp, c_p]),
    "mx_fields_to_records": (c_status, [c_pp, c_i64, c_int, c_size, c_p, c_p]),
    "mx_compose_offsets": (c_status, [c_p, c_i64, c_p, c_p, c_p]),
    "mx_offsets_regular": (c_status, [c_p, c_i64, c_p, c_p]),
    "mx_map": (c_status, [c_enum, c_enum, c_p, c_i64, c_p, c_p, c_p]),
    "mx_map2": (c_status, [c_enum, c_enum, c_p, c_p, c_i64, c_p, c_p]),
    "mx_reduce": (c_status, [c_enum, c_enum, c_p, c_i64, c_p, c_p, c_p, c_size, c_p]),
    "mx_map2_reduce": (c_status, [c_enum, c_enum, c_enum, c_p, c_p, c_i64, c_p, c_p, c_p, c_size, c_p]),
    "mx_dot_adjoint_f32": (c_status, [c_p, c_p, c_i64, c_p, c_p, c_p, c_p]),
    "mx_segmented_reduce": (c_status, [c_enum, c_enum, c_p, c_i64, c_p, c_i64, c_p, c_p, c_p, c_size, c_p]),
    "mx_segmented_reduce_noalloc": (c_status, [c_enum, c_enum, c_p, c_i64, c_p, c_i64, c_p, c_p, c_p]),
    "mx_segmented_noalloc_max_values": (c_i64, []),
    "mx_segmented_reduce_plain": (c_status, [c_enum, c_enum, c_p, c_i64, c_p, c_i64, c_p, c_p, c_p]),
    "mx_segmented_sum_adjoint_f32": (c_status, [c_p, c_p, c_i64, c_p, c_i64, c_p]),
    "mx_reduce_adjoint_f32": (c_status, [c_enum, c_p, c_i64, c_p, c_p, c_p, c_p, c_size, c_p]),
    "mx_segmented_reduce_adjoint_f32": (c_status, [c_enum, c_p, c_i64, c_p, c_i64, c_p, c_p, c_p, c_p]),
    "mx_map_map_reduce_f32": (c_status, [c_int, c_int, c_i64, c_i64, c_i64, c_p, c_p, c_p, c_p]),
    "mx_map_map_reduce_plain_f32": (c_status, [c_int, c_int, c_i64, c_i64, c_i64, c_p, c_p, c_p, c_p]),
    "mx_nbody_pair_workspace_bytes": (c_size, [c_i64]),
    "mx_nbody_accel_f32": (c_status, [c_p, c_i64, c_f32, c_f32, c_p, c_p, c_size, c_p]),
    "mx_nbody_step_f32": (c_status, [c_p, c_p, c_i64, c_f32, c_f32, c_f32, c_p, c_p, c_p, c_size, c_p]),
    "mx_nbody_step_plain_f32": (c_status, [c_p, c_p, c_i64, c_f32, c_f32, c_f32, c_p, c_p, c_p, c_p]),
    "mx_nbody_accel_vjp_f32": (c_status, [c_p, c_p, c_i64, c_f32, c_f32, c_p, c_p, c_size, c_p]),
    "mx_nbody_adjoint_step_f32": (c_status, [c_p, c_p, c_p, c_i64, c_f32, c_f32, c_f32, c_p, c_p, c_p, c_size,
                                             c_p]),
    "mx_nbody_kinetic_f32": (c_status, [c_p, c_p, c_i64, c_p, c_p]),
    "mx_nbody_workspace_bytes": (c_size, [c_i64, c_int, c_int]),
    "mx_nbody_ke_grad_f32": (c_status, [c_p, c_p, c_i64, c_f32, c_f32, c_f32, c_int, c_int, c_p, c_p, c_p, c_p,
                                        c_size, c_p]),
    "mx_nbody_ke_f32": (c_status, [c_p, c_p, c_i64, c_f32, c_f32, c_f32, c_int, c_int, c_p, c_p, c_size, c_p]),
    "mx_nbody_ke_vjp_f32": (c_status, [c_p, c_p, c_i64, c_f32, c_f32, c_f32, c_int, c_int, c_p, c_p, c_p, c_p,
                                       c_size, c_p]),
    "mx_kmeans_workspace_bytes": (c_size, [c_i64, c_int, c_int]),
    "mx_kmeans_step_f32": (c_status, [c_p, c_i64, c_int, c_p, c_int, c_p, c_p, c_p, c_p, c_size, c_p]),
    "mx_kmeans_debug_fallbacks": (c_i64, []),
    "mx_kmeans_step_plain_f32": (c_status, [c_p, c_i64, c_int, c_p, c_int, c_p, c_p, c_p, c_p, c_size, c_p]),
    "mx_kmeans_sse_f32": (c_status, [c_p, c_i64, c_int, c_p, c_p, c_p, c_p, c_size, c_p]),
    "mx_kmeans_sse_grad_f32": (c_status, [c_p, c_i64, c_int, c_p, c_p, c_p, c_p, c_p]),
    "mx_batch_plan_create": (c_status, [c_p, c_i64, c_p, c_pp]),
    "mx_batch_plan_destroy": (c_status, [c_p]),
    "mx_batch_workspace_bytes": (c_size, [c_p]),
    "mx_batch_get_config": (c_status, [c_p, c_p]),
    "mx_batch_set_config": (c_status, [c_p, c_p]),
    "mx_batch_forward": (c_status, [c_p, c_p, c_p, c_p, c_p, c_size, c_p]),
    "mx_batch_backward": (c_status, [c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_size, c_p]),
    "mx_batch_forward_plain": (c_status, [c_p, c_p, c_p, c_p, c_p]),
    "mx_batch_backward_plain": (c_status, [c_p, c_p, c_p, c_p, c_p, c_p, c_p]),
    "mx_batch_autotune": (c_status, [c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_size, ctypes.c_char_p, c_p, c_p]),
    "mx_histogram_u32": (c_status, [c_p, c_i64, c_i64, c_p, c_p, c_size, c_p]),
    "mx_stencil7_f32": (c_status, [c_p, c_p, c_i64, c_i64, c_i64, c_f32, c_f32, c_p]),
    "mx_mriq_f32": (c_status, [c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_p, c_i64, c_p, c_p, c_p]),
    "mx_tpacf_f32": (c_status, [c_p, c_p, c_p, c_i64, c_p, c_p, c_p, c_i64, c_int, c_p, c_int, c_p, c_p]),
    "mx_expr_create": (c_status, [c_p, c_int, c_int, c_int, c_enum, c_pp]),
    "mx_expr_destroy": (c_status, [c_p]),
    "mx_expr_prepare": (c_status, [c_p]),
    "mx_expr_source": (ctypes.c_char_p, [c_p]),
    "mx_expr_map": (c_status, [c_p, c_pp, c_i64, c_p, c_p]),
    "mx_expr_workspace_bytes": (c_size, [c_p, c_i64]),
    "mx_expr_map_reduce": (c_status, [c_p, c_enum, c_pp, c_i64, c_p, c_p, c_p, c_size, c_p]),
    "mx_expr_segmented_reduce": (c_status, [c_p, c_enum, c_pp, c_p, c_i64, c_p, c_p, c_p]),
    "mx_expr_loop_workspace_bytes": (c_size, [c_i64]),
    "mx_expr_loop_scatter": (c_status, [c_p, c_pp, c_i64, c_p, c_p, c_i64, c_p, c_size, c_p]),
    "mx_expr_vjp": (c_status, [c_p, c_pp, c_i64, c_p, c_p, c_pp, c_p]),
    "mx_records_layout": (c_status, [c_p, c_i64, c_size, c_p, c_int, c_p, c_p]),
    "mx_marshal_records": (c_status, [c_p, c_i64, c_size, c_p, c_int, c_p, c_size, c_p, c_size, c_p]),
    "mx_unmarshal_records": (c_status, [c_p, c_int, c_i64, c_p, c_size, c_p, c_size, c_p]),
    "mx_loop_create": (c_status, [c_p, c_int, c_p, c_int, c_enum, c_pp]),
    "mx_loop_destroy": (c_status, [c_p]),
    "mx_loop_prepare": (c_status, [c_p]),
    "mx_loop_source": (ctypes.c_char_p, [c_p]),
    "mx_loop_workspace_bytes": (c_size, [c_p, c_p]),
    "mx_loop_run": (c_status, [c_p, c_i64, c_p, c_p, c_size, c_p]),
    "mx_graph_begin": (c_status, [c_p]),
    "mx_graph_end": (c_status, [c_p, c_pp]),
    "mx_graph_launch": (c_status, [c_p, c_p]),
    "mx_graph_destroy": (c_status, [c_p]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libmx.so once and declare all signatures.  Raises ImportError."""
    global _lib
    if _lib is not None:
        return _lib
    # torch brings its own HIP runtime; loading it first makes libmx.so bind to
    # that same runtime (by soname) instead of starting a second one
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2211_00621_amd/build.py` "
                          "(the primitives have no CPU fallback)")
    try:
        lib = ctypes.CDLL(LIB_PATH)
    except OSError as e:  # pragma: no cover - environment specific
        raise ImportError(f"cannot load {LIB_PATH}: {e}") from e
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
