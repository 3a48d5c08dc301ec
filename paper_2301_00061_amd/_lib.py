"""ctypes view of libkc.so (include/kc.h). Argument marshalling only.

The library must be built (``python -m paper_2301_00061_amd.build``); loading
fails loudly otherwise -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkc.so")

KC_OK, KC_EINVAL, KC_ENOMEM, KC_EDEVICE, KC_EUNSUPPORTED = 0, -1, -2, -3, -4
MLP_PARAMS = 10497
NOALLOC_SCRATCH_BYTES = 4 << 20  # KC_NOALLOC_SCRATCH_BYTES

# every entry point declared in include/kc.h
EXPORTS = [
    "kc_create", "kc_destroy", "kc_last_error", "kc_rel_margin", "kc_abs_margin",
    "kc_lower_bound", "kc_lower_bound_noalloc", "kc_objective", "kc_objective_screen", "kc_fft", "kc_tighten", "kc_reduce", "kc_autotune", "kc_autotune_tighten",
    "kc_mlp_forward", "kc_mlp_backward", "kc_mlp_loss", "kc_mlp_adam", "kc_solve",
]


class Points(C.Structure):
    _fields_ = [("x", C.c_void_p), ("n", C.c_int64), ("ld", C.c_int64), ("d", C.c_int32),
                ("reserved", C.c_int32)]


class Nodes(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_boxes", C.c_int32), ("k_max", C.c_int32),
                ("reserved", C.c_int32), ("box_off", C.c_void_p), ("lo", C.c_void_p),
                ("hi", C.c_void_p)]


class Refs(C.Structure):
    _fields_ = [("n_refs", C.c_int32), ("max_per_box", C.c_int32), ("ref_off", C.c_void_p),
                ("ref", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("k", C.c_int32), ("batch", C.c_int32), ("i_sr", C.c_int32),
                ("use_bt", C.c_int32), ("use_seeds", C.c_int32), ("max_refs", C.c_int32),
                ("branching", C.c_int32), ("keep_order", C.c_int32), ("node_sr", C.c_int32),
                ("autotune", C.c_int32), ("fft_start", C.c_int64), ("max_nodes", C.c_int64), ("eps_rel", C.c_double),
                ("time_limit_s", C.c_double), ("mlp_w", C.c_void_p), ("verbose", C.c_int32),
                ("sb_first", C.c_int32), ("sb_every", C.c_int32), ("sb_cap", C.c_int32),
                ("sb_feat", C.c_void_p), ("sb_score", C.c_void_p), ("sb_node", C.c_void_p),
                ("sb_lo", C.c_void_p), ("sb_hi", C.c_void_p), ("sb_ka", C.c_void_p),
                ("sb_bounds", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("obj", C.c_double), ("lb", C.c_double), ("gap", C.c_double),
                ("fft_obj", C.c_double), ("centers", C.c_int64 * 64), ("nodes", C.c_int64),
                ("passes", C.c_int64), ("evals", C.c_int64), ("n_active", C.c_int64),
                ("seconds", C.c_double), ("lb_kernel_ms", C.c_double),
                ("tighten_kernel_ms", C.c_double), ("tighten_evals", C.c_int64),
                ("seeds_found", C.c_int32), ("status", C.c_int32), ("sb_rows", C.c_int32),
                ("sb_nodes", C.c_int32), ("node_sr_tries", C.c_int64),
                ("node_sr_kept", C.c_int64), ("obj_kernel_ms", C.c_double),
                ("obj_evals", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libkc.so and declares every signature; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libkc.so not found at {path}: build it with `python -m paper_2301_00061_amd.build`")
    L = C.CDLL(path)
    P, vp = C.POINTER, C.c_void_p
    st = C.c_int
    L.kc_create.restype = st
    L.kc_create.argtypes = [P(vp), C.c_int, C.c_char_p]
    L.kc_destroy.restype = None
    L.kc_destroy.argtypes = [vp]
    L.kc_last_error.restype = C.c_char_p
    L.kc_last_error.argtypes = [vp]
    L.kc_rel_margin.restype = C.c_double
    L.kc_rel_margin.argtypes = [C.c_int]
    L.kc_abs_margin.restype = C.c_double
    L.kc_abs_margin.argtypes = [C.c_int]
    L.kc_lower_bound.restype = st
    L.kc_lower_bound.argtypes = [vp, P(Points), P(Nodes), vp, vp, vp, vp, vp]
    L.kc_lower_bound_noalloc.restype = st
    L.kc_lower_bound_noalloc.argtypes = [vp, P(Points), P(Nodes), vp, vp, vp, vp, vp]
    L.kc_objective.restype = st
    L.kc_objective.argtypes = [vp, P(Points), C.c_int32, C.c_int32, vp, C.c_int32, vp, vp, vp]
    L.kc_objective_screen.restype = st
    L.kc_objective_screen.argtypes = [vp, P(Points), C.c_int32, C.c_int32, vp, C.c_float, vp, vp,
                                      vp, vp]
    L.kc_fft.restype = st
    L.kc_fft.argtypes = [vp, P(Points), C.c_int32, C.c_int32, vp, vp, vp, vp]
    L.kc_tighten.restype = st
    L.kc_tighten.argtypes = [vp, P(Points), P(Nodes), C.c_double, P(Refs), vp, vp, vp, vp, vp,
                             vp, vp, vp, vp, vp]
    L.kc_reduce.restype = st
    L.kc_reduce.argtypes = [vp, P(Points), vp, P(Nodes), P(Refs), C.c_double, C.c_double, vp, vp,
                            vp, C.c_int64, vp, vp]
    L.kc_autotune.restype = st
    L.kc_autotune.argtypes = [vp, P(Points), P(Nodes), C.c_int32, P(C.c_double), vp]
    L.kc_autotune_tighten.restype = st
    L.kc_autotune_tighten.argtypes = [vp, P(Points), P(Nodes), C.c_double, P(Refs), P(C.c_double), vp]
    L.kc_mlp_forward.restype = st
    L.kc_mlp_forward.argtypes = [vp, vp, vp, C.c_int64, vp, vp, vp]
    L.kc_mlp_backward.restype = st
    L.kc_mlp_backward.argtypes = [vp, vp, vp, vp, vp, C.c_int64, vp, vp]
    L.kc_mlp_loss.restype = st
    L.kc_mlp_loss.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int64, vp, vp, vp]
    L.kc_mlp_adam.restype = st
    L.kc_mlp_adam.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int32, C.c_float, vp]
    L.kc_solve.restype = st
    L.kc_solve.argtypes = [vp, P(Points), P(Opts), P(Result)]
    _lib = L
    return L
