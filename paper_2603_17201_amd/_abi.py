"""ctypes declarations of the fastloop C ABI (``include/fastloop.h``)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfastloop.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_float = ctypes.c_float
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_char_p = ctypes.c_char_p

FL_OK, FL_EINVAL, FL_ENOMEM, FL_EHIP, FL_ERANGE, FL_ENOTSUP = 0, -1, -2, -3, -4, -5
NOT_VISIBLE, NO_MATCH, ADD, FUSE, SKIP, INVALID = 0, 1, 2, 3, 4, 5
NO_DIST = 0x7FFF
MAX_KP = 65535


class Sim3(ctypes.Structure):
    _fields_ = [("sR", c_float * 9), ("t", c_float * 3), ("inv_s", c_float), ("pad", c_float * 3)]


class Pinhole(ctypes.Structure):
    _fields_ = [("fx", c_float), ("fy", c_float), ("cx", c_float), ("cy", c_float),
                ("width", c_float), ("height", c_float), ("pad", c_float * 2)]


class Params(ctypes.Structure):
    _fields_ = [("win_px", c_float), ("scale_factor", c_float), ("n_octaves", c_int32),
                ("grid_cols", c_int32), ("grid_rows", c_int32), ("hamming_th", c_int32),
                ("nn_ratio", c_float), ("flags", c_int32)]


class FuseOut(ctypes.Structure):
    _fields_ = [("best_idx", c_void_p), ("best_dist", c_void_p), ("second_dist", c_void_p),
                ("decision", c_void_p), ("target", c_void_p)]


class Keyframe(ctypes.Structure):
    _fields_ = [("n_kp", c_int32), ("kp_xy", c_void_p), ("kp_octave", c_void_p), ("kp_desc", c_void_p),
                ("kp_owner", c_void_p), ("cell_start", c_void_p), ("cell_kp", c_void_p)]


class Batch(ctypes.Structure):
    _fields_ = [("n_events", c_int32), ("n_kf", c_int32), ("n_mp", c_int32), ("n_kp_total", c_int32),
                ("n_pairs", c_int64),
                ("event_kf_offset", c_void_p), ("event_mp_offset", c_void_p), ("kp_offset", c_void_p),
                ("pair_offset", c_void_p), ("kf_sim3", c_void_p), ("kf_K", c_void_p), ("kf_T", c_void_p),
                ("pair_mp", c_void_p),
                ("kp_xy", c_void_p), ("kp_octave", c_void_p), ("kp_desc", c_void_p), ("kp_owner", c_void_p),
                ("mp_xyz", c_void_p), ("mp_desc", c_void_p), ("mp_dmax", c_void_p), ("mp_id", c_void_p)]


MAX_PASSES = 4   # FL_MAX_PASSES


class Pass(ctypes.Structure):
    _fields_ = [("kf_sim3", c_void_p), ("params", Params), ("out", FuseOut)]


class PoseGraph(ctypes.Structure):
    _fields_ = [("n_nodes", c_int32), ("n_edges", c_int32), ("S", c_void_p), ("M", c_void_p), ("edges", c_void_p),
                ("fixed", c_void_p)]


class PgoParams(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("cg_iters", c_int32), ("lam", c_double), ("cg_tol", c_double),
                ("cost", c_void_p), ("cg_used", c_void_p), ("lambdas", c_void_p), ("accepted", c_void_p),
                ("solver", c_int32), ("reserved", c_int32)]


PGO_MAX_BAND_NODES = 64   # FL_PGO_MAX_BAND_NODES
PGO_SOLVER_AUTO, PGO_SOLVER_CG, PGO_SOLVER_DIRECT, PGO_SOLVER_DIRECT_WIDE = 0, 1, 2, 3


class RefineInverse(ctypes.Structure):
    _fields_ = [("event_offset", c_void_p), ("xyz", c_void_p), ("uv", c_void_p), ("kf_idx", c_void_p),
                ("kf_T", c_void_p), ("kf_cam", c_void_p), ("n_kf", c_int32), ("flags", c_int32)]


class Refine(ctypes.Structure):
    _fields_ = [("n_iters", c_int32), ("huber_delta", c_float), ("event_S", c_void_p),
                ("event_S32", c_void_p), ("event_n_matched", c_void_p), ("n_rounds", c_int32),
                ("outlier_px", c_float), ("lm_lambda", c_float), ("flags", c_int32),
                ("inverse", ctypes.POINTER(RefineInverse))]


class Tuning(ctypes.Structure):
    _fields_ = [("pairs_per_lane", c_int32), ("lds_mode", c_int32), ("wg_per_cu", c_int32),
                ("xcd_aware", c_int32)]


# (name, restype, argtypes) of every exported function
PROF_SEARCH = 0   # FL_PROF_SEARCH
PROF_REFINE = 1   # FL_PROF_REFINE

SIGNATURES = [
    ("fl_create", c_int32, [ctypes.POINTER(c_void_p), c_int32]),
    ("fl_destroy", None, [c_void_p]),
    ("fl_last_error", c_char_p, []),
    ("fl_version", c_int32, []),
    ("fl_build_grid", c_int32, [c_void_p, c_int32, c_void_p, ctypes.POINTER(Pinhole), ctypes.POINTER(Params),
                                c_void_p, c_void_p, c_void_p]),
    ("fl_search_fuse", c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                 ctypes.POINTER(Keyframe), ctypes.POINTER(Sim3), ctypes.POINTER(Pinhole),
                                 ctypes.POINTER(Params), ctypes.POINTER(FuseOut), c_void_p]),
    ("fl_search_fuse_noalloc", c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(Keyframe),
                                         ctypes.POINTER(Sim3), ctypes.POINTER(Pinhole), ctypes.POINTER(Params),
                                         ctypes.POINTER(FuseOut), c_void_p]),
    ("fl_validate_batch", c_int32, [ctypes.POINTER(Batch), ctypes.POINTER(Params), ctypes.POINTER(FuseOut)]),
    ("fl_search_fuse_batched", c_int32, [c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(Params),
                                         ctypes.POINTER(FuseOut), ctypes.POINTER(Refine), c_void_p]),
    ("fl_search_fuse_passes", c_int32, [c_void_p, ctypes.POINTER(Batch), c_int32, ctypes.POINTER(Pass), c_void_p]),
    ("fl_search_fuse_graph_launch", c_int32, [c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(Params),
                                              ctypes.POINTER(FuseOut), ctypes.POINTER(Refine), c_void_p]),
    ("fl_refine_events", c_int32, [c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(FuseOut),
                                   ctypes.POINTER(Refine), c_void_p]),
    ("fl_reproj_residual_fwd", c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                         c_void_p, ctypes.POINTER(Pinhole), c_float, c_void_p, c_void_p,
                                         c_void_p, c_void_p]),
    ("fl_reproj_residual_bwd", c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                         c_void_p, ctypes.POINTER(Pinhole), c_float, c_double, c_void_p,
                                         c_void_p, c_void_p]),
    ("fl_reproj_residual_bwd_inv", c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                             c_void_p, ctypes.POINTER(Pinhole), c_float, c_double, c_void_p,
                                             c_void_p, c_void_p]),
    ("fl_pose_graph_optimize", c_int32, [c_void_p, ctypes.POINTER(PoseGraph), ctypes.POINTER(PgoParams), c_void_p]),
    ("fl_sim3_inverse", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("fl_sim3_exp_mul", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("fl_sim3_grad_xi", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("fl_gn_step", c_int32, [c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
    ("fl_get_tuning", c_int32, [c_void_p, ctypes.POINTER(Tuning)]),
    ("fl_set_tuning", c_int32, [c_void_p, ctypes.POINTER(Tuning)]),
    ("fl_autotune", c_int32, [c_void_p, ctypes.POINTER(Batch), ctypes.POINTER(Params), ctypes.POINTER(FuseOut),
                              c_int32, ctypes.POINTER(Tuning), ctypes.POINTER(c_float), c_void_p]),
    ("fl_set_stats", c_int32, [c_void_p, c_int32]),
    ("fl_get_stats", c_int32, [c_void_p, ctypes.POINTER(c_int64)]),
    ("fl_set_profiling", c_int32, [c_void_p, c_int32]),
    ("fl_get_profile", c_int32, [c_void_p, c_int32, ctypes.POINTER(c_double), ctypes.POINTER(c_int64)]),
    ("fl_valu_rate", c_int32, [c_void_p, c_int32, ctypes.POINTER(c_double), c_void_p]),
    ("fl_debug_set_list_cap", c_int32, [c_void_p, c_int32]),
    ("fl_debug_refine_tag", ctypes.c_uint32, [ctypes.c_uint32, c_int32]),
    ("fl_debug_refine_rows_cleared", c_int32, [ctypes.c_uint32]),
]

_lib = None


def load(path: str = LIB_PATH):
    """Load the built library.  There is no fallback: without it every entry
    point of this package raises."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing; build it with `python -m paper_2603_17201_amd.build`")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    msg = load().fl_last_error()
    return msg.decode() if msg else ""
