"""ctypes front end of the C search-and-fuse oracle (test infrastructure only).

The loop-fusion step (Sec. IV-D3; criteria in Sec. III-B) asks, for every map
point of the loop region and every covisible keyframe, whether the keyframe
already holds a keypoint that is close in the image and similar in
descriptor.  ``fl_oracle.c`` states the exact float32 definition; this module
only marshals NumPy arrays into it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def lib_path() -> str:
    return _LIB


def build_oracle(force: bool = False) -> str:
    """Compile the C oracle with strict IEEE float semantics (no contraction,
    no fast-math) so that every fmaf and every rounding is the written one."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-fno-builtin-popcount", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("win_px", ctypes.c_float), ("scale_factor", ctypes.c_float),
                ("n_octaves", ctypes.c_int32), ("grid_cols", ctypes.c_int32),
                ("grid_rows", ctypes.c_int32), ("hamming_th", ctypes.c_int32),
                ("nn_ratio", ctypes.c_float), ("flags", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is None:
        build_oracle()
        _lib = ctypes.CDLL(_LIB)
        _lib.orc_search_fuse.restype = ctypes.c_int
        _lib.orc_census_fp64.restype = ctypes.c_int
        _lib.orc_hamming256.restype = ctypes.c_int
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _params(p) -> _Params:
    return _Params(p.win_px, p.scale_factor, p.n_octaves, p.grid_cols, p.grid_rows,
                   p.hamming_th, p.nn_ratio, 0)


def _layout(src):
    """Event or Batch -> contiguous arrays plus the keyframe->event map."""
    if hasattr(src, "event_kf_offset"):
        ekf = np.asarray(src.event_kf_offset, np.int32)
        emp = np.ascontiguousarray(src.event_mp_offset, np.int32)
        kf_event = np.repeat(np.arange(len(ekf) - 1, dtype=np.int32), np.diff(ekf))
    else:
        emp = np.array([0, src.n_mp], np.int32)
        kf_event = np.zeros(src.n_kf, np.int32)
    c = np.ascontiguousarray
    return dict(
        n_kf=src.n_kf, kp_offset=c(src.kp_offset, np.int32), kp_xy=c(src.kp_xy, np.float32),
        kp_oct=c(src.kp_oct, np.int8), kp_desc=c(src.kp_desc, np.uint8),
        kp_owner=c(src.kp_owner, np.int32), kf_sim3=c(src.kf_sim3, np.float32),
        kf_cam=c(src.cams, np.float32), kf_event=c(kf_event, np.int32), event_mp_offset=emp,
        mp_xyz=c(src.mp_xyz, np.float32), mp_desc=c(src.mp_desc, np.uint8),
        mp_dmax=c(src.mp_dmax, np.float32), mp_id=c(src.mp_id, np.int32),
        pair_offset=c(src.pair_offset, np.int64),
        pair_mp=None if src.pair_mp is None else c(src.pair_mp, np.int32))


def search_fuse(src, params=None, use_grid: bool = False, use_dmax: bool = True,
                use_id: bool = True, overrides: dict | None = None):
    """Evaluate every pair of an Event or Batch.  Returns a dict with
    best_idx (i32), best_dist (i16), second_dist (i16), decision (u8),
    target (i32) and, for the grid variant, the counters n_visible,
    n_cells, n_kp_scanned, n_cand."""
    lib = _load()
    L = _layout(src)
    if overrides:
        L.update(overrides)
    P = _params(params if params is not None else src.params)
    n = int(L["pair_offset"][-1])
    out = dict(best_idx=np.empty(n, np.int32), best_dist=np.empty(n, np.int16),
               second_dist=np.empty(n, np.int16), decision=np.empty(n, np.uint8),
               target=np.empty(n, np.int32))
    cnt = np.zeros(4, np.int64)
    rc = lib.orc_search_fuse(
        ctypes.c_int(L["n_kf"]), _ptr(L["kp_offset"]), _ptr(L["kp_xy"]), _ptr(L["kp_oct"]),
        _ptr(L["kp_desc"]), _ptr(L["kp_owner"]), _ptr(L["kf_sim3"]), _ptr(L["kf_cam"]),
        _ptr(L["kf_event"]), _ptr(L["event_mp_offset"]), _ptr(L["mp_xyz"]), _ptr(L["mp_desc"]),
        _ptr(L["mp_dmax"]) if use_dmax else None, _ptr(L["mp_id"]) if use_id else None,
        _ptr(L["pair_offset"]), _ptr(L["pair_mp"]), ctypes.byref(P), ctypes.c_int(int(use_grid)),
        _ptr(out["best_idx"]), _ptr(out["best_dist"]), _ptr(out["second_dist"]),
        _ptr(out["decision"]), _ptr(out["target"]), _ptr(cnt))
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    if use_grid:
        out.update(n_visible=int(cnt[0]), n_cells=int(cnt[1]), n_kp_scanned=int(cnt[2]),
                   n_cand=int(cnt[3]))
    else:
        out.update(n_visible=int(cnt[0]))
    return out


def census_fp64(src, params=None, eps: float = 1e-3, overrides: dict | None = None):
    """FP64 boundary census of every valid, unobserved pair: a dict with
    n_diff (pairs whose float32 and float64 visibility, octave or candidate
    set differ), n_near_window (a keypoint within eps px of a window edge),
    n_near_image (the projection within eps px of an image edge) and n
    (pairs examined)."""
    lib = _load()
    L = _layout(src)
    if overrides:
        L.update(overrides)
    P = _params(params if params is not None else src.params)
    out = np.zeros(4, np.int64)
    rc = lib.orc_census_fp64(
        ctypes.c_int(L["n_kf"]), _ptr(L["kp_offset"]), _ptr(L["kp_xy"]), _ptr(L["kp_oct"]),
        _ptr(L["kp_owner"]), _ptr(L["kf_sim3"]), _ptr(L["kf_cam"]), _ptr(L["kf_event"]),
        _ptr(L["event_mp_offset"]), _ptr(L["mp_xyz"]), _ptr(L["mp_dmax"]), _ptr(L["mp_id"]),
        _ptr(L["pair_offset"]), _ptr(L["pair_mp"]), ctypes.byref(P), ctypes.c_double(eps),
        _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    return dict(n_diff=int(out[0]), n_near_window=int(out[1]), n=int(out[2]), n_near_image=int(out[3]))


def hamming256(a: np.ndarray, b: np.ndarray) -> int:
    lib = _load()
    a = np.ascontiguousarray(a, np.uint8)
    b = np.ascontiguousarray(b, np.uint8)
    assert a.size == 32 and b.size == 32
    return int(lib.orc_hamming256(_ptr(a), _ptr(b)))


def project(X, S16, cam8, dmax=None, params=None):
    """Float32 projection of points X [n,3] through one keyframe transform
    (``[sR, t, 1/s, pad]``) and camera row: (u, v, d, pred, visible)."""
    lib = _load()
    from synth import LoopParams  # parameters container only
    P = _params(params if params is not None else LoopParams())
    X = np.ascontiguousarray(X, np.float32).reshape(-1, 3)
    S16 = np.ascontiguousarray(S16, np.float32)
    cam8 = np.ascontiguousarray(cam8, np.float32)
    n = len(X)
    u = np.empty(n, np.float32)
    v = np.empty(n, np.float32)
    d = np.empty(n, np.float32)
    pred = np.empty(n, np.int32)
    vis = np.empty(n, np.uint8)
    dm = None if dmax is None else np.ascontiguousarray(dmax, np.float32)
    lib.orc_project.restype = ctypes.c_int
    rc = lib.orc_project(ctypes.c_int(n), _ptr(X), _ptr(S16), _ptr(cam8), _ptr(dm), ctypes.byref(P),
                         _ptr(u), _ptr(v), _ptr(d), _ptr(pred), _ptr(vis))
    if rc != 0:
        raise ValueError("oracle rejected the parameters")
    return u, v, d, pred, vis.astype(bool)


def build_grid(xy, cam8, params):
    """(cell_start [C*R+1], cell_kp [n]) of one keyframe's keypoints."""
    lib = _load()
    xy = np.ascontiguousarray(xy, np.float32).reshape(-1, 2)
    C, R = int(params.grid_cols), int(params.grid_rows)
    cs = np.empty(C * R + 1, np.int32)
    ck = np.empty(max(len(xy), 1), np.int32)
    lib.orc_build_grid.restype = ctypes.c_int
    rc = lib.orc_build_grid(ctypes.c_int(len(xy)), _ptr(xy), ctypes.c_int(C), ctypes.c_int(R),
                            ctypes.c_float(float(cam8[4])), ctypes.c_float(float(cam8[5])), _ptr(cs), _ptr(ck))
    if rc != 0:
        raise ValueError("oracle rejected the grid")
    return cs, ck[: len(xy)]
