"""Python binding of the fastloop C ABI: argument marshalling only.

Device arrays are torch tensors (PyTorch provides device memory and streams);
small host tables are NumPy arrays.  Every computation runs in the HIP
library; nothing here falls back to the CPU.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _abi
from ._abi import (Batch, FuseOut, Keyframe, Params, Pass, PgoParams, Pinhole, PoseGraph, Refine, RefineInverse,
                   Sim3, Tuning)


class FlError(ValueError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


def _check(rc: int, what: str):
    if rc != 0:
        raise FlError(rc, f"{what} failed ({rc}): {_abi.last_error()}")


def _ptr(t: Optional[torch.Tensor], dtype, name: str, align: int = 4, device=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.data_ptr() % align:
        raise ValueError(f"{name} must be {align}-byte aligned")
    return ctypes.c_void_p(t.data_ptr())


def _host(a, dtype, name):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def params_struct(p) -> Params:
    """Any object with win_px, scale_factor, n_octaves, grid_cols, grid_rows,
    hamming_th, nn_ratio (e.g. a dataclass) -> fl_params."""
    return Params(float(p.win_px), float(p.scale_factor), int(p.n_octaves), int(p.grid_cols),
                  int(p.grid_rows), int(p.hamming_th), float(p.nn_ratio), 0)


def sim3_struct(v) -> Sim3:
    v = np.asarray(v, np.float32).reshape(-1)
    s = Sim3()
    for i in range(9):
        s.sR[i] = float(v[i])
    for i in range(3):
        s.t[i] = float(v[9 + i])
    s.inv_s = float(v[12])
    return s


def pinhole_struct(v) -> Pinhole:
    v = np.asarray(v, np.float32).reshape(-1)
    return Pinhole(float(v[0]), float(v[1]), float(v[2]), float(v[3]), float(v[4]), float(v[5]))


@dataclass
class FuseOutputs:
    best_idx: torch.Tensor
    best_dist: torch.Tensor
    second_dist: torch.Tensor
    decision: torch.Tensor
    target: torch.Tensor

    @classmethod
    def empty(cls, n: int, device) -> "FuseOutputs":
        return cls(torch.empty(n, dtype=torch.int32, device=device),
                   torch.empty(n, dtype=torch.int16, device=device),
                   torch.empty(n, dtype=torch.int16, device=device),
                   torch.empty(n, dtype=torch.uint8, device=device),
                   torch.empty(n, dtype=torch.int32, device=device))

    def __setattr__(self, name, value):
        # rebinding an array drops the cached fl_fuse_out
        object.__setattr__(self, "_struct", None)
        object.__setattr__(self, name, value)

    def struct(self) -> FuseOut:
        """The fl_fuse_out of these arrays, built once and reused (a call
        then allocates no Python objects for it)."""
        st = self.__dict__.get("_struct")
        if st is None:
            dev = self.best_idx.device
            st = FuseOut(_ptr(self.best_idx, torch.int32, "best_idx", device=dev),
                         _ptr(self.best_dist, torch.int16, "best_dist", 2, dev),
                         _ptr(self.second_dist, torch.int16, "second_dist", 2, dev),
                         _ptr(self.decision, torch.uint8, "decision", 1, dev),
                         _ptr(self.target, torch.int32, "target", device=dev))
            object.__setattr__(self, "_struct", st)
        return st

    def numpy(self) -> dict:
        return {k: getattr(self, k).cpu().numpy() for k in
                ("best_idx", "best_dist", "second_dist", "decision", "target")}


class DeviceBatch:
    """A batch of loop events resident in HBM plus its host tables.

    Build it from any object exposing the array attributes of a batch
    (event_kf_offset, event_mp_offset, cams, kf_sim3, kf_T, mp_xyz, mp_desc,
    mp_dmax, mp_id, kp_offset, kp_xy, kp_oct, kp_desc, kp_owner, pair_offset,
    pair_mp) or of a single event (the same without the event offsets)."""

    def __init__(self, src, device="cuda:0", use_dmax: bool = True, use_id: bool = True):
        dev = torch.device(device)
        self.device = dev
        n_kf = int(np.asarray(src.kp_offset).shape[0] - 1)
        n_mp = int(np.asarray(src.mp_xyz).shape[0])
        if hasattr(src, "event_kf_offset"):
            ekf = np.asarray(src.event_kf_offset, np.int32)
            emp = np.asarray(src.event_mp_offset, np.int32)
        else:
            ekf = np.array([0, n_kf], np.int32)
            emp = np.array([0, n_mp], np.int32)
        self.h_event_kf_offset = np.ascontiguousarray(ekf)
        self.h_event_mp_offset = np.ascontiguousarray(emp)
        self.h_kp_offset = np.ascontiguousarray(src.kp_offset, np.int32)
        self.h_pair_offset = np.ascontiguousarray(src.pair_offset, np.int64)
        self.h_kf_sim3 = np.ascontiguousarray(src.kf_sim3, np.float32).reshape(n_kf, 16)
        self.h_kf_K = np.ascontiguousarray(src.cams, np.float32).reshape(n_kf, 8)
        kf_T = getattr(src, "kf_T", None)
        self.h_kf_T = None if kf_T is None else np.ascontiguousarray(kf_T, np.float32).reshape(n_kf, 12)

        def up(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a)).to(dev).view(dt) if a is not None else None

        self.kp_xy = up(np.asarray(src.kp_xy, np.float32).reshape(-1, 2), torch.float32)
        self.kp_oct = up(np.asarray(src.kp_oct, np.int8), torch.int8)
        self.kp_desc = up(np.asarray(src.kp_desc, np.uint8).reshape(-1, 32), torch.uint8)
        self.kp_owner = up(np.asarray(src.kp_owner, np.int32), torch.int32)
        self.mp_xyz = up(np.asarray(src.mp_xyz, np.float32).reshape(-1, 3), torch.float32)
        self.mp_desc = up(np.asarray(src.mp_desc, np.uint8).reshape(-1, 32), torch.uint8)
        self.mp_dmax = up(np.asarray(src.mp_dmax, np.float32), torch.float32) if use_dmax else None
        self.mp_id = up(np.asarray(src.mp_id, np.int32), torch.int32) if use_id else None
        pm = getattr(src, "pair_mp", None)
        self.pair_mp = None if pm is None else up(np.asarray(pm, np.int32), torch.int32)
        self.n_events = len(ekf) - 1
        self.n_kf = n_kf
        self.n_mp = n_mp
        self.n_kp_total = int(self.h_kp_offset[-1])
        self.n_pairs = int(self.h_pair_offset[-1])

    def __setattr__(self, name, value):
        # rebinding an array drops the cached fl_batch structs
        object.__setattr__(self, "_structs", {})
        object.__setattr__(self, name, value)

    def struct(self, with_T: bool = True) -> Batch:
        """The fl_batch of this batch, built once per with_T and reused."""
        b = self.__dict__.get("_structs", {}).get(with_T)
        if b is None:
            b = self._make_struct(with_T)
            self.__dict__.setdefault("_structs", {})[with_T] = b
        return b

    def _make_struct(self, with_T: bool) -> Batch:
        d = self.device
        b = Batch()
        b.n_events, b.n_kf, b.n_mp, b.n_kp_total, b.n_pairs = (self.n_events, self.n_kf, self.n_mp,
                                                               self.n_kp_total, self.n_pairs)
        b.event_kf_offset = self.h_event_kf_offset.ctypes.data_as(ctypes.c_void_p)
        b.event_mp_offset = self.h_event_mp_offset.ctypes.data_as(ctypes.c_void_p)
        b.kp_offset = self.h_kp_offset.ctypes.data_as(ctypes.c_void_p)
        b.pair_offset = self.h_pair_offset.ctypes.data_as(ctypes.c_void_p)
        b.kf_sim3 = self.h_kf_sim3.ctypes.data_as(ctypes.c_void_p)
        b.kf_K = self.h_kf_K.ctypes.data_as(ctypes.c_void_p)
        b.kf_T = (self.h_kf_T.ctypes.data_as(ctypes.c_void_p) if (with_T and self.h_kf_T is not None) else None)
        b.pair_mp = _ptr(self.pair_mp, torch.int32, "pair_mp", device=d)
        b.kp_xy = _ptr(self.kp_xy, torch.float32, "kp_xy", device=d)
        b.kp_octave = _ptr(self.kp_oct, torch.int8, "kp_oct", 1, d)
        b.kp_desc = _ptr(self.kp_desc, torch.uint8, "kp_desc", 16, d)
        b.kp_owner = _ptr(self.kp_owner, torch.int32, "kp_owner", device=d)
        b.mp_xyz = _ptr(self.mp_xyz, torch.float32, "mp_xyz", device=d)
        b.mp_desc = _ptr(self.mp_desc, torch.uint8, "mp_desc", 16, d)
        b.mp_dmax = _ptr(self.mp_dmax, torch.float32, "mp_dmax", device=d)
        b.mp_id = _ptr(self.mp_id, torch.int32, "mp_id", device=d)
        return b


class InversePairs:
    """The other direction of a loop's matches for two-sided refinement:
    points of the current side (xyz, float32 [n,3]) observed in loop-side
    keyframes (uv float32 [n,2], kf_idx int32 [n] into kf_T float32
    [n_kf,12] and kf_cam float32 [n_kf,4] = fx, fy, cx, cy), all device
    tensors, with event_offset (host, int64 [n_events+1]) giving each event's
    pairs."""

    def __init__(self, event_offset, xyz, uv, kf_idx, kf_T, kf_cam):
        self.event_offset = np.ascontiguousarray(event_offset, dtype=np.int64)
        self.xyz, self.uv, self.kf_idx, self.kf_T, self.kf_cam = xyz, uv, kf_idx, kf_T, kf_cam

    def struct(self, device) -> RefineInverse:
        n_kf = int(self.kf_T.shape[0]) if self.kf_T is not None else 0
        inv = RefineInverse(self.event_offset.ctypes.data_as(ctypes.c_void_p),
                            _ptr(self.xyz, torch.float32, "inverse.xyz", 16, device),
                            _ptr(self.uv, torch.float32, "inverse.uv", 8, device),
                            _ptr(self.kf_idx, torch.int32, "inverse.kf_idx", device=device),
                            _ptr(self.kf_T, torch.float32, "inverse.kf_T", device=device),
                            _ptr(self.kf_cam, torch.float32, "inverse.kf_cam", 16, device), n_kf, 0)
        inv._keep = self.event_offset
        return inv


class Context:
    """An fl_ctx: workspace, pinned staging and captured graphs of one device."""

    def __init__(self, device: int = 0):
        self._lib = _abi.load()
        self.device = torch.device("cuda", device)
        self._h = ctypes.c_void_p()
        _check(self._lib.fl_create(ctypes.byref(self._h), device), "fl_create")

    def close(self):
        if self._h:
            self._lib.fl_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def _stream(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(s.cuda_stream)

    # -- grid ------------------------------------------------------------
    def build_grid(self, kp_xy: torch.Tensor, cam8, params, stream=None):
        n = int(kp_xy.shape[0])
        cells = int(params.grid_cols) * int(params.grid_rows)
        cs = torch.empty(cells + 1, dtype=torch.int32, device=self.device)
        ck = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        K = pinhole_struct(cam8)
        P = params_struct(params)
        _check(self._lib.fl_build_grid(self._h, n, _ptr(kp_xy, torch.float32, "kp_xy", device=self.device),
                                       ctypes.byref(K), ctypes.byref(P), _ptr(cs, torch.int32, "cell_start"),
                                       _ptr(ck, torch.int32, "cell_kp"), self._stream(stream)), "fl_build_grid")
        return cs, ck[:n]

    # -- plain per-keyframe search ----------------------------------------
    def search_fuse(self, mp_xyz, mp_desc, mp_dmax, mp_id, kp_xy, kp_oct, kp_desc, kp_owner, sim3_16, cam8,
                    params, grid=None, out: Optional[FuseOutputs] = None, stream=None) -> FuseOutputs:
        d = self.device
        n = int(mp_xyz.shape[0])
        if out is None:
            out = FuseOutputs.empty(n, d)
        kf = Keyframe(int(kp_xy.shape[0]), _ptr(kp_xy, torch.float32, "kp_xy", device=d),
                      _ptr(kp_oct, torch.int8, "kp_oct", 1, d), _ptr(kp_desc, torch.uint8, "kp_desc", 16, d),
                      _ptr(kp_owner, torch.int32, "kp_owner", device=d),
                      _ptr(grid[0], torch.int32, "cell_start", device=d) if grid is not None else None,
                      _ptr(grid[1], torch.int32, "cell_kp", device=d) if grid is not None else None)
        S = sim3_struct(sim3_16)
        K = pinhole_struct(cam8)
        P = params_struct(params)
        o = out.struct()
        _check(self._lib.fl_search_fuse(self._h, n, _ptr(mp_xyz, torch.float32, "mp_xyz", device=d),
                                        _ptr(mp_desc, torch.uint8, "mp_desc", 16, d),
                                        _ptr(mp_dmax, torch.float32, "mp_dmax", device=d),
                                        _ptr(mp_id, torch.int32, "mp_id", device=d), ctypes.byref(kf),
                                        ctypes.byref(S), ctypes.byref(K), ctypes.byref(P), ctypes.byref(o),
                                        self._stream(stream)), "fl_search_fuse")
        return out

    # -- batched search ----------------------------------------------------
    def search_fuse_batched(self, batch: DeviceBatch, params, out: Optional[FuseOutputs] = None, refine=None,
                            stream=None) -> FuseOutputs:
        """refine: None or (n_iters, huber_delta, event_S, event_S32, n_matched)
        as for search_fuse_graph."""
        if out is None:
            out = FuseOutputs.empty(batch.n_pairs, self.device)
        b = batch.struct()
        P = params_struct(params)
        o = out.struct()
        r, rp = self._refine_struct(batch, refine)
        _check(self._lib.fl_search_fuse_batched(self._h, ctypes.byref(b), ctypes.byref(P), ctypes.byref(o), rp,
                                                self._stream(stream)), "fl_search_fuse_batched")
        return out

    def search_fuse_passes(self, batch: DeviceBatch, passes, stream=None) -> list:
        """Several searches of one resident batch in one launch.  passes: a
        sequence of (params, kf_sim3, out): kf_sim3 is None (the batch's) or a
        host array [n_kf, 16] in the batch's kf_sim3 form; out is a
        FuseOutputs or None (allocated).  Returns the outputs of every pass."""
        n = len(passes)
        arr = (Pass * max(n, 1))()
        keep, outs = [], []
        for i, (params, kf_sim3, out) in enumerate(passes):
            if out is None:
                out = FuseOutputs.empty(batch.n_pairs, self.device)
            outs.append(out)
            arr[i].params = params_struct(params)
            arr[i].out = out.struct()
            if kf_sim3 is not None:
                a = np.ascontiguousarray(kf_sim3, np.float32).reshape(batch.n_kf, 16)
                keep.append(a)
                arr[i].kf_sim3 = a.ctypes.data_as(ctypes.c_void_p)
        _check(self._lib.fl_search_fuse_passes(self._h, ctypes.byref(batch.struct()), n, arr, self._stream(stream)),
               "fl_search_fuse_passes")
        return outs

    def _refine_struct(self, batch, refine):
        """refine: (n_iters, huber_delta, event_S, event_S32, n_matched),
        optionally (n_rounds, outlier_px, lm_lambda) for robust refinement,
        and optionally an InversePairs (two-sided refinement) as the ninth
        element."""
        if refine is None:
            return None, None
        n_iters, delta, event_S, event_S32, n_matched = refine[:5]
        n_rounds, outlier_px, lm_lambda = (tuple(refine[5:8]) + (0, 0.0, 0.0)[len(refine[5:8]):])
        inverse = refine[8] if len(refine) > 8 else None
        r = Refine(int(n_iters), float(delta),
                   _ptr(event_S, torch.float64, "event_S", 8, self.device),
                   _ptr(event_S32, torch.float32, "event_S32", 16, self.device),
                   _ptr(n_matched, torch.int32, "event_n_matched", device=self.device),
                   int(n_rounds), float(outlier_px), float(lm_lambda), 0)
        if inverse is not None:
            inv = inverse.struct(self.device)
            r.inverse = ctypes.pointer(inv)
            r._keep = inv
        return r, ctypes.byref(r)

    def search_fuse_graph(self, batch: DeviceBatch, params, out: Optional[FuseOutputs] = None, refine=None,
                          stream=None) -> FuseOutputs:
        """refine: None or (n_iters, huber_delta, event_S f64 [n_events,13] (in/out),
        event_S32 f32 [n_events,16] or None, n_matched i32 [n_events] or None)."""
        if out is None:
            out = FuseOutputs.empty(batch.n_pairs, self.device)
        b = batch.struct()
        P = params_struct(params)
        o = out.struct()
        r, rp = self._refine_struct(batch, refine)
        _check(self._lib.fl_search_fuse_graph_launch(self._h, ctypes.byref(b), ctypes.byref(P), ctypes.byref(o),
                                                     rp, self._stream(stream)), "fl_search_fuse_graph_launch")
        return out

    def refine_events(self, batch: DeviceBatch, out: FuseOutputs, refine, stream=None):
        b = batch.struct()
        o = out.struct()
        r, rp = self._refine_struct(batch, refine)
        _check(self._lib.fl_refine_events(self._h, ctypes.byref(b), ctypes.byref(o), rp, self._stream(stream)),
               "fl_refine_events")

    # -- residual -------------------------------------------------------
    def _res_common(self, xyz, uv, kf_idx, kf_T, S32):
        d = self.device
        n = int(xyz.shape[0])
        n_kf = int(kf_T.shape[0]) if kf_T is not None else (1 if kf_idx is not None else 0)
        return (n, _ptr(xyz, torch.float32, "xyz", device=d), _ptr(uv, torch.float32, "uv", device=d),
                _ptr(kf_idx, torch.int32, "kf_idx", device=d), n_kf, _ptr(kf_T, torch.float32, "kf_T", device=d),
                _ptr(S32, torch.float32, "S32", 16, d))

    def residual_fwd(self, xyz, uv, kf_idx, kf_T, S32, cam8, delta, want_r: bool = True, stream=None):
        n, px, pu, pk, nkf, pT, pS = self._res_common(xyz, uv, kf_idx, kf_T, S32)
        r = torch.empty((n, 2), dtype=torch.float32, device=self.device) if want_r else None
        w = torch.empty(n, dtype=torch.float32, device=self.device) if want_r else None
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        K = pinhole_struct(cam8)
        _check(self._lib.fl_reproj_residual_fwd(self._h, n, px, pu, pk, nkf, pT, pS, ctypes.byref(K),
                                                float(delta), _ptr(r, torch.float32, "r"),
                                                _ptr(w, torch.float32, "w"), _ptr(loss, torch.float64, "loss", 8),
                                                self._stream(stream)), "fl_reproj_residual_fwd")
        return r, w, loss

    def residual_bwd(self, xyz, uv, kf_idx, kf_T, S32, cam8, delta, grad_scale: float = 1.0, want_H: bool = True,
                     inverse: bool = False, stream=None):
        """inverse: the pairs are observed through S^-1 and S32 is the float32
        form of S^-1 (fl_reproj_residual_bwd_inv); g and H are still with
        respect to S."""
        n, px, pu, pk, nkf, pT, pS = self._res_common(xyz, uv, kf_idx, kf_T, S32)
        g = torch.empty(7, dtype=torch.float64, device=self.device)
        H = torch.empty(28, dtype=torch.float64, device=self.device) if want_H else None
        K = pinhole_struct(cam8)
        name = "fl_reproj_residual_bwd_inv" if inverse else "fl_reproj_residual_bwd"
        _check(getattr(self._lib, name)(self._h, n, px, pu, pk, nkf, pT, pS, ctypes.byref(K), float(delta),
                                        float(grad_scale), _ptr(g, torch.float64, "g", 8),
                                        _ptr(H, torch.float64, "H", 8), self._stream(stream)), name)
        return g, H

    def pose_graph_optimize(self, S, M, edges, fixed=None, iters: int = 10, cg_iters: int = 500, lam: float = 1e-4,
                            cg_tol: float = 1e-10, solver: int = 0, history: bool = False, stream=None):
        """Essential-graph optimisation in place (Levenberg-Marquardt from
        damping lam; lam = 0: Gauss-Newton): S device float64 [n, 13],
        M device float64 [E, 13], edges host int32 [E, 2], fixed host bool
        [n] or None (node 0 held); solver 0 (direct when the reordered band
        fits, else conjugate gradients), 1 (conjugate gradients), 2
        (direct) or 3 (direct through the device-memory window, which wider
        bands take anyway).  Returns (cost [iters + 1], cg_used [iters], 0 for a
        direct solve) as device tensors, and with history=True also
        (lambdas [iters], accepted [iters])."""
        n = int(S.shape[0])
        e = np.ascontiguousarray(edges, np.int32).reshape(-1, 2)
        fx = None if fixed is None else np.ascontiguousarray(fixed, np.uint8).reshape(n)
        cost = torch.empty(iters + 1, dtype=torch.float64, device=self.device)
        used = torch.empty(max(iters, 1), dtype=torch.int32, device=self.device)
        lams = torch.empty(max(iters, 1), dtype=torch.float64, device=self.device)
        acc = torch.empty(max(iters, 1), dtype=torch.uint8, device=self.device)
        G = PoseGraph(n, int(e.shape[0]), _ptr(S, torch.float64, "S", 8, self.device),
                      _ptr(M, torch.float64, "M", 8, self.device), e.ctypes.data_as(ctypes.c_void_p),
                      None if fx is None else fx.ctypes.data_as(ctypes.c_void_p))
        Pp = PgoParams(int(iters), int(cg_iters), float(lam), float(cg_tol),
                       _ptr(cost, torch.float64, "cost", 8, self.device), _ptr(used, torch.int32, "cg_used"),
                       _ptr(lams, torch.float64, "lambdas", 8, self.device), _ptr(acc, torch.uint8, "accepted", 1),
                       int(solver), 0)
        _check(self._lib.fl_pose_graph_optimize(self._h, ctypes.byref(G), ctypes.byref(Pp), self._stream(stream)),
               "fl_pose_graph_optimize")
        if history:
            return cost, used[:iters], lams[:iters], acc[:iters]
        return cost, used[:iters]

    def sim3_inverse(self, S_in, S_out=None, S32=None, stream=None):
        """S^-1 in float64 and its float32 form (device tensors)."""
        if S_out is None:
            S_out = torch.empty(13, dtype=torch.float64, device=self.device)
        if S32 is None:
            S32 = torch.empty(16, dtype=torch.float32, device=self.device)
        _check(self._lib.fl_sim3_inverse(self._h, _ptr(S_in, torch.float64, "S_in", 8),
                                         _ptr(S_out, torch.float64, "S_out", 8), _ptr(S32, torch.float32, "S32", 16),
                                         self._stream(stream)), "fl_sim3_inverse")
        return S_out, S32

    def sim3_exp_mul(self, xi, S_in, S_out=None, S32=None, stream=None):
        if S_out is None:
            S_out = torch.empty(13, dtype=torch.float64, device=self.device)
        if S32 is None:
            S32 = torch.empty(16, dtype=torch.float32, device=self.device)
        _check(self._lib.fl_sim3_exp_mul(self._h, _ptr(xi, torch.float64, "xi", 8), _ptr(S_in, torch.float64, "S_in", 8),
                                         _ptr(S_out, torch.float64, "S_out", 8), _ptr(S32, torch.float32, "S32", 16),
                                         self._stream(stream)), "fl_sim3_exp_mul")
        return S_out, S32

    def sim3_grad_xi(self, xi, g, scale=None, out=None, stream=None):
        """scale * J_l(xi)^T g: the gradient with respect to xi of S = exp(xi) S0
        from the left-perturbation gradient g at S (device float64 tensors)."""
        if out is None:
            out = torch.empty(7, dtype=torch.float64, device=self.device)
        _check(self._lib.fl_sim3_grad_xi(self._h, _ptr(xi, torch.float64, "xi", 8), _ptr(g, torch.float64, "g", 8),
                                         _ptr(scale, torch.float64, "scale", 8), _ptr(out, torch.float64, "out", 8),
                                         self._stream(stream)), "fl_sim3_grad_xi")
        return out

    def gn_step(self, g, H, S, S32=None, lam: float = 0.0, stream=None):
        _check(self._lib.fl_gn_step(self._h, _ptr(g, torch.float64, "g", 8), _ptr(H, torch.float64, "H", 8),
                                    float(lam), _ptr(S, torch.float64, "S", 8), _ptr(S32, torch.float32, "S32", 16),
                                    self._stream(stream)), "fl_gn_step")
        return S, S32

    # -- tuning / stats -------------------------------------------------
    def get_tuning(self) -> Tuning:
        t = Tuning()
        _check(self._lib.fl_get_tuning(self._h, ctypes.byref(t)), "fl_get_tuning")
        return t

    def set_tuning(self, pairs_per_lane=1, lds_mode=2, wg_per_cu=1, xcd_aware=1):
        t = Tuning(pairs_per_lane, lds_mode, wg_per_cu, xcd_aware)
        _check(self._lib.fl_set_tuning(self._h, ctypes.byref(t)), "fl_set_tuning")

    def autotune(self, batch: DeviceBatch, params, out: FuseOutputs, reps: int = 3, stream=None):
        b = batch.struct()
        P = params_struct(params)
        o = out.struct()
        t = Tuning()
        ms = ctypes.c_float()
        _check(self._lib.fl_autotune(self._h, ctypes.byref(b), ctypes.byref(P), ctypes.byref(o), int(reps),
                                     ctypes.byref(t), ctypes.byref(ms), self._stream(stream)), "fl_autotune")
        return (t.pairs_per_lane, t.lds_mode, t.wg_per_cu, t.xcd_aware), ms.value

    def set_stats(self, on: bool):
        _check(self._lib.fl_set_stats(self._h, int(bool(on))), "fl_set_stats")

    def get_stats(self):
        v = (ctypes.c_int64 * 4)()
        _check(self._lib.fl_get_stats(self._h, v), "fl_get_stats")
        return dict(n_visible=v[0], n_cells=v[1], n_kp_scanned=v[2], n_cand=v[3])

    def set_profiling(self, on: bool):
        _check(self._lib.fl_set_profiling(self._h, int(bool(on))), "fl_set_profiling")

    def get_profile(self, kernel: str = "search"):
        """(summed ms, launches) of the eager kernels of class `kernel`
        ("search" or "refine") since profiling was enabled or last read."""
        k = {"search": _abi.PROF_SEARCH, "refine": _abi.PROF_REFINE}[kernel]
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self._lib.fl_get_profile(self._h, k, ctypes.byref(ms), ctypes.byref(n)), "fl_get_profile")
        return ms.value, n.value

    def valu_rate(self, iters: int = 10000, stream=None) -> float:
        """Measured issue rate (lane-ops/s) of the Hamming instructions on
        every compute unit; synchronises the stream."""
        r = ctypes.c_double()
        _check(self._lib.fl_valu_rate(self._h, int(iters), ctypes.byref(r), self._stream(stream)), "fl_valu_rate")
        return r.value

    def debug_set_list_cap(self, cap: int):
        _check(self._lib.fl_debug_set_list_cap(self._h, int(cap)), "fl_debug_set_list_cap")


def search_fuse_noalloc(mp_xyz, mp_desc, mp_dmax, mp_id, kp_xy, kp_oct, kp_desc, kp_owner, sim3_16, cam8, params,
                        grid=None, out: Optional[FuseOutputs] = None, stream=None) -> FuseOutputs:
    """fl_search_fuse_noalloc on the current device: the plain search without a
    context, its scratch in the library's static device array (the output
    tensors, when not given, are still allocated here by torch)."""
    lib = _abi.load()
    d = mp_xyz.device
    n = int(mp_xyz.shape[0])
    if out is None:
        out = FuseOutputs.empty(n, d)
    kf = Keyframe(int(kp_xy.shape[0]), _ptr(kp_xy, torch.float32, "kp_xy", device=d),
                  _ptr(kp_oct, torch.int8, "kp_oct", 1, d), _ptr(kp_desc, torch.uint8, "kp_desc", 16, d),
                  _ptr(kp_owner, torch.int32, "kp_owner", device=d),
                  _ptr(grid[0], torch.int32, "cell_start", device=d) if grid is not None else None,
                  _ptr(grid[1], torch.int32, "cell_kp", device=d) if grid is not None else None)
    S = sim3_struct(sim3_16)
    K = pinhole_struct(cam8)
    P = params_struct(params)
    o = out.struct()
    s = stream if stream is not None else torch.cuda.current_stream(d)
    _check(lib.fl_search_fuse_noalloc(n, _ptr(mp_xyz, torch.float32, "mp_xyz", device=d),
                                      _ptr(mp_desc, torch.uint8, "mp_desc", 16, d),
                                      _ptr(mp_dmax, torch.float32, "mp_dmax", device=d),
                                      _ptr(mp_id, torch.int32, "mp_id", device=d), ctypes.byref(kf), ctypes.byref(S),
                                      ctypes.byref(K), ctypes.byref(P), ctypes.byref(o), ctypes.c_void_p(s.cuda_stream)),
           "fl_search_fuse_noalloc")
    return out


class Sim3Residual(torch.autograd.Function):
    """loss = sum_i Huber(|pi(T_k exp(xi) S0 X_i) - uv_i|).

    forward(xi [7] f64, S0 [13] f64, xyz, uv, kf_idx, kf_T, cam8, delta, ctx)
    The backward is the hand-written kernel pair: the residual backward
    gives g, the gradient with respect to a left perturbation of
    S = exp(xi) S0, and fl_sim3_grad_xi turns it into dL/dxi =
    grad_out * J_l(xi)^T g (J_l the Sim3 left Jacobian; the identity at
    xi = 0)."""

    @staticmethod
    def forward(fctx, xi, S0, xyz, uv, kf_idx, kf_T, cam8, delta, flctx: Context):
        xi = xi.detach().contiguous()
        S, S32 = flctx.sim3_exp_mul(xi, S0.contiguous())
        _, _, loss = flctx.residual_fwd(xyz, uv, kf_idx, kf_T, S32, cam8, delta, want_r=False)
        fctx.save_for_backward(xyz, uv, S32, xi)
        fctx.kf_idx = kf_idx
        fctx.kf_T = kf_T
        fctx.cam8 = cam8
        fctx.delta = delta
        fctx.flctx = flctx
        return loss.reshape(())

    @staticmethod
    def backward(fctx, grad_out):
        xyz, uv, S32, xi = fctx.saved_tensors
        g, _ = fctx.flctx.residual_bwd(xyz, uv, fctx.kf_idx, fctx.kf_T, S32, fctx.cam8, fctx.delta, 1.0,
                                       want_H=False)
        scale = grad_out.detach().to(torch.float64).contiguous().reshape(1)
        gx = fctx.flctx.sim3_grad_xi(xi, g, scale)
        return (gx, None, None, None, None, None, None, None, None)
