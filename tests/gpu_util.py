"""Helpers shared by the GPU parity tests (marshalling only)."""
from __future__ import annotations

import numpy as np
import torch

FIELDS = ("best_idx", "best_dist", "second_dist", "decision", "target")


def dev():
    return torch.device("cuda:0")


def t(a, dtype=None):
    x = torch.from_numpy(np.ascontiguousarray(a)).to(dev())
    return x if dtype is None else x.view(dtype)


def assert_same(got: dict, exp: dict, label: str = ""):
    for k in FIELDS:
        g, e = np.asarray(got[k]), np.asarray(exp[k])
        assert g.shape == e.shape, (label, k, g.shape, e.shape)
        bad = np.nonzero(g != e)[0]
        assert bad.size == 0, (f"{label}: {k} differs at {bad.size} of {g.size} pairs; first {bad[:5].tolist()}: "
                               f"got {g[bad[:5]].tolist()} expected {e[bad[:5]].tolist()}")


def plain_per_keyframe(ctx, ev, params, use_dmax=True, use_id=True, with_grid=False):
    """Run fl_search_fuse keyframe by keyframe over a dense or sparse event and
    concatenate the outputs in pair order."""
    X = t(ev.mp_xyz)
    D = t(ev.mp_desc)
    M = t(ev.mp_dmax) if use_dmax else None
    I = t(ev.mp_id) if use_id else None
    outs = []
    for k in range(ev.n_kf):
        a, b = int(ev.kp_offset[k]), int(ev.kp_offset[k + 1])
        kx, ko, kd, kw = t(ev.kp_xy[a:b]), t(ev.kp_oct[a:b]), t(ev.kp_desc[a:b]), t(ev.kp_owner[a:b])
        grid = ctx.build_grid(kx, ev.cams[k], params) if with_grid else None
        if ev.pair_mp is None:
            o = ctx.search_fuse(X, D, M, I, kx, ko, kd, kw, ev.kf_sim3[k], ev.cams[k], params, grid=grid)
        else:
            sel = ev.pair_mp[ev.pair_offset[k]:ev.pair_offset[k + 1]]
            ids = ev.mp_id[sel] if use_id else sel.astype(np.int32)
            o = ctx.search_fuse(t(ev.mp_xyz[sel]), t(ev.mp_desc[sel]),
                                t(ev.mp_dmax[sel]) if use_dmax else None, t(ids),
                                kx, ko, kd, kw, ev.kf_sim3[k], ev.cams[k], params, grid=grid)
        outs.append(o.numpy())
    return {f: np.concatenate([o[f] for o in outs]) if outs else np.zeros(0) for f in FIELDS}
