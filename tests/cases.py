"""Hand-built test cases shared by the oracle pins and the GPU parity tests."""
from __future__ import annotations

import json
import os

import numpy as np

from synth import Event, LoopParams

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _bits(a, b):
    bits = np.zeros(256, bool)
    bits[a:b] = True
    return np.packbits(bits, bitorder="little")


def single_kf_event(xyz, desc, dmax, ids, kp_xy, kp_oct, kp_desc, kp_owner, sim3_16, cam8,
                    params: LoopParams, name="case") -> Event:
    n_mp = len(xyz)
    n_kp = len(kp_xy)
    return Event(
        cams=np.asarray(cam8, np.float32).reshape(1, 8), kf_T=np.zeros((1, 12)),
        S_true=np.zeros(13), S_init=np.zeros(13),
        kf_sim3=np.asarray(sim3_16, np.float32).reshape(1, 16),
        mp_xyz=np.asarray(xyz, np.float32).reshape(-1, 3),
        mp_desc=np.asarray(desc, np.uint8).reshape(-1, 32),
        mp_dmax=np.asarray(dmax, np.float32), mp_id=np.asarray(ids, np.int32),
        kp_offset=np.array([0, n_kp], np.int32),
        kp_xy=np.asarray(kp_xy, np.float32).reshape(-1, 2), kp_oct=np.asarray(kp_oct, np.int8),
        kp_desc=np.asarray(kp_desc, np.uint8).reshape(-1, 32),
        kp_owner=np.asarray(kp_owner, np.int32),
        pair_offset=np.array([0, n_mp], np.int64), pair_mp=None,
        planted_kf=np.zeros(0, np.int32), planted_kp=np.zeros(0, np.int32),
        planted_mp=np.zeros(0, np.int32), planted_kind=np.zeros(0, np.int8),
        params=params, name=name)


def hand_case():
    """The hand-worked fixture: (event, expected outputs dict)."""
    with open(os.path.join(GOLDEN, "fusion_hand_case.json")) as f:
        g = json.load(f)
    pts = g["points"]
    kps = g["keypoints"]
    params = LoopParams(**g["params"])
    ev = single_kf_event(
        xyz=[p["xyz"] for p in pts], desc=np.zeros((len(pts), 32), np.uint8),
        dmax=[p["dmax"] for p in pts], ids=[p["id"] for p in pts],
        kp_xy=[k["xy"] for k in kps], kp_oct=[k["octave"] for k in kps],
        kp_desc=np.stack([_bits(*k["bits"]) for k in kps]), kp_owner=[k["owner"] for k in kps],
        sim3_16=g["sim3"], cam8=g["camera"], params=params, name="hand")
    exp = {k: np.asarray(v) for k, v in g["expected"].items()}
    return ev, exp


def conflict_case(order):
    """Five points with identical descriptors within 0.1 px of each other
    (plus one far away), all matching the same free keypoint; `order`
    permutes the points.  Returns (event, index of the original point 0 in
    the permuted order)."""
    rng = np.random.default_rng(7)
    desc = rng.integers(0, 256, 32, dtype=np.uint8)
    base = np.array([[0.25, -0.5, 2.0]] * 5 + [[-0.5, 0.5, 2.0]])
    base[:5, 0] += np.arange(5) * 0.0004    # 0.02 px apart in u
    order = np.asarray(order)
    xyz = base[order]
    ids = (500 + order).astype(np.int32)
    kp_desc = np.stack([desc, rng.integers(0, 256, 32, dtype=np.uint8)])
    ev = single_kf_event(
        xyz=xyz, desc=np.tile(desc, (6, 1)), dmax=np.ones(6), ids=ids,
        kp_xy=[[62.6, 25.1], [25.0, 75.0]], kp_oct=[0, 0], kp_desc=kp_desc, kp_owner=[-1, -1],
        sim3_16=[1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0],
        cam8=[100, 100, 50, 50, 100, 100, 0, 0],
        params=LoopParams(win_px=3.0, n_octaves=4, grid_cols=8, grid_rows=8), name="conflict")
    return ev


def with_near_duplicates(ev, frac=0.4, flips=(2, 10), seed=7):
    """A one-keyframe event with extra keypoints next to a fraction of its
    planted ones: 0.4 px away, same octave, free, with a few descriptor bits
    flipped, so the second-best distance of those points comes close to the
    best and the ratio test has something to reject."""
    import dataclasses
    assert ev.n_kf == 1
    rng = np.random.default_rng(seed)
    planted = np.asarray(ev.planted_kp[ev.planted_kf == 0], np.int64)
    pick = rng.choice(planted, size=int(frac * len(planted)), replace=False)
    desc = ev.kp_desc[pick].copy()
    for r in range(len(pick)):
        bits = rng.choice(256, size=int(rng.integers(flips[0], flips[1] + 1)), replace=False)
        for b in bits:
            desc[r, b // 8] ^= np.uint8(1 << (b % 8))
    xy = ev.kp_xy[pick] + np.float32(0.4)
    n0 = int(ev.kp_offset[1])
    return dataclasses.replace(
        ev,
        kp_xy=np.concatenate([ev.kp_xy, xy.astype(np.float32)]),
        kp_oct=np.concatenate([ev.kp_oct, ev.kp_oct[pick]]),
        kp_desc=np.concatenate([ev.kp_desc, desc]),
        kp_owner=np.concatenate([ev.kp_owner, np.full(len(pick), -1, np.int32)]),
        kp_offset=np.array([0, n0 + len(pick)], dtype=ev.kp_offset.dtype),
        name=ev.name + "+dup")


def census_case():
    """The hand-worked census fixture: (event, eps, expected counts)."""
    with open(os.path.join(GOLDEN, "census_hand_case.json")) as f:
        g = json.load(f)
    pts, kps = g["points"], g["keypoints"]
    n = len(pts)
    ev = single_kf_event(
        xyz=[p["xyz"] for p in pts], desc=np.zeros((n, 32), np.uint8), dmax=np.ones(n),
        ids=[p["id"] for p in pts], kp_xy=[k["xy"] for k in kps], kp_oct=[k["octave"] for k in kps],
        kp_desc=np.zeros((len(kps), 32), np.uint8), kp_owner=[k["owner"] for k in kps],
        sim3_16=g["sim3"], cam8=g["camera"], params=LoopParams(**g["params"]), name="census")
    return ev, g["eps"], g["expected"]


def overshoot_graph():
    """A 10-keyframe loop (synth.gen_pose_graph seed 14) whose start has three
    free keyframes turned by 2-3 rad about random axes, moved by ~2 m and
    rescaled: from there the first undamped steps overshoot (the candidate's
    cost is 30-45% above the accepted one), so Levenberg-Marquardt refuses
    them before it converges."""
    import synth
    from oracle import sim3
    d = dict(synth.gen_pose_graph(n=10, seed=14, covis=2, n_loops=2))
    rng = np.random.default_rng(0)
    S0 = d["S0"].copy()
    for node in rng.choice(np.arange(1, 10), 3, replace=False):
        xi = np.zeros(7)
        xi[:3] = rng.normal(size=3)
        xi[:3] *= rng.uniform(2.0, 3.0) / np.linalg.norm(xi[:3])
        xi[3:6] = rng.normal(size=3) * 2
        xi[6] = rng.normal() * 0.8
        S0[node] = sim3.compose(sim3.exp(xi), S0[node])
    d["S0"] = S0
    return d
