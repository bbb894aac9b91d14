"""Synthetic stand-ins for the loop events of the paper's EuRoC / TUM-VI runs.

The paper evaluates loop fusion (Sec. IV-D3, Table I) on real stereo-inertial
sequences that are not available here.  These generators produce loop events
with the camera shapes of those datasets (752x480 and 512x512 pinholes) and
the structure the fusion step sees: map points of the loop region, covisible
keyframes with ORB-like keypoints spread over 8 octaves, 256-bit descriptors,
and a Sim3 loop correction.  Every random draw comes from
``numpy.random.Generator(PCG64(seed))``.

Scene recipe (all workloads):
  * A point is anchored to a keyframe ``a``: pixel ~ U(image), depth ~ U[d0, d1],
    and its world position is the back-projection through the anchor's Sim3.
  * Its distance invariance is ``dmax = 0.95 * d_ref * 1.2**o_ref`` with
    ``o_ref ~ U{0..7}`` and ``d_ref`` the metric distance to the anchor, so the
    point is seen at octave ``o_ref`` from the anchor, 5% away from a boundary.
  * Keypoints of a keyframe are a mix of planted observations (projection of a
    visible point + N(0, sigma^2) px per axis, descriptor = point descriptor
    with every bit flipped with probability 0.05, octave = the octave the
    point is detected at from that keyframe), pre-owned duplicates (planted
    the same way but already owned by another map point with a fresh id) and
    outliers (uniform position, uniform octave, random descriptor).  The order
    of keypoints inside a keyframe is shuffled.

Pose conventions: ``T_k = (R_k, t_k)`` maps world to camera ``k``.  A Sim3 is
stored as 13 float64 ``[R (row-major 9), t (3), s]`` acting as
``X -> s R X + t``.  The per-keyframe search transform is ``T_k o S`` whose
float32 form ``[sR (9), t (3), 1/s, 0, 0, 0]`` is what the search consumes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

N_OCT = 8
SCALE = 1.2

# (fx, fy, cx, cy, width, height)
CAM_752 = (458.0, 458.0, 367.0, 248.0, 752.0, 480.0)
CAM_512 = (190.0, 190.0, 256.0, 256.0, 512.0, 512.0)

FRESH_ID_BASE = 1_000_000_000      # ids of map points outside the loop region
POINT_ID_BASE = 1000               # ids of loop-region points: base + global index


@dataclass
class LoopParams:
    """Thresholds of the fusion search (window 3 px x 1.2^octave, 64x48 grid,
    Hamming threshold 50, ratio test off)."""
    win_px: float = 3.0
    scale_factor: float = SCALE
    n_octaves: int = N_OCT
    grid_cols: int = 64
    grid_rows: int = 48
    hamming_th: int = 50
    nn_ratio: float = 0.0


def verification_params() -> LoopParams:
    """Thresholds taken for the projection searches of loop verification
    (one keyframe, or three in one launch): a 10 px x 1.2^octave window and
    the nearest-neighbour ratio test at 0.75, Hamming threshold 50.  The
    paper gives no constants for that stage; these are a reading."""
    return LoopParams(win_px=10.0, nn_ratio=0.75)


def search_transforms(ev, S) -> np.ndarray:
    """The float32 search transforms T_k o S of every keyframe of `ev` for a
    float64 Sim3 S, in the form of Event.kf_sim3."""
    T = np.asarray(ev.kf_T, np.float64).reshape(-1, 12)
    return np.stack([_sim3_f32(_compose_T_S(r[:9].reshape(3, 3), r[9:], S)) for r in T])


def perturbed(S, deg: float, metres: float, dscale: float, seed: int) -> np.ndarray:
    """A float64 Sim3 near S (rotated by `deg`, shifted by `metres`, scaled
    by 1 + dscale, in seeded random directions)."""
    return _perturb(np.random.Generator(np.random.PCG64(seed)), np.asarray(S, np.float64), deg, metres, dscale)


# Robust refinement after the verification search: 2 rounds of 5 steps, the
# inlier bound at the 99% quantile of a chi-square with 2 degrees of freedom
# for 1 px noise (sqrt(9.21) px), Levenberg-Marquardt from lambda = 1e-3.
# The paper gives no constants for its Sim3 optimisation; these are a reading.
ROBUST_ITERS, ROBUST_ROUNDS, ROBUST_OUTLIER_PX, ROBUST_LM_LAMBDA = 5, 2, 3.035, 1e-3


def gen_c2_misplaced(seed: int = 202) -> Event:
    """The loop event with 10% of its planted keypoints moved 6-9 px away
    (wrong associations the verification window still matches)."""
    return gen_c2(seed=seed, misplace=(0.1, 6.0, 9.0))


def ps2_passes(ev, seed: int = 5):
    """The two projection searches on the current keyframe around the Sim3
    optimisation, as (params, kf_sim3) pairs: one at the event's starting
    Sim3 with the verification thresholds (10 px x 1.2^octave, ratio 0.75),
    one at a Sim3 moved by 0.05 deg, 5 mm and 0.1% scale (a refined estimate)
    with a 5 px window and ratio 0.9.  The paper gives no constants for these
    searches; these are a reading."""
    rng = np.random.Generator(np.random.PCG64(seed))
    S_b = _perturb(rng, np.asarray(ev.S_init, np.float64), 0.05, 0.005, 0.001)
    return [(verification_params(), np.asarray(ev.kf_sim3, np.float32)),
            (LoopParams(win_px=5.0, nn_ratio=0.9), search_transforms(ev, S_b))]


@dataclass
class Event:
    """One loop event.  Keyframe-major arrays are concatenated over keyframes."""
    cams: np.ndarray            # f32 [n_kf, 8]  fx fy cx cy w h 0 0
    kf_T: np.ndarray            # f64 [n_kf, 12] world->camera R (row-major), t
    S_true: np.ndarray          # f64 [13] loop Sim3 used to synthesise observations
    S_init: np.ndarray          # f64 [13] Sim3 the search runs at (and GN starts from)
    kf_sim3: np.ndarray         # f32 [n_kf, 16] T_k o S_init as sR, t, 1/s, pad
    mp_xyz: np.ndarray          # f32 [n_mp, 3]
    mp_desc: np.ndarray         # u8  [n_mp, 32]
    mp_dmax: np.ndarray         # f32 [n_mp]
    mp_id: np.ndarray           # i32 [n_mp]
    kp_offset: np.ndarray       # i32 [n_kf + 1]
    kp_xy: np.ndarray           # f32 [n_kp, 2]
    kp_oct: np.ndarray          # i8  [n_kp]
    kp_desc: np.ndarray         # u8  [n_kp, 32]
    kp_owner: np.ndarray        # i32 [n_kp]  -1 = free
    pair_offset: np.ndarray     # i64 [n_kf + 1]
    pair_mp: Optional[np.ndarray]  # i32 [n_pairs] local point index, None = dense
    planted_kf: np.ndarray      # i32  keyframe of each planted keypoint
    planted_kp: np.ndarray      # i32  local keypoint index
    planted_mp: np.ndarray      # i32  point index
    planted_kind: np.ndarray    # i8   0 free, 1 pre-owned duplicate, 2 observed (owner = own id)
    params: LoopParams = field(default_factory=LoopParams)
    name: str = ""

    @property
    def n_kf(self) -> int:
        return int(self.cams.shape[0])

    @property
    def n_mp(self) -> int:
        return int(self.mp_xyz.shape[0])

    @property
    def n_pairs(self) -> int:
        return int(self.pair_offset[-1])

    @property
    def dense(self) -> bool:
        return self.pair_mp is None


@dataclass
class Batch:
    """Several events concatenated: keyframes, keypoints, points and pairs."""
    events: List[Event]
    event_kf_offset: np.ndarray   # i32 [n_events + 1]
    event_mp_offset: np.ndarray   # i32 [n_events + 1]
    cams: np.ndarray
    kf_T: np.ndarray
    kf_sim3: np.ndarray
    mp_xyz: np.ndarray
    mp_desc: np.ndarray
    mp_dmax: np.ndarray
    mp_id: np.ndarray
    kp_offset: np.ndarray         # i32 [n_kf + 1] global keypoint offsets
    kp_xy: np.ndarray
    kp_oct: np.ndarray
    kp_desc: np.ndarray
    kp_owner: np.ndarray
    pair_offset: np.ndarray       # i64 [n_kf + 1]
    pair_mp: Optional[np.ndarray]  # i32, local point index within the event
    params: LoopParams

    @property
    def n_events(self) -> int:
        return len(self.events)

    @property
    def n_kf(self) -> int:
        return int(self.cams.shape[0])

    @property
    def n_mp(self) -> int:
        return int(self.mp_xyz.shape[0])

    @property
    def n_pairs(self) -> int:
        return int(self.pair_offset[-1])


# ----------------------------------------------------------------------------
# scene geometry helpers (synthesis only)

def _rodrigues(axis: np.ndarray, angle: float) -> np.ndarray:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * (K @ K)


def _unit(rng) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _sim3(R, t, s) -> np.ndarray:
    return np.concatenate([np.asarray(R, np.float64).reshape(9), np.asarray(t, np.float64), [float(s)]])


def _split(S):
    return S[:9].reshape(3, 3), S[9:12], float(S[12])


def _random_loop_sim3(rng, s_lo, s_hi, max_deg, trans) -> np.ndarray:
    s = rng.uniform(s_lo, s_hi) if s_hi > s_lo else s_lo
    ang = np.deg2rad(rng.uniform(0.0, max_deg)) if max_deg > 0 else 0.0
    R = _rodrigues(_unit(rng), ang)
    t = _unit(rng) * trans
    return _sim3(R, t, s)


def _perturb(rng, S, deg, metres, dscale) -> np.ndarray:
    """A Sim3 near S: rotated by `deg` about a random axis, shifted by `metres`
    in a random direction and scaled by (1 + dscale)."""
    R, t, s = _split(S)
    Rp = _rodrigues(_unit(rng), np.deg2rad(deg))
    return _sim3(Rp @ R, Rp @ t + _unit(rng) * metres, s * (1.0 + dscale))


def _arc_poses(n, radius, spacing):
    """Keyframes on a circular arc, optical axes toward the arc's centre.
    Returns world->camera (R, t) for each keyframe."""
    dphi = spacing / radius
    centre = np.array([0.0, 0.0, radius])
    out = []
    for k in range(n):
        phi = (k - 0.5 * (n - 1)) * dphi
        c = centre + radius * np.array([np.sin(phi), 0.0, -np.cos(phi)])
        Rwc = np.array([[np.cos(phi), 0.0, -np.sin(phi)],
                        [0.0, 1.0, 0.0],
                        [np.sin(phi), 0.0, np.cos(phi)]])  # columns = camera axes in world
        R = Rwc.T
        out.append((R, -R @ c))
    return out


def _compose_T_S(R_k, t_k, S):
    """(T_k o S)(X) = s R_k R X + R_k t + t_k, as a float64 Sim3."""
    R, t, s = _split(S)
    return _sim3(R_k @ R, R_k @ t + t_k, s)


def _sim3_f32(S) -> np.ndarray:
    R, t, s = _split(S)
    out = np.zeros(16, np.float32)
    out[:9] = (s * R).reshape(9).astype(np.float32)
    out[9:12] = t.astype(np.float32)
    out[12] = np.float32(1.0 / s)
    return out


def _cam_row(cam) -> np.ndarray:
    return np.array(list(cam) + [0.0, 0.0], np.float32)


def _backproject(cam, u, v, z, S):
    """World points seen at pixel (u, v), depth z, through Sim3 S."""
    fx, fy, cx, cy, _, _ = cam
    q = np.stack([(u - cx) / fx * z, (v - cy) / fy * z, z], axis=1)
    R, t, s = _split(S)
    return ((q - t) @ R) / s        # R^T (q - t) / s, row-vector form


def _camera_coords(X, S):
    R, t, s = _split(S)
    return X @ (s * R).T + t


def _detect_octave(d, dmax, n_oct):
    """Octave a point at metric distance d is detected at (scene rule):
    ceil(log(dmax / d) / log 1.2) clipped to [0, n_oct - 1]."""
    with np.errstate(divide="ignore", invalid="ignore"):
        o = np.ceil(np.log(dmax / d) / np.log(SCALE))
    o = np.where(np.isfinite(o), o, n_oct - 1)
    return np.clip(o, 0, n_oct - 1).astype(np.int8)


def _flip_bits(rng, desc, p):
    n = desc.shape[0]
    bits = rng.random((n, 256), dtype=np.float32) < p
    mask = np.packbits(bits, axis=1, bitorder="little")
    return desc ^ mask


# ----------------------------------------------------------------------------
# generic event builder

def gen_event(rng, *, cam, kf_poses, S_true, S_init, n_mp, depth, anchors,
              covis=None, kp_counts, frac_planted, frac_outlier, frac_dup,
              pix_sigma=1.0, flip_p=0.05, skip_frac=0.0, misplace=None, id_base=POINT_ID_BASE,
              fresh_base=FRESH_ID_BASE, params=None, name="") -> Event:
    """Build one loop event.

    anchors : int array [n_mp], the keyframe each point is generated from.
    covis   : None for dense pairs (every point against every keyframe), else
              (start, count) int arrays giving each point's consecutive run of
              covisible keyframes.
    """
    params = params or LoopParams()
    n_kf = len(kf_poses)
    cams = np.tile(_cam_row(cam), (n_kf, 1))
    fx, fy, cx, cy, W, H = cam
    kf_T = np.stack([np.concatenate([R.reshape(9), t]) for R, t in kf_poses])
    S_kf_true = [_compose_T_S(R, t, S_true) for R, t in kf_poses]
    S_kf_init = [_compose_T_S(R, t, S_init) for R, t in kf_poses]
    kf_sim3 = np.stack([_sim3_f32(S) for S in S_kf_init])

    # map points
    u = rng.uniform(0.0, W, n_mp)
    v = rng.uniform(0.0, H, n_mp)
    z = rng.uniform(depth[0], depth[1], n_mp)
    X = np.empty((n_mp, 3))
    for a in np.unique(anchors):
        sel = anchors == a
        X[sel] = _backproject(cam, u[sel], v[sel], z[sel], S_kf_true[a])
    o_ref = rng.integers(0, params.n_octaves, n_mp)
    ray = np.sqrt(((u - cx) / fx) ** 2 + ((v - cy) / fy) ** 2 + 1.0)
    s_true = S_true[12]
    d_ref = z * ray / s_true
    dmax = 0.95 * d_ref * SCALE ** o_ref
    mp_xyz = X.astype(np.float32)
    mp_desc = rng.integers(0, 256, (n_mp, 32), dtype=np.uint8)
    mp_dmax = dmax.astype(np.float32)
    mp_id = (id_base + np.arange(n_mp)).astype(np.int32)

    # pairs
    if covis is None:
        pair_offset = np.arange(n_kf + 1, dtype=np.int64) * n_mp
        pair_lists = None
        pair_mp = None
    else:
        start, count = covis
        pair_lists = []
        for k in range(n_kf):
            pair_lists.append(np.nonzero((start <= k) & (k < start + count))[0].astype(np.int32))
        pair_offset = np.zeros(n_kf + 1, np.int64)
        pair_offset[1:] = np.cumsum([len(p) for p in pair_lists])
        pair_mp = np.concatenate(pair_lists) if pair_lists else np.zeros(0, np.int32)

    kp_xy_l, kp_oct_l, kp_desc_l, kp_owner_l = [], [], [], []
    pk_kf, pk_kp, pk_mp, pk_kind = [], [], [], []
    kp_offset = np.zeros(n_kf + 1, np.int32)
    fresh = fresh_base
    Xd = mp_xyz.astype(np.float64)
    for k in range(n_kf):
        n_kp = int(kp_counts[k])
        q = _camera_coords(Xd, S_kf_true[k])
        with np.errstate(divide="ignore", invalid="ignore"):
            uu = fx * q[:, 0] / q[:, 2] + cx
            vv = fy * q[:, 1] / q[:, 2] + cy
        vis = (q[:, 2] > 0) & (uu >= 0) & (uu < W) & (vv >= 0) & (vv < H)
        if pair_lists is not None:
            cand = pair_lists[k][vis[pair_lists[k]]]
        else:
            cand = np.nonzero(vis)[0]
        n_pl = int(round(frac_planted * n_kp))
        n_out = int(round(frac_outlier * n_kp))
        n_dup = n_kp - n_pl - n_out if frac_dup > 0 else 0
        if frac_dup <= 0:
            n_out = n_kp - n_pl
        want = n_pl + n_dup
        if want > len(cand):            # too few visible points: fill with outliers
            scale = len(cand) / max(want, 1)
            n_pl = int(n_pl * scale)
            n_dup = len(cand) - n_pl
            n_out = n_kp - n_pl - n_dup
        chosen = rng.choice(cand, size=n_pl + n_dup, replace=False) if n_pl + n_dup > 0 else np.zeros(0, np.int64)
        d_k = np.linalg.norm(q[chosen], axis=1) / S_kf_true[k][12]
        oct_pl = _detect_octave(d_k, mp_dmax[chosen].astype(np.float64), params.n_octaves)
        xy_pl = np.stack([uu[chosen], vv[chosen]], axis=1) + rng.normal(0.0, pix_sigma, (len(chosen), 2))
        if misplace is not None and n_pl > 0:
            # wrong associations: planted keypoints moved away from their point's
            # projection, descriptor kept (gross outliers of the refinement)
            frac, lo, hi = misplace
            m = rng.random(n_pl) < frac
            ang = rng.uniform(0.0, 2 * np.pi, n_pl)
            dist = rng.uniform(lo, hi, n_pl)
            xy_pl[:n_pl][m] += (dist[:, None] * np.stack([np.cos(ang), np.sin(ang)], axis=1))[m]
        desc_pl = _flip_bits(rng, mp_desc[chosen], flip_p)
        owner_pl = np.full(len(chosen), -1, np.int64)
        kind = np.zeros(len(chosen), np.int8)
        owner_pl[n_pl:] = fresh + np.arange(n_dup)
        kind[n_pl:] = 1
        fresh += n_dup
        if skip_frac > 0 and n_pl > 0:
            n_skip = int(round(skip_frac * n_kp))
            n_skip = min(n_skip, n_pl)
            owner_pl[:n_skip] = mp_id[chosen[:n_skip]]
            kind[:n_skip] = 2
        xy_out = np.stack([rng.uniform(0.0, W, n_out), rng.uniform(0.0, H, n_out)], axis=1)
        oct_out = rng.integers(0, params.n_octaves, n_out).astype(np.int8)
        desc_out = rng.integers(0, 256, (n_out, 32), dtype=np.uint8)
        xy = np.concatenate([xy_pl, xy_out]).astype(np.float32)
        octs = np.concatenate([oct_pl, oct_out]).astype(np.int8)
        desc = np.concatenate([desc_pl, desc_out]).astype(np.uint8)
        owner = np.concatenate([owner_pl, np.full(n_out, -1)]).astype(np.int32)
        perm = rng.permutation(n_kp)
        inv = np.empty(n_kp, np.int64)
        inv[perm] = np.arange(n_kp)
        kp_xy_l.append(xy[perm])
        kp_oct_l.append(octs[perm])
        kp_desc_l.append(desc[perm])
        kp_owner_l.append(owner[perm])
        pk_kf.append(np.full(len(chosen), k, np.int32))
        pk_kp.append(inv[: len(chosen)].astype(np.int32))
        pk_mp.append(chosen.astype(np.int32))
        pk_kind.append(kind)
        kp_offset[k + 1] = kp_offset[k] + n_kp

    cat = lambda L, dt, shape: (np.concatenate(L).astype(dt) if L else np.zeros(shape, dt))  # noqa: E731
    return Event(
        cams=cams, kf_T=kf_T, S_true=S_true, S_init=S_init, kf_sim3=kf_sim3,
        mp_xyz=mp_xyz, mp_desc=mp_desc, mp_dmax=mp_dmax, mp_id=mp_id,
        kp_offset=kp_offset,
        kp_xy=cat(kp_xy_l, np.float32, (0, 2)).reshape(-1, 2),
        kp_oct=cat(kp_oct_l, np.int8, (0,)),
        kp_desc=cat(kp_desc_l, np.uint8, (0, 32)).reshape(-1, 32),
        kp_owner=cat(kp_owner_l, np.int32, (0,)),
        pair_offset=pair_offset, pair_mp=pair_mp,
        planted_kf=cat(pk_kf, np.int32, (0,)), planted_kp=cat(pk_kp, np.int32, (0,)),
        planted_mp=cat(pk_mp, np.int32, (0,)), planted_kind=cat(pk_kind, np.int8, (0,)),
        params=params, name=name)


# ----------------------------------------------------------------------------
# the five workloads

def gen_c1(seed: int = 101) -> Event:
    """Plain single call: 1 keyframe 752x480, 1,000 keypoints (600 planted from
    distinct points, 400 outliers), 2,000 points at depth 1-10 m, S with
    scale 1.03, 2 deg rotation, 0.1 m translation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = _rodrigues(_unit(rng), np.deg2rad(2.0))
    t = _unit(rng) * 0.1
    S = _sim3(R, t, 1.03)
    poses = [(np.eye(3), np.zeros(3))]
    return gen_event(rng, cam=CAM_752, kf_poses=poses, S_true=S, S_init=S, n_mp=2000,
                     depth=(1.0, 10.0), anchors=np.zeros(2000, np.int64), kp_counts=[1000],
                     frac_planted=0.6, frac_outlier=0.4, frac_dup=0.0, name="c1")


def gen_c2(seed: int = 202, skip_frac: float = 0.0, n_kf: int = 20, n_mp: int = 15000,
           n_kp: int = 1200, perturb: bool = True, misplace=None, kp_counts=None) -> Event:
    """Loop event: 20 keyframes 752x480 on a 3 m arc of radius 5 m, 1,200
    keypoints each (50% planted, 30% outliers, 20% pre-owned duplicates),
    15,000 points at depth 0.5-20 m in the middle keyframe's frustum, loop
    Sim3 with scale U[0.95, 1.05], rotation <= 5 deg, 0.1 m translation.
    The search runs at a Sim3 perturbed from the truth by 0.1 deg, 1 cm and
    0.2% scale (the state before refinement).  misplace = (fraction, lo, hi)
    moves that fraction of the planted keypoints U[lo, hi] px away from their
    point's projection (wrong associations).  kp_counts (one per keyframe)
    replaces n_kf x n_kp keypoint counts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if kp_counts is not None:
        n_kf = len(kp_counts)
    S = _random_loop_sim3(rng, 0.95, 1.05, 5.0, 0.1)
    S_init = _perturb(rng, S, 0.1, 0.01, 0.002) if perturb else S
    poses = _arc_poses(n_kf, 5.0, 3.0 / max(n_kf - 1, 1))
    mid = n_kf // 2
    return gen_event(rng, cam=CAM_752, kf_poses=poses, S_true=S, S_init=S_init, n_mp=n_mp,
                     depth=(0.5, 20.0), anchors=np.full(n_mp, mid),
                     kp_counts=list(kp_counts) if kp_counts is not None else [n_kp] * n_kf,
                     frac_planted=0.5, frac_outlier=0.3, frac_dup=0.2, skip_frac=skip_frac,
                     misplace=misplace, name="c2")


def _trunc_geom(rng, n, p, lo, hi):
    k = np.arange(lo, hi + 1)
    w = (1.0 - p) ** (k - lo) * p
    return rng.choice(k, size=n, p=w / w.sum())


def gen_c3(seed: int = 303, n_kf: int = 60, n_mp: int = 60000, kp_lo: int = 300,
           kp_hi: int = 2500, id_base: int = POINT_ID_BASE, fresh_base: int = FRESH_ID_BASE) -> Event:
    """Batched uneven event: 60 keyframes 512x512 (fx = fy = 190, cx = cy = 256)
    spaced 0.1 m on a 3 m-radius arc, keypoints U{300..2500} per keyframe,
    60,000 points each anchored to a random keyframe, covisible with a run of
    c ~ truncated Geometric(0.125) on {1..40} consecutive keyframes around
    its anchor; pairs are the (point, covisible keyframe) list."""
    rng = np.random.Generator(np.random.PCG64(seed))
    S = _random_loop_sim3(rng, 0.95, 1.05, 5.0, 0.1)
    S_init = _perturb(rng, S, 0.1, 0.01, 0.002)
    poses = _arc_poses(n_kf, 3.0, 0.1)
    anchors = rng.integers(0, n_kf, n_mp)
    c = np.minimum(_trunc_geom(rng, n_mp, 0.125, 1, 40), n_kf)
    start = np.clip(anchors - (c - 1) // 2, 0, n_kf - c)
    kp_counts = rng.integers(kp_lo, kp_hi + 1, n_kf)
    return gen_event(rng, cam=CAM_512, kf_poses=poses, S_true=S, S_init=S_init, n_mp=n_mp,
                     depth=(0.5, 20.0), anchors=anchors, covis=(start, c), kp_counts=kp_counts,
                     frac_planted=0.5, frac_outlier=0.3, frac_dup=0.2, id_base=id_base,
                     fresh_base=fresh_base, name="c3")


def gen_c4(seed: int = 404, n: int = 50000, outlier_frac: float = 0.1, outlier_px: float = 20.0,
           pix_sigma: float = 1.0):
    """Residual workload: 50,000 matched pairs of points (752x480 camera,
    pixel uniform, depth 1-10 m) observed through a loop Sim3 with one
    identity keyframe pose; observations = projection + N(0, 1) px, 10% of
    them displaced by 20 px in a uniform direction.  Returns a dict with
    float32 xyz [n,3], uv [n,2], the true Sim3 (13 f64), the camera row,
    and the tangent offset xi0 = (1 deg about x, 5 cm along y, 0.02) at which
    the gradient is evaluated."""
    rng = np.random.Generator(np.random.PCG64(seed))
    S = _random_loop_sim3(rng, 0.95, 1.05, 5.0, 0.1)
    fx, fy, cx, cy, W, H = CAM_752
    u = rng.uniform(0.0, W, n)
    v = rng.uniform(0.0, H, n)
    z = rng.uniform(1.0, 10.0, n)
    X = _backproject(CAM_752, u, v, z, S).astype(np.float32)
    q = _camera_coords(X.astype(np.float64), S)
    uv = np.stack([fx * q[:, 0] / q[:, 2] + cx, fy * q[:, 1] / q[:, 2] + cy], axis=1)
    uv += rng.normal(0.0, pix_sigma, (n, 2))
    out = rng.random(n) < outlier_frac
    th = rng.uniform(0.0, 2 * np.pi, n)
    uv[out] += outlier_px * np.stack([np.cos(th[out]), np.sin(th[out])], axis=1)
    xi0 = np.array([np.deg2rad(1.0), 0.0, 0.0, 0.0, 0.05, 0.0, 0.02])
    # an evaluation point near the truth built from plain pose algebra (for
    # timing runs): rotate 1 deg about x, shift 5 cm along y, scale by e^0.02
    R, t, s = _split(S)
    Rd = _rodrigues(np.array([1.0, 0.0, 0.0]), np.deg2rad(1.0))
    sd = float(np.exp(0.02))
    S_eval = _sim3(Rd @ R, sd * (Rd @ t) + np.array([0.0, 0.05, 0.0]), sd * s)
    return dict(xyz=X, uv=uv.astype(np.float32), S_true=S, cam=_cam_row(CAM_752),
                xi0=xi0, S_eval=S_eval, S_eval_f32=_sim3_f32(S_eval), outlier=out, huber_delta=2.45)


def _sim3_inverse(S):
    R, t, sc = _split(S)
    return _sim3(R.T, -(R.T @ t) / sc, 1.0 / sc)


def _observed_side(rng, n, S_map, n_views, pix_sigma, outlier_frac, outlier_px, cam=CAM_752):
    """n points seen in n_views keyframes (poses of ~6 deg and ~0.5 m):
    pixel ~ U(image), depth ~ U[1, 10] m, X back-projected through T_k o S_map,
    observation = pixel + N(0, pix_sigma), a fraction displaced by outlier_px.
    Returns ((xyz f32, uv f32, keyframe i32, poses f32 [n_views,12]), outlier mask)."""
    W, H = cam[4], cam[5]
    poses = [(_rodrigues(_unit(rng), np.deg2rad(rng.uniform(0.0, 6.0))), _unit(rng) * rng.uniform(0.0, 0.5))
             for _ in range(n_views)]
    T = np.stack([np.concatenate([Rk.reshape(9), tk]) for Rk, tk in poses]).astype(np.float32)
    kf = rng.integers(0, n_views, n).astype(np.int32)
    u, v, z = rng.uniform(0.0, W, n), rng.uniform(0.0, H, n), rng.uniform(1.0, 10.0, n)
    X = np.empty((n, 3))
    for k, (Rk, tk) in enumerate(poses):
        m = kf == k
        X[m] = _backproject(cam, u[m], v[m], z[m], _compose_T_S(Rk, tk, S_map))
    uv = np.stack([u, v], axis=1) + rng.normal(0.0, pix_sigma, (n, 2))
    out = rng.random(n) < outlier_frac
    th = rng.uniform(0.0, 2 * np.pi, n)
    uv[out] += outlier_px * np.stack([np.cos(th[out]), np.sin(th[out])], axis=1)
    return (X.astype(np.float32), uv.astype(np.float32), kf, T), out


def gen_inverse_pairs(S_true, n: int, seed: int, n_views: int = 4, pix_sigma: float = 1.0,
                      outlier_frac: float = 0.1, outlier_px: float = 20.0):
    """The other direction of a loop event's matches (two-sided refinement):
    n points of the current side observed in n_views loop-side keyframes
    through T_m o S_true^-1, with the noise and outliers of gen_bidir.
    Returns (xyz f32 [n,3], uv f32 [n,2], keyframe i32 [n], poses f32
    [n_views,12])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    side, _ = _observed_side(rng, n, _sim3_inverse(np.asarray(S_true, np.float64)), n_views, pix_sigma,
                             outlier_frac, outlier_px)
    return side


def gen_bidir(seed: int = 505, n_fwd: int = 20000, n_bwd: int = 20000, n_views: int = 4,
              pix_sigma: float = 1.0, outlier_frac: float = 0.1, outlier_px: float = 20.0):
    """Matches seen from both sides of a loop (752x480 camera, depth 1-10 m):
    loop-side points observed in current-side keyframes through T_k o S
    ("fwd"), and current-side points observed in loop-side keyframes through
    T_m o S^-1 ("bwd"); n_views keyframes per side with poses of ~6 deg and
    ~0.5 m, pixel noise N(0, pix_sigma), a fraction displaced by outlier_px.
    The start S0 is the truth moved by 0.5 deg, 2 cm and 1% scale.  Each set
    is (xyz f32 [n,3], uv f32 [n,2], keyframe index i32 [n], poses f32
    [n_views,12])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    S = _random_loop_sim3(rng, 0.95, 1.05, 5.0, 0.1)
    fwd, out_f = _observed_side(rng, n_fwd, S, n_views, pix_sigma, outlier_frac, outlier_px)
    bwd, out_b = _observed_side(rng, n_bwd, _sim3_inverse(S), n_views, pix_sigma, outlier_frac, outlier_px)
    S0 = _perturb(rng, S, 0.5, 0.02, 0.01)
    return dict(S_true=S, S0=S0, cam=_cam_row(CAM_752), fwd=fwd, bwd=bwd, outlier_fwd=out_f, outlier_bwd=out_b,
                huber_delta=2.45)


def gen_pose_graph(n: int = 1000, seed: int = 606, covis: int = 3, n_loops: int = 8, noise_deg: float = 0.1,
                   noise_m: float = 0.01, noise_scale: float = 0.001, drift: bool = True, laps: int = 1,
                   cross: int = 0):
    """An essential graph after a loop closure: n keyframes on a closed loop
    of radius 5 m (world -> camera poses, scale 1), edges (i, i + d) for
    d = 1..covis along the trajectory (spanning tree and covisibility), and
    n_loops loop edges joining the trajectory's last keyframes to its first
    ones.  With laps > 1 the trajectory runs round the loop laps times (a
    spiral whose radius grows by 0.25 m a lap), and every keyframe of a later
    lap is joined to the `cross` keyframes of the lap before that pass
    closest to the same place (the covisibility across laps once their map
    points are fused: several loops in one graph, whose reordered band is
    then several times wider).  Each edge measures M_ij = S_j S_i^-1 of the
    true poses, moved by N(0, noise) in rotation (deg), translation (m) and
    log scale.  The start chains the odometry edges (i, i + 1) from
    keyframe 0 with an extra drift of 0.02 deg, 2 mm and 0.2% scale per step
    (the state before the loop is corrected).  Keyframe 0 is fixed.  Returns
    dict(S_true [n,13], S0 [n,13], edges int32 [E,2] (host), M [E,13],
    fixed bool [n])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    S_true = []
    for i in range(n):
        a = 2 * np.pi * laps * i / n
        rad = 5.0 + 0.25 * laps * i / n if laps > 1 else 5.0
        R = _rodrigues(np.array([0.0, 1.0, 0.0]), -a)            # facing along the loop
        c = np.array([rad * np.cos(a), 0.1 * np.sin(3 * a), rad * np.sin(a)])
        S_true.append(_sim3(R, -R @ c, 1.0))
    S_true = np.stack(S_true)

    def inv(S):
        R, t, sc = _split(S)
        return _sim3(R.T, -(R.T @ t) / sc, 1.0 / sc)

    def mul(A, B):
        Ra, ta, sa = _split(A)
        Rb, tb, sb = _split(B)
        return _sim3(Ra @ Rb, sa * (Ra @ tb) + ta, sa * sb)

    def noisy(S, deg, m, ls):
        R, t, sc = _split(S)
        Rn = _rodrigues(_unit(rng), np.deg2rad(abs(rng.normal(0.0, deg)))) if deg > 0 else np.eye(3)
        return _sim3(Rn @ R, Rn @ t + rng.normal(0.0, m, 3), sc * float(np.exp(rng.normal(0.0, ls))))

    edges = [(i, i + d) for d in range(1, covis + 1) for i in range(n - d)]
    for k in range(n_loops):
        edges.append((n - 1 - k, k))
    if laps > 1 and cross > 0:
        period = n / laps
        for i in range(int(np.ceil(period)), n):
            j0 = int(round(i - period)) - cross // 2
            edges.extend((j, i) for j in range(max(j0, 0), min(j0 + cross, i - covis)))
    edges = np.array(sorted(set(edges)) if laps > 1 else sorted(edges), np.int32)
    M = np.stack([noisy(mul(S_true[j], inv(S_true[i])), noise_deg, noise_m, noise_scale) for i, j in edges])
    # the start: odometry chained from keyframe 0, with drift
    odo = {(int(i), int(j)): M[k] for k, (i, j) in enumerate(edges) if j == i + 1}
    S0 = [S_true[0]]
    for i in range(n - 1):
        step = odo[(i, i + 1)]
        if drift:
            step = mul(_sim3(_rodrigues(np.array([0.0, 1.0, 0.0]), np.deg2rad(0.02)), np.array([0.002, 0.0, 0.0]),
                             1.002), step)
        S0.append(mul(step, S0[-1]))
    fixed = np.zeros(n, bool)
    fixed[0] = True
    return dict(S_true=S_true, S0=np.stack(S0), edges=edges, M=M, fixed=fixed)


def gen_c5_event(e: int, n_kf: Optional[int] = None, n_mp: Optional[int] = None) -> Event:
    """Event e of the 200-event stream (seed 5000 + e): n_kf ~ U{5..80},
    camera 752x480 or 512x512 with probability 1/2, keypoints U{300..2500}
    per keyframe, n_mp ~ U{5,000..100,000}, dense pairs; the search runs at
    the truth perturbed by 0.1 deg, 1 cm and 0.2% scale."""
    rng = np.random.Generator(np.random.PCG64(5000 + e))
    nk = int(rng.integers(5, 81)) if n_kf is None else n_kf
    nm = int(rng.integers(5000, 100001)) if n_mp is None else n_mp
    big = rng.random() < 0.5
    cam = CAM_752 if big else CAM_512
    S = _random_loop_sim3(rng, 0.95, 1.05, 5.0, 0.1)
    S_init = _perturb(rng, S, 0.1, 0.01, 0.002)
    poses = _arc_poses(nk, 5.0, 3.0 / 19.0) if big else _arc_poses(nk, 3.0, 0.1)
    kp_counts = rng.integers(300, 2501, nk)
    return gen_event(rng, cam=cam, kf_poses=poses, S_true=S, S_init=S_init, n_mp=nm,
                     depth=(0.5, 20.0), anchors=np.full(nm, nk // 2), kp_counts=kp_counts,
                     frac_planted=0.5, frac_outlier=0.3, frac_dup=0.2, name=f"c5.{e}")


def gen_tiny(seed: int, n_kf: int = 3, n_mp: int = 200, n_kp=(60, 90), cam=CAM_752,
             sparse: bool = False, skip_frac: float = 0.05, params: Optional[LoopParams] = None) -> Event:
    """Small events for exhaustive CPU checks and multi-tile GPU parity at
    ragged sizes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    S = _random_loop_sim3(rng, 0.95, 1.05, 5.0, 0.1)
    S_init = _perturb(rng, S, 0.1, 0.01, 0.002)
    poses = _arc_poses(n_kf, 5.0, 0.3)
    kp_counts = rng.integers(n_kp[0], n_kp[1] + 1, n_kf)
    if sparse:
        anchors = rng.integers(0, n_kf, n_mp)
        c = rng.integers(1, n_kf + 1, n_mp)
        start = np.clip(anchors - (c - 1) // 2, 0, n_kf - c)
        covis = (start, c)
    else:
        anchors = np.full(n_mp, n_kf // 2)
        covis = None
    return gen_event(rng, cam=cam, kf_poses=poses, S_true=S, S_init=S_init, n_mp=n_mp,
                     depth=(0.5, 20.0), anchors=anchors, covis=covis, kp_counts=kp_counts,
                     frac_planted=0.5, frac_outlier=0.3, frac_dup=0.2, skip_frac=skip_frac,
                     params=params, name=f"tiny{seed}")


def concat_events(events: List[Event]) -> Batch:
    """Concatenate events into one batch.  Point ids are taken as they are;
    callers that batch events generated independently should give them
    disjoint id ranges (``id_base``) so ids stay unique within an event."""
    if not events:
        raise ValueError("no events")
    params = events[0].params
    ekf = np.zeros(len(events) + 1, np.int32)
    emp = np.zeros(len(events) + 1, np.int32)
    kp_off = [np.zeros(1, np.int32)]
    pair_off = [np.zeros(1, np.int64)]
    kp_base = 0
    pair_base = 0
    any_sparse = any(not ev.dense for ev in events)
    pair_mp = []
    for i, ev in enumerate(events):
        ekf[i + 1] = ekf[i] + ev.n_kf
        emp[i + 1] = emp[i] + ev.n_mp
        kp_off.append(ev.kp_offset[1:] + kp_base)
        pair_off.append(ev.pair_offset[1:] + pair_base)
        kp_base += int(ev.kp_offset[-1])
        pair_base += ev.n_pairs
        if any_sparse:
            if ev.dense:
                pair_mp.append(np.tile(np.arange(ev.n_mp, dtype=np.int32), ev.n_kf))
            else:
                pair_mp.append(ev.pair_mp)
    cat = np.concatenate
    return Batch(
        events=list(events), event_kf_offset=ekf, event_mp_offset=emp,
        cams=cat([e.cams for e in events]), kf_T=cat([e.kf_T for e in events]),
        kf_sim3=cat([e.kf_sim3 for e in events]),
        mp_xyz=cat([e.mp_xyz for e in events]), mp_desc=cat([e.mp_desc for e in events]),
        mp_dmax=cat([e.mp_dmax for e in events]), mp_id=cat([e.mp_id for e in events]),
        kp_offset=cat(kp_off).astype(np.int32), kp_xy=cat([e.kp_xy for e in events]),
        kp_oct=cat([e.kp_oct for e in events]), kp_desc=cat([e.kp_desc for e in events]),
        kp_owner=cat([e.kp_owner for e in events]), pair_offset=cat(pair_off).astype(np.int64),
        pair_mp=(cat(pair_mp).astype(np.int32) if any_sparse else None), params=params)
