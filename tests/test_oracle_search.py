"""Pins of the CPU search-and-fuse oracle against facts that do not come from
the oracle itself: a hand-worked case, brute force vs the cell grid,
Hamming identities, recovery of planted correspondences at the closed-form
rate, projection invariants of the pinhole/Sim3 model and the FP64 census."""
import itertools

import numpy as np
import pytest
from scipy.stats import binom

import oracle
import synth
from cases import conflict_case, hand_case

FIELDS = ("best_idx", "best_dist", "second_dist", "decision", "target")


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in FIELDS)


def test_hand_worked_case():
    ev, exp = hand_case()
    for grid in (False, True):
        out = oracle.search_fuse(ev, use_grid=grid)
        for k in FIELDS:
            assert out[k].tolist() == exp[k].tolist(), (k, grid)


@pytest.mark.parametrize("order", [list(p) for p in itertools.islice(itertools.permutations(range(6)), 0, 720, 97)])
def test_add_conflict_lowest_index_wins(order):
    ev = conflict_case(order)
    out = oracle.search_fuse(ev)
    dup = [i for i, o in enumerate(order) if o < 5]          # positions of the 5 duplicates
    winner = min(dup)
    assert out["decision"][winner] == oracle.ADD and out["target"][winner] == -1
    for i in dup:
        if i != winner:
            assert out["decision"][i] == oracle.FUSE
            assert out["target"][i] == ev.mp_id[winner]
    far = order.index(5)
    assert out["decision"][far] == oracle.NO_MATCH


def test_hamming_identities():
    rng = np.random.default_rng(3)
    for _ in range(50):
        a = rng.integers(0, 256, 32, dtype=np.uint8)
        b = rng.integers(0, 256, 32, dtype=np.uint8)
        assert oracle.hamming256(a, a) == 0
        assert oracle.hamming256(a, ~a) == 256
        assert oracle.hamming256(a, b) == int(np.unpackbits(a ^ b).sum())
        assert oracle.hamming256(a, b) == oracle.hamming256(b, a)


@pytest.mark.parametrize("seed", range(12))
def test_grid_equals_brute_force_tiny(seed):
    sparse = seed % 2 == 1
    ev = synth.gen_tiny(seed, n_kf=1 + seed % 4, n_mp=40 + 7 * seed, n_kp=(5, 32), sparse=sparse)
    for use_dmax, use_id in [(True, True), (False, True), (True, False)]:
        a = oracle.search_fuse(ev, use_grid=False, use_dmax=use_dmax, use_id=use_id)
        b = oracle.search_fuse(ev, use_grid=True, use_dmax=use_dmax, use_id=use_id)
        assert same(a, b)


@pytest.mark.parametrize("gen", ["c1", "c2", "c3"])
def test_grid_equals_brute_force_workloads(gen):
    ev = {"c1": synth.gen_c1, "c2": lambda: synth.gen_c2(skip_frac=0.05), "c3": synth.gen_c3}[gen]()
    a = oracle.search_fuse(ev, use_grid=False)
    b = oracle.search_fuse(ev, use_grid=True)
    assert same(a, b)
    # every decision class the method has appears
    dec = np.bincount(a["decision"], minlength=6)
    assert dec[oracle.NO_MATCH] > 0 and dec[oracle.ADD] > 0
    if gen != "c1":
        assert dec[oracle.FUSE] > 0 and dec[oracle.NOT_VISIBLE] > 0


def _recovery(ev, out):
    p = ev.pair_offset[ev.planted_kf] + ev.planted_mp
    keep = ev.planted_kind != 2
    p = p[keep]
    d = out["decision"][p]
    ok = (out["best_idx"][p] == ev.planted_kp[keep]) & ((d == oracle.ADD) | (d == oracle.FUSE))
    return int(ok.sum()), len(p)


@pytest.mark.parametrize("gen", ["c1", "c2"])
def test_planted_recovery_closed_form(gen):
    # A planted keypoint lies within +-3 px on both axes with probability
    # P(|N(0,1)| <= 3)^2 = 0.99461 (windows only grow at higher octaves); its
    # descriptor distance is Binomial(256, 0.05), above 50 with probability
    # 1e-14.  The miss count must be consistent with at most 1 - 0.99461.
    ev = synth.gen_c1() if gen == "c1" else synth.gen_c2(perturb=False)
    out = oracle.search_fuse(ev, use_grid=True)
    ok, n = _recovery(ev, out)
    p_in = (2 * 0.5 * (1 + __import__("math").erf(3 / np.sqrt(2))) - 1) ** 2
    assert abs(p_in - 0.99461) < 1e-5
    # one-sided binomial bound at 1e-6
    assert n - ok <= binom.ppf(1 - 1e-6, n, 1 - p_in), (ok, n)


@pytest.mark.parametrize("gen", ["c1", "c2"])
def test_no_false_accepts(gen):
    # A random 256-bit descriptor is within 50 bits of another with
    # probability 5.7e-24: every accepted pair must be a planted one.
    ev = synth.gen_c1() if gen == "c1" else synth.gen_c2()
    out = oracle.search_fuse(ev, use_grid=True)
    acc = np.nonzero((out["decision"] == oracle.ADD) | (out["decision"] == oracle.FUSE))[0]
    kf = np.searchsorted(ev.pair_offset, acc, side="right") - 1
    mp = acc - ev.pair_offset[kf]
    planted = set(zip(ev.planted_kf.tolist(), ev.planted_kp.tolist(), ev.planted_mp.tolist()))
    bad = [(k, b, m) for k, b, m in zip(kf.tolist(), out["best_idx"][acc].tolist(), mp.tolist())
           if (k, b, m) not in planted]
    assert not bad


def _pinhole64(X, S16, cam):
    """Textbook projection through the 3x4 matrix K [A | t] in float64."""
    A = S16[:9].astype(np.float64).reshape(3, 3)
    t = S16[9:12].astype(np.float64)
    K = np.array([[cam[0], 0, cam[2]], [0, cam[1], cam[3]], [0, 0, 1.0]])
    P = K @ np.hstack([A, t[:, None]])
    h = np.hstack([X.astype(np.float64), np.ones((len(X), 1))]) @ P.T
    return h[:, 0] / h[:, 2], h[:, 1] / h[:, 2], h[:, 2]


def test_projection_is_the_textbook_pinhole():
    ev = synth.gen_c2()
    for k in (0, 7, 19):
        u, v, d, pred, vis = oracle.project(ev.mp_xyz, ev.kf_sim3[k], ev.cams[k], ev.mp_dmax)
        U, V, Z = _pinhole64(ev.mp_xyz, ev.kf_sim3[k], ev.cams[k])
        W, H = ev.cams[k][4], ev.cams[k][5]
        vis64 = (Z > 0) & (U >= 0) & (U < W) & (V >= 0) & (V < H)
        inner = vis64 & (U > 1e-2) & (U < W - 1e-2) & (V > 1e-2) & (V < H - 1e-2)
        assert np.array_equal(vis[inner], vis64[inner])
        assert np.max(np.abs(u[inner] - U[inner])) < 2e-3
        assert np.max(np.abs(v[inner] - V[inner])) < 2e-3
        # metric distance: |q| / s with s = |row 0 of sR|
        s = np.linalg.norm(ev.kf_sim3[k][:3].astype(np.float64))
        A = ev.kf_sim3[k][:9].astype(np.float64).reshape(3, 3)
        q = ev.mp_xyz.astype(np.float64) @ A.T + ev.kf_sim3[k][9:12]
        dd = np.linalg.norm(q, axis=1) / s
        assert np.max(np.abs(d[inner] / dd[inner] - 1)) < 1e-5


def test_predicted_octave_is_ceil_log_ratio():
    # pred = ceil(log(dmax/d) / log 1.2) clipped to [0, 7], away from boundaries.
    ev = synth.gen_c1()
    u, v, d, pred, vis = oracle.project(ev.mp_xyz, ev.kf_sim3[0], ev.cams[0], ev.mp_dmax)
    x = np.log(ev.mp_dmax[vis].astype(np.float64) / d[vis]) / np.log(1.2)
    ref = np.clip(np.ceil(x), 0, 7)
    far = np.abs(x - np.round(x)) > 1e-4
    assert np.array_equal(pred[vis][far], ref[far])
    # the anchor keyframe sees every point at its generation octave
    assert far.mean() > 0.99


def test_sim3_rescaling_invariance_exact():
    # (lambda s R, lambda t, inv_s / lambda) with lambda = 2 scales q exactly,
    # leaves q/z and |q| inv_s unchanged, so every output is identical.
    ev = synth.gen_c2(n_kf=4, n_mp=3000)
    base = oracle.search_fuse(ev)
    S2 = ev.kf_sim3.copy()
    S2[:, :12] *= 2
    S2[:, 12] /= 2
    out = oracle.search_fuse(ev, overrides=dict(kf_sim3=S2))
    assert same(base, out)


def test_identity_sim3_exact_planting():
    # Keypoints placed exactly at the float64 projection of their point,
    # with the point's descriptor, are found with distance 0.
    rng = np.random.default_rng(11)
    cam = np.array(synth.CAM_752 + (0.0, 0.0), np.float32)
    n = 300
    u = rng.uniform(20, 730, n)
    v = rng.uniform(20, 460, n)
    z = rng.uniform(1, 10, n)
    X = np.stack([(u - cam[2]) / cam[0] * z, (v - cam[3]) / cam[1] * z, z], 1).astype(np.float32)
    U, V, _ = _pinhole64(X, np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32), cam)
    desc = rng.integers(0, 256, (n, 32), dtype=np.uint8)
    from cases import single_kf_event
    ev = single_kf_event(X, desc, np.ones(n), np.arange(n), np.stack([U, V], 1), np.zeros(n),
                         desc, -np.ones(n), [1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], cam,
                         synth.LoopParams())
    out = oracle.search_fuse(ev)
    assert np.array_equal(out["best_idx"], np.arange(n))
    assert np.all(out["best_dist"] == 0)
    assert np.all(out["decision"] == oracle.ADD)


def test_fp64_census_hand_case():
    # Points placed at known float32/float64 offsets from window and image
    # edges (tests/golden/census_hand_case.json): each count derived by hand.
    from cases import census_case
    ev, eps, exp = census_case()
    r = oracle.census_fp64(ev, eps=eps)
    assert r == exp, (r, exp)
    # every point moved 1 px right and 1 px down in the image: each keypoint
    # and image edge is then about 1 px from the nearest window or image edge
    X = ev.mp_xyz.copy()
    X[:, 0] += X[:, 2]
    X[:, 1] += X[:, 2]
    far = oracle.census_fp64(ev, eps=eps, overrides=dict(mp_xyz=X))
    assert far == dict(n=8, n_diff=0, n_near_window=0, n_near_image=0), far


# Census rates of the synthetic workloads (pairs examined, result-changing
# pairs, keypoints within 1e-3 px of a window edge, projections within 1e-3
# px of an image edge), recorded from this oracle.  The result-changing rate
# must stay below 0.01%; the window-edge rate is a property of the keypoint
# density (about density x window perimeter x 2 eps per visible pair) and is
# recorded, with the 0.01% target met on C1 and C2 and missed on C3.
CENSUS = {"c1": (2000, 0, 0, 0), "c2": (300000, 0, 26, 3), "c3": (466090, 1, 62, 11)}


@pytest.mark.parametrize("gen", ["c1", "c2", "c3"])
def test_fp64_boundary_census(gen):
    ev = {"c1": synth.gen_c1, "c2": synth.gen_c2, "c3": synth.gen_c3}[gen]()
    r = oracle.census_fp64(ev, eps=1e-3)
    n = r["n"]
    assert r["n_diff"] / n < 1e-4, r
    assert (n, r["n_diff"], r["n_near_window"], r["n_near_image"]) == CENSUS[gen], r


def test_edge_cases():
    ev = synth.gen_tiny(5, n_kf=3, n_mp=120, n_kp=(20, 40))
    out = oracle.search_fuse(ev)
    # points behind the camera, NaN and Inf coordinates are NOT_VISIBLE
    X = ev.mp_xyz.copy()
    X[0] = [np.nan, 0, 1]
    X[1] = [0, 0, np.inf]
    X[2] = [0, np.inf, 5]
    S = ev.kf_sim3
    bad = oracle.search_fuse(ev, overrides=dict(mp_xyz=X))
    for k in range(ev.n_kf):
        for p in (0, 1, 2):
            o = ev.pair_offset[k] + p
            if out["decision"][o] != oracle.SKIP:
                assert bad["decision"][o] == oracle.NOT_VISIBLE
                assert bad["best_idx"][o] == -1 and bad["best_dist"][o] == oracle.NO_DIST
    # an empty keyframe: nothing to match
    kp_off = ev.kp_offset.copy()
    n0 = kp_off[1]
    empty = dict(kp_offset=np.concatenate([[0, 0], kp_off[2:] - n0]).astype(np.int32),
                 kp_xy=ev.kp_xy[n0:].copy(), kp_oct=ev.kp_oct[n0:].copy(),
                 kp_desc=ev.kp_desc[n0:].copy(), kp_owner=ev.kp_owner[n0:].copy())
    e = oracle.search_fuse(ev, overrides=empty)
    d0 = e["decision"][: ev.pair_offset[1]]
    assert set(np.unique(d0).tolist()) <= {oracle.NOT_VISIBLE, oracle.NO_MATCH}
    assert np.all(e["best_idx"][: ev.pair_offset[1]] == -1)
    for k in FIELDS:   # other keyframes unaffected
        assert np.array_equal(e[k][ev.pair_offset[1]:], out[k][ev.pair_offset[1]:])
    # sparse pairs naming a point outside the event are INVALID
    sp = synth.gen_tiny(6, n_kf=2, n_mp=50, n_kp=(10, 20), sparse=True)
    pm = sp.pair_mp.copy()
    pm[0] = -1
    pm[-1] = 50
    r = oracle.search_fuse(sp, overrides=dict(pair_mp=pm))
    assert r["decision"][0] == oracle.INVALID and r["decision"][-1] == oracle.INVALID
    # no points at all
    z = oracle.search_fuse(ev, overrides=dict(pair_offset=np.zeros(ev.n_kf + 1, np.int64)))
    assert len(z["decision"]) == 0
    del S


def test_octave_extremes_and_threshold():
    ev, _ = hand_case()
    # octave gate at pred = 0 admits octave -1 and 0 only; with dmax absent the
    # gate is off and pred = n_octaves - 1 (largest window)
    out = oracle.search_fuse(ev, use_dmax=False)
    # point 5 now sees kp12 (octave 3): candidate, h = 0 -> accepted ADD
    assert out["best_idx"][5] == 12 and out["decision"][5] == oracle.ADD
    # threshold 49 rejects point 6 (h = 50); threshold 51 accepts point 7
    p49 = synth.LoopParams(**{**ev.params.__dict__, "hamming_th": 49})
    assert oracle.search_fuse(ev, params=p49)["decision"][6] == oracle.NO_MATCH
    p51 = synth.LoopParams(**{**ev.params.__dict__, "hamming_th": 51})
    assert oracle.search_fuse(ev, params=p51)["decision"][7] == oracle.ADD
    # ratio test 0.8: point 0 (10 < 0.8*20) keeps its match, point 9 (7 vs 7) loses it
    pr = synth.LoopParams(**{**ev.params.__dict__, "nn_ratio": 0.8})
    r = oracle.search_fuse(ev, params=pr)
    assert r["decision"][0] == oracle.ADD and r["decision"][9] == oracle.NO_MATCH


def test_grid_is_a_stable_counting_sort_by_cell():
    ev = synth.gen_c3(n_kf=3, n_mp=1000)
    p = ev.params
    for k in range(ev.n_kf):
        a, b = int(ev.kp_offset[k]), int(ev.kp_offset[k + 1])
        xy = ev.kp_xy[a:b]
        cs, ck = oracle.build_grid(xy, ev.cams[k], p)
        # every keypoint lies in the cell it is listed under, in float64
        cw = ev.cams[k][4] / p.grid_cols
        ch = ev.cams[k][5] / p.grid_rows
        cells = np.repeat(np.arange(p.grid_cols * p.grid_rows), np.diff(cs))
        cx, cy = cells % p.grid_cols, cells // p.grid_cols
        x, y = xy[ck, 0].astype(np.float64), xy[ck, 1].astype(np.float64)
        inner = (x > 0) & (x < ev.cams[k][4]) & (y > 0) & (y < ev.cams[k][5])
        assert np.all((x[inner] >= cx[inner] * cw - 1e-3) & (x[inner] <= (cx[inner] + 1) * cw + 1e-3))
        assert np.all((y[inner] >= cy[inner] * ch - 1e-3) & (y[inner] <= (cy[inner] + 1) * ch + 1e-3))
        assert sorted(ck.tolist()) == list(range(b - a))
        for c in range(len(cs) - 1):
            seg = ck[cs[c]:cs[c + 1]]
            assert np.all(np.diff(seg) > 0)
