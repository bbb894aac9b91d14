"""GPU parity of search-and-fuse against the CPU oracle: every output of every
pair bit-exact, for the plain per-keyframe path, the batched persistent path
and the graph-replayed path, on the hand-worked case, small ragged events,
the full loop-event workloads, multi-event batches, every tuning and the
list-overflow paths."""
import itertools

import numpy as np
import pytest
import torch

import oracle
import synth
from cases import conflict_case, hand_case, with_near_duplicates
from gpu_util import FIELDS, assert_same, dev, plain_per_keyframe, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2603_17201_amd as fl
    c = fl.Context(0)
    yield c
    c.close()


def batched(ctx, src, params=None, graph=False, use_dmax=True, use_id=True):
    import paper_2603_17201_amd as fl
    b = fl.DeviceBatch(src, device=dev(), use_dmax=use_dmax, use_id=use_id)
    p = params if params is not None else src.params
    out = ctx.search_fuse_graph(b, p) if graph else ctx.search_fuse_batched(b, p)
    return out.numpy()


def test_hand_case(ctx):
    ev, exp = hand_case()
    for mode in ("plain", "batched", "graph"):
        got = plain_per_keyframe(ctx, ev, ev.params) if mode == "plain" else batched(ctx, ev, graph=mode == "graph")
        assert_same(got, exp, mode)


@pytest.mark.parametrize("order", [list(p) for p in itertools.islice(itertools.permutations(range(6)), 0, 720, 181)])
def test_conflict_rule(ctx, order):
    ev = conflict_case(order)
    exp = oracle.search_fuse(ev)
    assert_same(plain_per_keyframe(ctx, ev, ev.params), exp, "plain")
    assert_same(batched(ctx, ev), exp, "batched")


@pytest.mark.parametrize("seed", range(10))
def test_tiny_events(ctx, seed):
    sparse = seed % 3 == 2
    ev = synth.gen_tiny(100 + seed, n_kf=1 + seed % 5, n_mp=37 + 61 * seed, n_kp=(3 + seed, 90 + 40 * seed),
                        sparse=sparse, skip_frac=0.05)
    for use_dmax, use_id in [(True, True), (False, True), (True, False)]:
        exp = oracle.search_fuse(ev, use_dmax=use_dmax, use_id=use_id)
        assert_same(batched(ctx, ev, use_dmax=use_dmax, use_id=use_id), exp, f"batched {seed} {use_dmax} {use_id}")
        assert_same(plain_per_keyframe(ctx, ev, ev.params, use_dmax, use_id), exp, f"plain {seed}")


def test_c1_single_call(ctx):
    ev = synth.gen_c1()
    exp = oracle.search_fuse(ev, use_grid=True)
    assert_same(plain_per_keyframe(ctx, ev, ev.params), exp, "plain")
    assert_same(plain_per_keyframe(ctx, ev, ev.params, with_grid=True), exp, "plain+grid")
    assert_same(batched(ctx, ev), exp, "batched")


@pytest.fixture(scope="module")
def c2():
    ev = synth.gen_c2(skip_frac=0.05)
    return ev, oracle.search_fuse(ev, use_grid=True)


def test_c2_plain(ctx, c2):
    ev, exp = c2
    assert_same(plain_per_keyframe(ctx, ev, ev.params), exp, "plain")


def test_c2_batched_and_graph(ctx, c2):
    ev, exp = c2
    assert_same(batched(ctx, ev), exp, "batched")
    for _ in range(3):   # replays of the captured graph
        assert_same(batched(ctx, ev, graph=True), exp, "graph")


def test_c2_every_tuning_and_repeat(ctx, c2):
    import paper_2603_17201_amd as fl
    ev, exp = c2
    b = fl.DeviceBatch(ev, device=dev())
    try:
        for ppl, mode, wpc, xa in itertools.product((1, 2, 4), (0, 1, 2), (1, 2), (0, 1)):
            ctx.set_tuning(ppl, mode, wpc, xa)
            got = ctx.search_fuse_batched(b, ev.params).numpy()
            assert_same(got, exp, f"tuning {ppl} {mode} {wpc} {xa}")
    finally:
        ctx.set_tuning()
    first = ctx.search_fuse_batched(b, ev.params).numpy()
    for _ in range(5):
        assert_same(ctx.search_fuse_batched(b, ev.params).numpy(), first, "repeat")


def test_c2_stats_match_oracle_counters(ctx, c2):
    import paper_2603_17201_amd as fl
    ev, exp = c2
    b = fl.DeviceBatch(ev, device=dev())
    ctx.set_stats(True)
    try:
        got = ctx.search_fuse_batched(b, ev.params).numpy()
        torch.cuda.synchronize()
        st = ctx.get_stats()
    finally:
        ctx.set_stats(False)
    assert_same(got, exp, "stats run")
    for k in ("n_visible", "n_cells", "n_kp_scanned", "n_cand"):
        assert st[k] == exp[k], (k, st[k], exp[k])


def test_list_overflow_paths(ctx):
    ev = synth.gen_c2(n_kf=4, n_mp=4000, skip_frac=0.02)
    exp = oracle.search_fuse(ev)
    ctx.debug_set_list_cap(16)
    try:
        assert_same(batched(ctx, ev), exp, "batched overflow")
        assert_same(plain_per_keyframe(ctx, ev, ev.params), exp, "plain overflow")
    finally:
        ctx.debug_set_list_cap(0)


def test_c3_sparse_pairs(ctx):
    ev = synth.gen_c3()
    exp = oracle.search_fuse(ev, use_grid=True)
    assert_same(batched(ctx, ev), exp, "c3 batched")
    assert_same(batched(ctx, ev, graph=True), exp, "c3 graph")


def test_multi_event_batch(ctx):
    evs = [synth.gen_c3(seed=310 + i, n_kf=8 + 5 * i, n_mp=3000 + 1000 * i, id_base=1000 + 10 ** 6 * i,
                        fresh_base=10 ** 9 + 10 ** 7 * i) for i in range(3)]
    evs.append(synth.gen_tiny(55, n_kf=3, n_mp=500))
    B = synth.concat_events(evs)
    exp = oracle.search_fuse(B, use_grid=True)
    assert_same(batched(ctx, B), exp, "multi batched")
    assert_same(batched(ctx, B, graph=True), exp, "multi graph")


def test_edge_cases(ctx):
    import paper_2603_17201_amd as fl
    ev = synth.gen_tiny(7, n_kf=3, n_mp=150, n_kp=(20, 40))
    # NaN / Inf coordinates and a point behind every camera
    X = ev.mp_xyz.copy()
    X[0] = [np.nan, 0, 1]
    X[1] = [0, 0, np.inf]
    X[2] = [0, 0, -1e6]
    ev.mp_xyz = X
    exp = oracle.search_fuse(ev)
    assert_same(batched(ctx, ev), exp, "nonfinite")
    assert_same(plain_per_keyframe(ctx, ev, ev.params), exp, "nonfinite plain")
    # an empty keyframe in the middle of a batch
    n0, n1 = int(ev.kp_offset[1]), int(ev.kp_offset[2])
    keep = np.r_[0:n0, n1:int(ev.kp_offset[-1])]
    ev.kp_offset = np.array([0, n0, n0, n0 + int(ev.kp_offset[-1]) - n1], np.int32)
    ev.kp_xy, ev.kp_oct, ev.kp_desc, ev.kp_owner = (ev.kp_xy[keep], ev.kp_oct[keep], ev.kp_desc[keep],
                                                    ev.kp_owner[keep])
    exp = oracle.search_fuse(ev)
    assert_same(batched(ctx, ev), exp, "empty keyframe")
    assert_same(plain_per_keyframe(ctx, ev, ev.params), exp, "empty keyframe plain")
    # sparse pairs naming points outside the event
    sp = synth.gen_tiny(8, n_kf=2, n_mp=60, n_kp=(10, 30), sparse=True)
    sp.pair_mp = sp.pair_mp.copy()
    sp.pair_mp[0] = -5
    sp.pair_mp[-1] = 60
    exp = oracle.search_fuse(sp)
    assert exp["decision"][0] == oracle.INVALID
    assert_same(batched(ctx, sp), exp, "invalid pairs")
    # no pairs at all
    b = fl.DeviceBatch(ev, device=dev())
    b.h_pair_offset = np.zeros_like(b.h_pair_offset)
    b.n_pairs = 0
    b.pair_mp = t(np.zeros(1, np.int32))
    out = ctx.search_fuse_batched(b, ev.params)
    assert out.decision.numel() == 0


def test_grid_build_matches_definition(ctx):
    ev = synth.gen_c3(n_kf=4, n_mp=2000)
    p = ev.params
    for k in range(ev.n_kf):
        a, b = int(ev.kp_offset[k]), int(ev.kp_offset[k + 1])
        xy = ev.kp_xy[a:b]
        cs, ck = ctx.build_grid(t(xy), ev.cams[k], p)
        cs, ck = cs.cpu().numpy(), ck.cpu().numpy()
        ecs, eck = oracle.build_grid(xy, ev.cams[k], p)
        assert np.array_equal(cs, ecs) and np.array_equal(ck, eck)


def test_host_validation_errors(ctx):
    import paper_2603_17201_amd as fl
    ev = synth.gen_tiny(9, n_kf=2, n_mp=50)
    b = fl.DeviceBatch(ev, device=dev())
    bad = synth.LoopParams(n_octaves=40)
    with pytest.raises(fl.FlError) as e:
        ctx.search_fuse_batched(b, bad)
    assert e.value.code == -4
    with pytest.raises(ValueError):   # host tensor where a device tensor is required
        ctx.search_fuse(torch.zeros((4, 3)), t(np.zeros((4, 32), np.uint8)), None, None,
                        t(np.zeros((1, 2), np.float32)), t(np.zeros(1, np.int8)), t(np.zeros((1, 32), np.uint8)),
                        t(np.zeros(1, np.int32)), np.zeros(16, np.float32), ev.cams[0], ev.params)


def test_valu_rate_probe(ctx):
    # the issue-rate probe used for roofline reporting: a plausible rate
    # (between 1 and 200 T lane-ops/s) and its argument range enforced
    rate = ctx.valu_rate(iters=2000)
    assert 1e12 < rate < 2e14, rate
    import paper_2603_17201_amd as fl
    with pytest.raises(ValueError):
        ctx.valu_rate(iters=0)
    assert fl.last_error()


def test_staging_ring_reuse_with_changing_tables(ctx):
    # 60 eager calls cycling through three batches: every call uploads new
    # tables, so each staging buffer is rewritten several times, each time
    # after a fence that follows its previous fetch; every result must hold
    import paper_2603_17201_amd as fl
    evs = [synth.gen_tiny(70 + i, n_kf=2 + i, n_mp=300 + 50 * i) for i in range(3)]
    exps = [oracle.search_fuse(ev) for ev in evs]
    bs = [fl.DeviceBatch(ev, device=dev()) for ev in evs]
    outs = [fl.FuseOutputs.empty(b.n_pairs, dev()) for b in bs]
    for it in range(60):
        i = it % 3
        ctx.search_fuse_batched(bs[i], evs[i].params, outs[i])
        if it % 7 == 0 or it >= 57:
            assert_same(outs[i].numpy(), exps[i], f"call {it}")


def test_graph_ring_reuse_with_changing_tables(ctx):
    # 30 graph launches cycling through three batches of one shape (so the
    # captured graphs are reused): each graph's table buffer is rewritten
    # after a fence that follows its previous replay; every result must hold
    import paper_2603_17201_amd as fl
    evs = [synth.gen_tiny(80 + i, n_kf=3, n_mp=400) for i in range(3)]
    exps = [oracle.search_fuse(ev) for ev in evs]
    bs = [fl.DeviceBatch(ev, device=dev()) for ev in evs]
    outs = [fl.FuseOutputs.empty(b.n_pairs, dev()) for b in bs]
    for it in range(30):
        i = it % 3
        ctx.search_fuse_graph(bs[i], evs[i].params, outs[i])
        if it % 4 == 0 or it >= 27:
            assert_same(outs[i].numpy(), exps[i], f"graph call {it}")


def _accepted(o):
    return int(((o["decision"] == oracle.ADD) | (o["decision"] == oracle.FUSE)).sum())


def test_projection_search_one_keyframe(ctx):
    """Loop verification's single projection search: every point against one
    keyframe with near-duplicate keypoints, the wider window and the ratio
    test on; the plain call and a batched launch, bit-exact."""
    ev = with_near_duplicates(synth.gen_c1())
    P = synth.verification_params()
    exp = oracle.search_fuse(ev, params=P)
    loose = oracle.search_fuse(ev, params=synth.LoopParams(win_px=P.win_px))
    assert _accepted(exp) < _accepted(loose)   # the ratio test rejects some matches here
    assert_same(plain_per_keyframe(ctx, ev, P), exp, "PS1 plain")
    assert_same(batched(ctx, ev, params=P), exp, "PS1 batched")
    assert_same(batched(ctx, ev, params=P, graph=True), exp, "PS1 graph")


def test_projection_search_three_keyframes_one_launch(ctx):
    """Loop verification's triple projection search in one launch: the same
    points against three keyframes (one event, dense pairs), and three
    independent one-keyframe searches batched together; ratio test on."""
    P = synth.verification_params()
    ev = synth.gen_c2(seed=212, n_kf=3, n_mp=15000)
    exp = oracle.search_fuse(ev, params=P, use_grid=True)
    assert_same(batched(ctx, ev, params=P), exp, "PS3 one event")
    assert_same(batched(ctx, ev, params=P, graph=True), exp, "PS3 one event, graph")
    evs = [with_near_duplicates(synth.gen_c1(seed=101 + i), seed=7 + i) for i in range(3)]
    B = synth.concat_events(evs)
    exp3 = oracle.search_fuse(B, params=P)
    assert _accepted(exp3) < _accepted(oracle.search_fuse(B, params=synth.LoopParams(win_px=P.win_px)))
    assert_same(batched(ctx, B, params=P), exp3, "PS3 three events")


def test_c2_with_ratio_test(ctx):
    """The full loop event with the ratio test on (0.75) and the fusion
    window."""
    ev = synth.gen_c2()
    P = synth.LoopParams(nn_ratio=0.75)
    exp = oracle.search_fuse(ev, params=P, use_grid=True)
    assert_same(batched(ctx, ev, params=P), exp, "c2 ratio")


def test_keyframe_at_the_packed_key_limit(ctx):
    # a keyframe of FL_MAX_KP = 65,535 keypoints (the 16-bit index of the
    # packed key) between two ordinary ones: too large for LDS, so the
    # batched launch takes its global-grid mode; the plain path runs each
    # keyframe on its own
    import paper_2603_17201_amd as fl
    ev = synth.gen_c2(seed=515, n_mp=4000, kp_counts=[1200, fl.MAX_KP, 1200])
    exp = oracle.search_fuse(ev, use_grid=True)
    assert int(exp["best_idx"].max()) > 60000   # indices near the limit are matched
    assert_same(batched(ctx, ev), exp, "batched")
    assert_same(batched(ctx, ev, graph=True), exp, "graph")
    assert_same(plain_per_keyframe(ctx, ev, ev.params), exp, "plain")


@pytest.mark.parametrize("big", [6000, 20000])
def test_one_large_keyframe_among_small_ones(ctx, big):
    # one keyframe of `big` keypoints among 1,200-keypoint ones: the LDS
    # footprint is sized by the largest, so the launch stages fewer octave
    # buckets (6,000) or falls back to global grids (20,000) for every
    # keyframe; every tuning stays bit-exact
    ev = synth.gen_c2(seed=616 + big, n_mp=3000, kp_counts=[1200, 1200, big, 1200, 1200])
    exp = oracle.search_fuse(ev, use_grid=True)
    saved = ctx.get_tuning()
    try:
        for ppl, mode in itertools.product((1, 2, 4), (0, 1, 2)):
            ctx.set_tuning(ppl, mode, 1, 1)
            assert_same(batched(ctx, ev), exp, f"ppl {ppl} mode {mode}")
    finally:
        ctx.set_tuning(saved.pairs_per_lane, saved.lds_mode, saved.wg_per_cu, saved.xcd_aware)
