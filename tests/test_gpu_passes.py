"""GPU parity of several searches of one resident batch in one launch (the
concurrent projection searches of task parallelism, Sec. IV-C): every pass
bit-exact against the oracle run on that pass's transforms and thresholds,
on one keyframe, a dense loop event, a sparse uneven event, the global-grid
staging mode, the list-overflow path and the most passes; and the rejected
arguments."""
import dataclasses

import pytest

import oracle
import synth
from cases import with_near_duplicates
from gpu_util import FIELDS, assert_same, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2603_17201_amd as fl
    c = fl.Context(0)
    yield c
    c.close()


def run_passes(ctx, ev, passes):
    import paper_2603_17201_amd as fl
    b = fl.DeviceBatch(ev, device=dev())
    outs = ctx.search_fuse_passes(b, [(P, S, None) for P, S in passes])
    return [o.numpy() for o in outs]


def expected(ev, passes, use_grid=True):
    return [oracle.search_fuse(dataclasses.replace(ev, kf_sim3=S), params=P, use_grid=use_grid)
            for P, S in passes]


def check(ctx, ev, passes, label, use_grid=True):
    got = run_passes(ctx, ev, passes)
    exp = expected(ev, passes, use_grid)
    for p, (g, e) in enumerate(zip(got, exp)):
        assert_same(g, e, f"{label} pass {p}")
    return got, exp


def test_two_searches_on_one_keyframe(ctx):
    """The searches before and after the Sim3 optimisation on the current
    keyframe: different transforms, windows and ratios, one launch."""
    ev = with_near_duplicates(synth.gen_c1())
    passes = synth.ps2_passes(ev)
    got, exp = check(ctx, ev, passes, "ps2", use_grid=False)
    # the passes do differ, and each equals its own single-pass batched call
    assert any((got[0][k] != got[1][k]).any() for k in FIELDS)
    import paper_2603_17201_amd as fl
    b = fl.DeviceBatch(dataclasses.replace(ev, kf_sim3=passes[1][1]), device=dev())
    assert_same(ctx.search_fuse_batched(b, passes[1][0]).numpy(), got[1], "pass 1 vs single-pass call")


def test_three_passes_loop_event(ctx):
    ev = synth.gen_c2(n_kf=6, n_mp=6000)
    S2 = synth.search_transforms(ev, synth.perturbed(ev.S_init, 0.2, 0.02, 0.003, seed=11))
    passes = [(synth.LoopParams(), ev.kf_sim3),
              (synth.verification_params(), ev.kf_sim3),
              (synth.LoopParams(win_px=5.0, nn_ratio=0.9, hamming_th=40), S2)]
    check(ctx, ev, passes, "c2x3")


def test_passes_sparse_uneven_event(ctx):
    ev = synth.gen_c3(n_kf=24, n_mp=8000)
    check(ctx, ev, synth.ps2_passes(ev, seed=9), "c3x2")


@pytest.mark.parametrize("lds_mode", [0, 1])
def test_passes_other_staging_modes(ctx, lds_mode):
    """Global grids (built once per keyframe, shared by its passes) and the
    records-only LDS mode."""
    ev = synth.gen_c2(n_kf=5, n_mp=5000)
    ctx.set_tuning(1, lds_mode, 1, 1)
    try:
        check(ctx, ev, synth.ps2_passes(ev, seed=3), f"mode {lds_mode}")
    finally:
        ctx.set_tuning()


def test_most_passes_with_list_overflow(ctx):
    """FL_MAX_PASSES passes, with the ADD lists capped so that the
    resolution scans each pass's decisions against its own claims."""
    import paper_2603_17201_amd as fl
    ev = synth.gen_c2(n_kf=4, n_mp=4000, skip_frac=0.02)
    passes = [(synth.LoopParams(win_px=w), synth.search_transforms(
        ev, synth.perturbed(ev.S_init, 0.05 * i, 0.005 * i, 0.001 * i, seed=21 + i)))
        for i, w in enumerate((3.0, 4.0, 6.0, 8.0))]
    assert len(passes) == fl._abi.MAX_PASSES
    check(ctx, ev, passes, "4 passes")
    ctx.debug_set_list_cap(16)
    try:
        check(ctx, ev, passes, "4 passes, overflow")
    finally:
        ctx.debug_set_list_cap(0)


def test_rejected_arguments(ctx):
    import paper_2603_17201_amd as fl
    ev = synth.gen_c1()
    b = fl.DeviceBatch(ev, device=dev())
    P = synth.verification_params()
    with pytest.raises(fl.FlError):
        ctx.search_fuse_passes(b, [])
    with pytest.raises(fl.FlError):
        ctx.search_fuse_passes(b, [(P, None, None)] * (fl._abi.MAX_PASSES + 1))
    with pytest.raises(fl.FlError):   # grid differs from pass 0
        ctx.search_fuse_passes(b, [(P, None, None), (synth.LoopParams(grid_cols=32), None, None)])
    out = fl.FuseOutputs.empty(b.n_pairs, dev())
    with pytest.raises(fl.FlError):   # two passes writing the same arrays
        ctx.search_fuse_passes(b, [(P, None, out), (P, None, out)])
