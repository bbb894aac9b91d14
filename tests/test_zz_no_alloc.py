"""The allocation-free plain search (fl_search_fuse_noalloc, its scratch in a
static device array) against the plain search with the context's workspace
(fl_search_fuse): every output bit-exact on two calls in a row, the second
with a smaller input (the static array keeps the first call's contents),
and the second call against the oracle as well."""
import pytest

import oracle
import synth
from gpu_util import FIELDS, assert_same, t

pytestmark = pytest.mark.gpu


def _both(ctx, ev, k):
    import paper_2603_17201_amd as fl
    a, b = int(ev.kp_offset[k]), int(ev.kp_offset[k + 1])
    args = (t(ev.mp_xyz), t(ev.mp_desc), t(ev.mp_dmax), t(ev.mp_id), t(ev.kp_xy[a:b]), t(ev.kp_oct[a:b]),
            t(ev.kp_desc[a:b]), t(ev.kp_owner[a:b]), ev.kf_sim3[k], ev.cams[k], ev.params)
    ref = ctx.search_fuse(*args).numpy()
    got = fl.search_fuse_noalloc(*args).numpy()
    return got, ref


def test_noalloc_matches_workspace_search_on_two_calls_the_second_smaller():
    import paper_2603_17201_amd as fl
    ctx = fl.Context(0)
    try:
        big = synth.gen_c2(seed=909, n_kf=2, n_mp=6000)      # 1,200 keypoints, 6,000 points
        small = synth.gen_tiny(4243, n_kf=1, n_mp=700, n_kp=(150, 160))
        got, ref = _both(ctx, big, 1)
        assert_same(got, ref, "first call")
        got, ref = _both(ctx, small, 0)
        assert_same(got, ref, "second, smaller call")
        exp = oracle.search_fuse(small)
        assert_same(got, {f: exp[f] for f in FIELDS}, "second call against the oracle")
    finally:
        ctx.close()
