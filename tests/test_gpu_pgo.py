"""GPU parity of the essential-graph optimisation (exact Jacobians,
Levenberg-Marquardt) against the float64 oracle, for every solver (banded
Cholesky through an LDS window or through device memory, conjugate
gradients): exact recovery of a consistent graph, the
oracle's poses, cost history, damping and accept/refuse sequence on noisy
graphs (Gauss-Newton, small and large damping, a start that makes the
undamped step overshoot, several held nodes, the smallest graphs, several
band windows, graphs of several loops up to the widest band the direct
solver takes), the two band windows' identical results, the solver choice
and its limit, and convergence and determinism on 1,000 keyframes on one and
on three laps."""
import numpy as np
import pytest
import torch

import synth
from oracle import pgo, sim3
from gpu_util import dev, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2603_17201_amd as fl
    c = fl.Context(0)
    yield c
    c.close()


def _err(A, B):
    return max(np.linalg.norm(sim3.log(sim3.compose(a, sim3.inverse(b)))) for a, b in zip(A, B))


def _run(ctx, d, fixed=None, **kw):
    S = t(d["S0"].copy())
    cost, used, lams, acc = ctx.pose_graph_optimize(S, t(d["M"]), d["edges"], fixed, history=True, **kw)
    return S.cpu().numpy(), cost.cpu().numpy(), used.cpu().numpy(), lams.cpu().numpy(), acc.cpu().numpy()


def _oracle(d, fixed=None, iters=3, lam=1e-4, S0=None):
    h, lams, acc = [], [], []
    S = pgo.optimize(d["S0"] if S0 is None else S0, d["edges"], d["M"], d["fixed"] if fixed is None else fixed,
                     iters=iters, lam=lam, history=h, lambdas=lams, accepted=acc)
    return S, np.array(h), np.array(lams), np.array(acc, np.uint8)


CG, DIRECT, DIRECT_WIDE = 1, 2, 3


@pytest.mark.parametrize("solver", [CG, DIRECT, DIRECT_WIDE])
def test_consistent_graph_is_recovered_exactly(ctx, solver):
    d = synth.gen_pose_graph(n=12, seed=11, covis=2, n_loops=2, noise_deg=0.0, noise_m=0.0, noise_scale=0.0)
    S, cost, used, lams, acc = _run(ctx, d, iters=6, cg_tol=1e-13, solver=solver)
    assert _err(S, d["S_true"]) < 1e-9
    assert cost[-1] < 1e-18 < cost[0]
    assert np.array_equal(S[0], d["S0"][0])


@pytest.mark.parametrize("solver", [CG, DIRECT, DIRECT_WIDE])
@pytest.mark.parametrize("lam", [0.0, 1e-4, 0.1])
def test_noisy_graph_matches_oracle(ctx, lam, solver):
    # three iterations: every decision has a relative margin above 1e-7
    d = synth.gen_pose_graph(n=14, seed=13, covis=2, n_loops=3)
    S_ref, h, lams_ref, acc_ref = _oracle(d, iters=3, lam=lam)
    S, cost, used, lams, acc = _run(ctx, d, iters=3, lam=lam, cg_tol=1e-14, cg_iters=2000, solver=solver)
    tol = 1e-8 if solver == CG else 1e-9
    assert _err(S, S_ref) < tol, _err(S, S_ref)
    assert np.max(np.abs(cost - h) / h) < 1e-9
    assert np.array_equal(acc, acc_ref) and np.array_equal(lams, lams_ref), (acc, acc_ref, lams, lams_ref)
    assert all(u > 0 for u in used) if solver == CG else all(u == 0 for u in used)


@pytest.mark.parametrize("solver", [CG, DIRECT, DIRECT_WIDE])
def test_refused_steps_match_oracle(ctx, solver):
    """Three free keyframes start 2-3 rad off: the undamped steps overshoot,
    the iterations are refused, the damping grows and the poses are kept
    until the steps are short enough; the device follows the oracle's
    accept/refuse sequence (every decision far from a tie) exactly."""
    from cases import overshoot_graph
    d = overshoot_graph()
    S_ref, h, lams_ref, acc_ref = _oracle(d, iters=8, lam=1e-6)
    assert not acc_ref.all()
    S, cost, used, lams, acc = _run(ctx, d, iters=8, lam=1e-6, cg_tol=1e-14, cg_iters=2000, solver=solver)
    assert np.array_equal(acc, acc_ref) and np.array_equal(lams, lams_ref), (acc, acc_ref)
    assert np.max(np.abs(cost - h) / h) < 1e-9
    assert _err(S, S_ref) < (1e-8 if solver == CG else 1e-9)
    k = int(np.argmin(acc))
    assert cost[k + 1] == cost[k]


@pytest.mark.parametrize("solver", [CG, DIRECT, DIRECT_WIDE])
def test_several_held_nodes(ctx, solver):
    d = synth.gen_pose_graph(n=12, seed=17, covis=2, n_loops=2)
    fixed = np.zeros(12, bool)
    fixed[[0, 5, 9]] = True
    S_ref, _, _, _ = _oracle(d, fixed=fixed, iters=2)
    S, _, _, _, _ = _run(ctx, d, fixed=fixed, iters=2, cg_tol=1e-14, cg_iters=2000, solver=solver)
    for n in (0, 5, 9):
        assert np.array_equal(S[n], d["S0"][n])
    assert _err(S, S_ref) < 1e-8


@pytest.mark.parametrize("kw", [
    dict(n=2, covis=1, n_loops=0),     # one free keyframe: a single 7x7 block
    dict(n=3, covis=2, n_loops=0),     # band as tall as the matrix
    dict(n=30, covis=5, n_loops=3),    # reordered span of 11 keyframes: the widest band taken
    dict(n=60, covis=4, n_loops=6),    # 413 unknowns through a window of 63 rows
], ids=["n2", "n3", "widest", "windows"])
def test_direct_solve_matches_oracle(ctx, kw):
    d = synth.gen_pose_graph(seed=29, **kw)
    S_ref, h, lams_ref, acc_ref = _oracle(d, iters=2)
    S, cost, used, lams, acc = _run(ctx, d, iters=2, solver=DIRECT)
    assert all(u == 0 for u in used)
    assert _err(S, S_ref) < 1e-9, _err(S, S_ref)
    # a graph with one edge is solved exactly: its later costs are rounding
    # (about 1e-26), compared against an absolute floor
    assert np.all(np.abs(cost - h) <= 1e-9 * h + 1e-20)
    assert np.array_equal(S[0], d["S0"][0])


def _rcm_band(d):
    """The reordered band, in keyframes, that the library computes: reverse
    Cuthill-McKee over the free nodes (breadth-first from a free node of
    least degree in each component, neighbours by rising degree, then
    index), the widest span of an edge between free nodes, plus one."""
    n, held = len(d["S0"]), np.asarray(d["fixed"], bool)
    deg, adj = np.zeros(n, int), [[] for _ in range(n)]
    for i, j in d["edges"]:
        adj[i].append(j)
        adj[j].append(i)
        if not held[i] and not held[j]:
            deg[i] += 1
            deg[j] += 1
    seen, seq = np.zeros(n, bool), []
    for r in sorted((v for v in range(n) if not held[v]), key=lambda v: deg[v]):
        if seen[r]:
            continue
        seen[r] = True
        head = len(seq)
        seq.append(r)
        while head < len(seq):
            v = seq[head]
            head += 1
            nb = [u for u in adj[v] if not held[u] and not seen[u]]
            seen[nb] = True
            seq.extend(sorted(nb, key=lambda u: (deg[u], u)))
    pos = -np.ones(n, int)
    pos[np.array(seq[::-1], int)] = np.arange(len(seq))
    return 1 + max(abs(pos[i] - pos[j]) for i, j in d["edges"] if pos[i] >= 0 and pos[j] >= 0)


def test_solver_choice_and_band_limit(ctx):
    """Automatic choice: direct on a loop (band of 7 keyframes) and on a
    graph of several loops (a band of 22), conjugate gradients where the
    reordered band spans more keyframes than the direct solver takes; asking
    for a direct solve there is an error, and so is an unknown solver."""
    import paper_2603_17201_amd as fl
    loop = synth.gen_pose_graph(n=40, seed=31, covis=3, n_loops=3)
    _, _, used, _, _ = _run(ctx, loop, iters=2)
    assert all(u == 0 for u in used)
    laps = synth.gen_pose_graph(n=150, seed=31, laps=3, cross=3)
    assert _rcm_band(laps) == 22
    _, _, used, _, _ = _run(ctx, laps, iters=1)
    assert all(u == 0 for u in used)
    over = synth.gen_pose_graph(n=70, seed=31, covis=64, n_loops=0)
    assert _rcm_band(over) == fl.PGO_MAX_BAND_NODES + 1
    S_ref, _, _, _ = _oracle(over, iters=1)
    S, _, used, _, _ = _run(ctx, over, iters=1, cg_tol=1e-14, cg_iters=3000)
    assert all(u > 0 for u in used)
    assert _err(S, S_ref) < 1e-8
    for solver in (DIRECT, DIRECT_WIDE):
        with pytest.raises(fl.FlError):
            _run(ctx, over, iters=1, solver=solver)
    with pytest.raises(fl.FlError):
        _run(ctx, loop, iters=1, solver=4)


@pytest.mark.parametrize("kw", [
    dict(n=2, covis=1, n_loops=0),
    dict(n=3, covis=2, n_loops=0),
    dict(n=30, covis=5, n_loops=3),
    dict(n=60, covis=4, n_loops=6),
    dict(n=200, covis=3, n_loops=8),
], ids=["n2", "n3", "widest", "windows", "loop200"])
def test_device_memory_window_is_identical_to_lds_window(ctx, kw):
    """Both band factorisations take the same floating-point steps in the
    same order: on every band the LDS window takes, the device-memory window
    gives the same poses, costs and decisions bit for bit."""
    d = synth.gen_pose_graph(seed=29, **kw)
    a = _run(ctx, d, iters=3, solver=DIRECT)
    b = _run(ctx, d, iters=3, solver=DIRECT_WIDE)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("kw,band", [
    (dict(n=150, laps=2, cross=1), 14),
    (dict(n=150, laps=3, cross=3), 22),
    (dict(n=150, laps=4, cross=1), 35),
    (dict(n=120, laps=6, cross=3), 42),
    (dict(n=70, covis=63, n_loops=0), 64),
], ids=["laps2", "laps3", "laps4", "laps6", "band64"])
def test_several_loops_direct_solve_matches_oracle(ctx, kw, band):
    """Graphs of several loops (a spiral trajectory of 2-6 laps whose
    keyframes are joined to the lap before; reordered bands of 14-42
    keyframes) and the widest band the direct solver takes (64 keyframes,
    448 scalars a row): the Levenberg-Marquardt iterations against the
    oracle's dense solves."""
    d = synth.gen_pose_graph(seed=29, **kw)
    assert _rcm_band(d) == band
    iters = 1 if band == 64 else 2
    S_ref, h, lams_ref, acc_ref = _oracle(d, iters=iters)
    S, cost, used, lams, acc = _run(ctx, d, iters=iters)
    assert all(u == 0 for u in used)
    assert np.array_equal(acc, acc_ref)
    assert np.array_equal(lams, lams_ref)
    assert _err(S, S_ref) < 1e-9, _err(S, S_ref)
    assert np.max(np.abs(cost - h) / h) < 1e-9


def test_several_loops_with_held_keyframes_and_an_unconnected_one(ctx):
    """Three laps with keyframes held along the trajectory (the band is taken
    over the free ones only) and one keyframe whose every edge was removed
    (held by the solve: a unit diagonal, no step), through the automatic
    choice of the device-memory window: the oracle's poses, and the held and
    unconnected keyframes unmoved."""
    d = synth.gen_pose_graph(n=150, seed=33, laps=3, cross=3)
    lone = 77
    keep = [k for k, (i, j) in enumerate(d["edges"]) if lone not in (i, j)]
    d = dict(d, edges=d["edges"][keep], M=d["M"][keep])
    fixed = np.zeros(150, bool)
    fixed[[0, 40, 90, 140]] = True
    assert _rcm_band(dict(d, fixed=fixed)) > 12
    # the oracle's dense solve needs the unconnected keyframe held explicitly
    S_ref, h, _, acc_ref = _oracle(d, fixed=fixed | (np.arange(150) == lone), iters=2)
    S, cost, used, _, acc = _run(ctx, d, fixed=fixed, iters=2)
    assert all(u == 0 for u in used)
    assert np.array_equal(acc, acc_ref)
    for n in (0, 40, 90, 140, lone):
        assert np.array_equal(S[n], d["S0"][n])
    assert _err(S, S_ref) < 1e-9, _err(S, S_ref)
    assert np.max(np.abs(cost - h) / h) < 1e-9


def test_several_loops_of_1000_keyframes_converge_deterministically(ctx):
    """1,000 keyframes on three laps (a reordered band of 24 keyframes):
    repeatable to the bit, accepted costs never rise, and the drift is
    removed."""
    d = synth.gen_pose_graph(n=1000, seed=606, laps=3, cross=3)
    assert _rcm_band(d) == 24
    S1, cost, used, _, acc = _run(ctx, d, iters=10)
    S2, cost2, _, _, _ = _run(ctx, d, iters=10)
    assert all(u == 0 for u in used)
    assert np.array_equal(S1, S2) and np.array_equal(cost, cost2)
    assert cost[-1] < 1e-3 * cost[0]
    assert all(b <= a for a, b in zip(cost, cost[1:]))
    assert _err(S1, d["S_true"]) < 0.1 * _err(d["S0"], d["S_true"])


@pytest.mark.parametrize("solver", [CG, DIRECT, DIRECT_WIDE])
def test_loop_of_1000_keyframes_converges_deterministically(ctx, solver):
    d = synth.gen_pose_graph(n=1000, seed=606)
    S1, cost, used, _, acc = _run(ctx, d, iters=10, solver=solver)
    S2, cost2, _, _, _ = _run(ctx, d, iters=10, solver=solver)
    assert np.array_equal(S1, S2) and np.array_equal(cost, cost2)
    assert cost[-1] < 1e-3 * cost[0]
    assert all(b <= a for a, b in zip(cost, cost[1:]))   # accepted costs never rise
    assert _err(S1, d["S_true"]) < 0.1 * _err(d["S0"], d["S_true"])


def test_loop_of_200_keyframes_direct_step_matches_oracle(ctx):
    """A loop of 200 keyframes (1,393 unknowns, the band window 28 times
    over): the exact step from the drifted start against the oracle's dense
    solve."""
    d = synth.gen_pose_graph(n=200, seed=606)
    S_ref, h, lams_ref, acc_ref = _oracle(d, iters=1)
    S, cost, used, lams, acc = _run(ctx, d, iters=1, solver=DIRECT)
    assert all(u == 0 for u in used)
    assert np.array_equal(acc, acc_ref)
    assert _err(S, S_ref) < 1e-9, _err(S, S_ref)
    assert np.max(np.abs(cost - h) / h) < 1e-9
