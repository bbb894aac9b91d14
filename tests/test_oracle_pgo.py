"""Pins of the float64 pose-graph oracle: exact edge Jacobians against
central differences of the edge error, the adjoint and left-Jacobian
identities, exact recovery of a consistent graph from a drifted start,
invariance under a change of world frame, Levenberg-Marquardt reducing to
Gauss-Newton as the damping vanishes, a monotone accepted cost, and the
several-loop workload's structure and exact recovery."""
import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import pgo, sim3


def _err(A, B):
    return max(np.linalg.norm(sim3.log(sim3.compose(a, sim3.inverse(b)))) for a, b in zip(A, B))


@pytest.fixture(scope="module")
def clean():
    return synth.gen_pose_graph(n=12, seed=11, covis=2, n_loops=2, noise_deg=0.0, noise_m=0.0, noise_scale=0.0)


def test_adjoint_moves_a_perturbation_through_a_pose():
    # exp(Ad(S) x) = S exp(x) S^-1, by the matrix exponential of the generators
    rng = np.random.default_rng(1)
    for _ in range(5):
        S = sim3.exp(rng.normal(size=7) * 0.7)
        x = rng.normal(size=7) * 0.3
        lhs = expm(sim3.generator(pgo.adjoint(S) @ x))
        rhs = sim3.to_matrix(S) @ expm(sim3.generator(x)) @ np.linalg.inv(sim3.to_matrix(S))
        assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_left_jacobian_by_central_differences():
    # log(exp(x + h d) exp(x)^-1) / h -> J_l(x) d
    rng = np.random.default_rng(2)
    for scale in (1e-8, 0.1, 0.8):
        x = rng.normal(size=7) * scale
        h = 1e-6
        J = np.zeros((7, 7))
        for c in range(7):
            d = np.zeros(7)
            d[c] = h
            J[:, c] = (sim3.log(sim3.compose(sim3.exp(x + d), sim3.inverse(sim3.exp(x))))
                       - sim3.log(sim3.compose(sim3.exp(x - d), sim3.inverse(sim3.exp(x))))) / (2 * h)
        assert np.max(np.abs(J - pgo.left_jacobian(x))) < 1e-8, scale
    assert np.array_equal(pgo.left_jacobian(np.zeros(7)), np.eye(7))


def test_edge_jacobians_are_exact():
    # central differences of e_ij under left perturbations of S_i and S_j
    # (h = 1e-6: truncation ~1e-12, rounding ~1e-10) agree to 1e-7 relative,
    # on edges far from consistent (large errors exercise J_l(e)^-1)
    rng = np.random.default_rng(3)
    for trial in range(6):
        Si = sim3.exp(rng.normal(size=7) * 0.8)
        Sj = sim3.exp(rng.normal(size=7) * 0.8)
        M = sim3.exp(rng.normal(size=7) * 0.8)
        Ji, Jj = pgo.edge_jacobians(Si, Sj, M)
        h = 1e-6
        for side, J in ((0, Ji), (1, Jj)):
            F = np.zeros((7, 7))
            for c in range(7):
                d = np.zeros(7)
                d[c] = h
                if side == 0:
                    ep = pgo.edge_error(sim3.compose(sim3.exp(d), Si), Sj, M)
                    em = pgo.edge_error(sim3.compose(sim3.exp(-d), Si), Sj, M)
                else:
                    ep = pgo.edge_error(Si, sim3.compose(sim3.exp(d), Sj), M)
                    em = pgo.edge_error(Si, sim3.compose(sim3.exp(-d), Sj), M)
                F[:, c] = (ep - em) / (2 * h)
            assert np.max(np.abs(F - J)) / np.max(np.abs(J)) < 1e-7, (trial, side)
    # a consistent edge: J_j = Ad(M^-1), J_i = -Ad(M^-1 S_j S_i^-1) = -Ad(I) = -I
    d = synth.gen_pose_graph(n=4, seed=5, covis=1, n_loops=0, noise_deg=0.0, noise_m=0.0, noise_scale=0.0)
    i, j = d["edges"][0]
    Ji, Jj = pgo.edge_jacobians(d["S_true"][i], d["S_true"][j], d["M"][0])
    assert np.max(np.abs(Ji + np.eye(7))) < 1e-12
    assert np.max(np.abs(Jj - pgo.adjoint(sim3.inverse(d["M"][0])))) < 1e-12


def test_consistent_graph_is_recovered_exactly(clean):
    d = clean
    assert pgo.cost(d["S_true"], d["edges"], d["M"]) < 1e-24
    assert _err(d["S0"], d["S_true"]) > 1e-3
    h = []
    S = pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=6, history=h)
    assert _err(S, d["S_true"]) < 1e-9
    assert h[-1] < 1e-18 < h[0]
    assert np.array_equal(S[0], d["S0"][0])   # the held node does not move


def test_world_frame_change_moves_the_solution_with_it():
    """F is unchanged when every pose is right-multiplied by one Sim3 G (the
    world frame changes; relative transforms do not), so the optimum of the
    moved start is the moved optimum."""
    d = synth.gen_pose_graph(n=10, seed=12, covis=2, n_loops=2)
    G = sim3.exp(np.array([0.2, -0.1, 0.3, 1.0, 2.0, -0.5, 0.1]))
    S = pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=3)
    S0g = np.stack([sim3.compose(s, G) for s in d["S0"]])
    Sg = pgo.optimize(S0g, d["edges"], d["M"], d["fixed"], iters=3)
    assert _err(Sg, [sim3.compose(s, G) for s in S]) < 1e-8


def test_levenberg_marquardt_cost_is_monotone_and_drift_is_corrected():
    d = synth.gen_pose_graph(n=16, seed=13, covis=2, n_loops=3)
    h, lams, acc = [], [], []
    S = pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=6, history=h, lambdas=lams, accepted=acc)
    assert all(b <= a for a, b in zip(h, h[1:])), h
    assert h[-1] < 0.05 * h[0]
    assert _err(S, d["S_true"]) < 0.5 * _err(d["S0"], d["S_true"])   # down to the edge noise
    # the damping follows the accept / reject rule
    for k in range(len(acc) - 1):
        assert lams[k + 1] == pytest.approx(lams[k] / 10 if acc[k] else lams[k] * 10)


def test_levenberg_marquardt_tends_to_gauss_newton():
    """As the damping vanishes every step is the Gauss-Newton step (all
    accepted on this graph), so both runs end at the same poses."""
    d = synth.gen_pose_graph(n=10, seed=14, covis=2, n_loops=2)
    S_gn = pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=3, lam=0.0)
    acc = []
    S_lm = pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=3, lam=1e-12, accepted=acc)
    assert all(acc)
    assert _err(S_lm, S_gn) < 1e-9


def test_large_damping_barely_moves_and_rejects_raise_it():
    """A huge damping takes a tiny step; a step that increases F is refused,
    the poses are kept and the damping grows tenfold."""
    d = synth.gen_pose_graph(n=10, seed=14, covis=2, n_loops=2)
    steps = [_err(pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=1, lam=lam), d["S0"])
             for lam in (1e-2, 1.0, 1e2, 1e9)]
    assert all(b < a for a, b in zip(steps, steps[1:])) and steps[-1] < 1e-6, steps
    # a start from which the undamped steps overshoot: refused, poses kept,
    # damping up tenfold, with a margin far above rounding
    from cases import overshoot_graph
    d = overshoot_graph()
    h, acc, lams, cand = [], [], [], []
    pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=8, lam=1e-6, history=h, accepted=acc,
                 lambdas=lams, candidates=cand)
    assert acc == [True, False, False, False, False, True, True, True], acc
    for k in range(8):
        assert abs(cand[k] - h[k]) > 0.2 * h[k]          # every decision is far from a tie
        assert (cand[k] < h[k]) == acc[k]
        assert h[k + 1] == (cand[k] if acc[k] else h[k])
        if k < 7:
            assert lams[k + 1] == pytest.approx(lams[k] / 10 if acc[k] else 10 * lams[k])


def test_several_laps_graph_structure_and_exact_recovery():
    """The several-loop workload: every keyframe of a later lap is joined to
    keyframes of the lap before that sit at about the same place (the same
    angle on the spiral, radii 0.25 m apart), the consistent graph is
    recovered exactly from its drifted start, and one lap gives the
    single-loop graph edge for edge."""
    n, laps, cross = 60, 3, 3
    d = synth.gen_pose_graph(n=n, seed=14, covis=2, n_loops=2, laps=laps, cross=cross, noise_deg=0.0,
                             noise_m=0.0, noise_scale=0.0)
    period = n / laps
    e = {(int(i), int(j)) for i, j in d["edges"]}
    cross_edges = [(i, j) for i, j in e if j - i > 2 and not (i >= n - 2 and j < 2)]
    assert cross_edges
    # camera centres of the world -> camera poses
    c = np.stack([-np.asarray(S[:9]).reshape(3, 3).T @ S[9:12] for S in d["S_true"]])
    step = max(np.linalg.norm(c[k + 1] - c[k]) for k in range(n - 1))
    for i, j in cross_edges:
        assert abs((j - i) - period) <= cross // 2 + 1
        # about the same place: within the offset's keyframe spacings plus the radius step of a lap
        assert np.linalg.norm(c[i] - c[j]) <= (cross // 2 + 1) * step + 0.25 + 1e-9
    assert all(sum(1 for i, j in e if j == k and j - i > 2) == cross for k in range(int(np.ceil(period)) + 2, n - 2))
    h = []
    S = pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=6, history=h)
    assert _err(S, d["S_true"]) < 1e-9 and h[-1] < 1e-18
    one = synth.gen_pose_graph(n=n, seed=14, covis=2, n_loops=2)
    same = synth.gen_pose_graph(n=n, seed=14, covis=2, n_loops=2, laps=1, cross=cross)
    assert np.array_equal(one["edges"], same["edges"]) and np.array_equal(one["M"], same["M"])
