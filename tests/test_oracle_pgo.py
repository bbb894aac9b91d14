"""Pins of the float64 pose-graph oracle: exact recovery of a consistent
graph from a drifted start, invariance under a change of world frame, the
held node, and a decreasing cost on a noisy loop."""
import numpy as np
import pytest

import synth
from oracle import pgo, sim3


def _err(A, B):
    return max(np.linalg.norm(sim3.log(sim3.compose(a, sim3.inverse(b)))) for a, b in zip(A, B))


@pytest.fixture(scope="module")
def clean():
    return synth.gen_pose_graph(n=12, seed=11, covis=2, n_loops=2, noise_deg=0.0, noise_m=0.0, noise_scale=0.0)


def test_consistent_graph_is_recovered_exactly(clean):
    d = clean
    assert pgo.cost(d["S_true"], d["edges"], d["M"]) < 1e-24
    assert _err(d["S0"], d["S_true"]) > 1e-3
    h = []
    S = pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=6, history=h)
    assert _err(S, d["S_true"]) < 1e-9
    assert h[-1] < 1e-18 < h[0]
    assert np.array_equal(S[0], d["S0"][0])   # the held node does not move


def test_world_frame_change_moves_the_solution_with_it(clean):
    """F is unchanged when every pose is right-multiplied by one Sim3 G (the
    world frame changes; relative transforms do not), so the optimum of the
    moved start is the moved optimum."""
    d = synth.gen_pose_graph(n=10, seed=12, covis=2, n_loops=2)
    G = sim3.exp(np.array([0.2, -0.1, 0.3, 1.0, 2.0, -0.5, 0.1]))
    S = pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=3)
    S0g = np.stack([sim3.compose(s, G) for s in d["S0"]])
    Sg = pgo.optimize(S0g, d["edges"], d["M"], d["fixed"], iters=3)
    assert _err(Sg, [sim3.compose(s, G) for s in S]) < 1e-8


def test_noisy_loop_cost_decreases_and_drift_is_corrected():
    d = synth.gen_pose_graph(n=16, seed=13, covis=2, n_loops=3)
    h = []
    S = pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=3, history=h)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(h, h[1:])), h
    assert h[-1] < 0.05 * h[0]
    assert _err(S, d["S_true"]) < 0.5 * _err(d["S0"], d["S_true"])   # down to the edge noise


def test_damped_steps_reach_the_same_optimum():
    """Damping slows the weakly constrained directions but keeps the
    optimum; a huge damping barely moves."""
    d = synth.gen_pose_graph(n=10, seed=14, covis=2, n_loops=2)
    S_gn = pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=3)
    S_lm = pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=3, lam=1e-9)
    assert _err(S_lm, S_gn) < 1e-7
    steps = [_err(pgo.optimize(d["S0"], d["edges"], d["M"], d["fixed"], iters=1, lam=lam), d["S0"])
             for lam in (1e-2, 1.0, 1e2, 1e9)]
    assert all(b < a for a, b in zip(steps, steps[1:])) and steps[-1] < 1e-6, steps
