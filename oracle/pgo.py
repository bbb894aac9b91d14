"""Sim3 pose-graph optimisation of the essential graph, in float64 (test
infrastructure only).

Loop correction propagates the loop's Sim3 to every keyframe by optimising
the essential graph (Sec. III-B loop correction, Sec. IV-F graph
optimisation): keyframe poses S_i (world -> camera Sim3s) joined by edges
that measure their relative transform, M_ij ~ S_j S_i^-1.  The paper solves
it with Levenberg-Marquardt and Jacobians from automatic differentiation and
gives no formulas; the reading taken here:

    e_ij = log(M_ij^-1 S_j S_i^-1)          (7-vector, zero for a consistent edge)
    F    = sum over edges of e_ij^T e_ij    (unit information)

Nodes move by left perturbations S_i <- exp(d_i) S_i; the Jacobians of e_ij
with respect to d_i and d_j are central differences with step h; the normal
equations (H + lambda diag H) d = -g over the free nodes are solved directly.
"""
from __future__ import annotations

import numpy as np

from . import sim3


def edge_error(S_i, S_j, M) -> np.ndarray:
    return sim3.log(sim3.compose(sim3.inverse(M), sim3.compose(S_j, sim3.inverse(S_i))))


def edge_jacobians(S_i, S_j, M, h=1e-5):
    """(J_i, J_j), each 7x7: d e_ij / d d_i and d e_ij / d d_j by central
    differences of the left perturbations."""
    Ji, Jj = np.zeros((7, 7)), np.zeros((7, 7))
    for k in range(7):
        dk = np.zeros(7)
        dk[k] = h
        Ji[:, k] = (edge_error(sim3.compose(sim3.exp(dk), S_i), S_j, M)
                    - edge_error(sim3.compose(sim3.exp(-dk), S_i), S_j, M)) / (2 * h)
        Jj[:, k] = (edge_error(S_i, sim3.compose(sim3.exp(dk), S_j), M)
                    - edge_error(S_i, sim3.compose(sim3.exp(-dk), S_j), M)) / (2 * h)
    return Ji, Jj


def cost(S, edges, M) -> float:
    return float(sum(np.dot(e, e) for e in (edge_error(S[i], S[j], M[k]) for k, (i, j) in enumerate(edges))))


def optimize(S0, edges, M, fixed, iters=10, lam=0.0, h=1e-5, history=None):
    """`iters` Gauss-Newton steps (lam = 0) or steps damped by lam diag H
    (fixed lam) over the free nodes; fixed[i] true holds node i.  Returns
    the poses; `history`, if a list, receives F before every step and at
    the end."""
    S = np.array(S0, np.float64, copy=True)
    n = len(S)
    free = np.nonzero(~np.asarray(fixed, bool))[0]
    col = -np.ones(n, np.int64)
    col[free] = np.arange(len(free))
    for _ in range(iters):
        H = np.zeros((7 * len(free), 7 * len(free)))
        g = np.zeros(7 * len(free))
        F = 0.0
        for k, (i, j) in enumerate(edges):
            e = edge_error(S[i], S[j], M[k])
            F += float(e @ e)
            Ji, Jj = edge_jacobians(S[i], S[j], M[k], h)
            for a, Ja in ((i, Ji), (j, Jj)):
                if col[a] < 0:
                    continue
                ra = slice(7 * col[a], 7 * col[a] + 7)
                g[ra] += Ja.T @ e
                for b, Jb in ((i, Ji), (j, Jj)):
                    if col[b] >= 0:
                        H[ra, 7 * col[b]:7 * col[b] + 7] += Ja.T @ Jb
        if history is not None:
            history.append(F)
        d = np.linalg.solve(H + lam * np.diag(np.diag(H)), -g)
        for a in free:
            S[a] = sim3.compose(sim3.exp(d[7 * col[a]:7 * col[a] + 7]), S[a])
    if history is not None:
        history.append(cost(S, edges, M))
    return S
