"""Sim3 pose-graph optimisation of the essential graph, in float64 (test
infrastructure only).

Loop correction propagates the loop's Sim3 to every keyframe by optimising
the essential graph (Sec. III-B loop correction, Sec. IV-F graph
optimisation): keyframe poses S_i (world -> camera Sim3s) joined by edges
that measure their relative transform, M_ij ~ S_j S_i^-1.  The paper
optimises it by Levenberg-Marquardt with Jacobians that are exact
derivatives (automatic differentiation instead of numerical
differentiation) and gives no formulas; the reading taken here:

    e_ij = log(M_ij^-1 S_j S_i^-1)          (7-vector, zero for a consistent edge)
    F    = sum over edges of e_ij^T e_ij    (unit information)

Nodes move by left perturbations S_i <- exp(d_i) S_i.  With E = M^-1 S_j S_i^-1
and e = log E, a perturbation of S_j gives M^-1 exp(d) S_j S_i^-1 =
exp(Ad(M^-1) d) E and one of S_i gives E exp(-d) = exp(-Ad(E) d) E, and to
first order log(exp(x) E) = e + J_l(e)^-1 x, so the exact Jacobians are

    J_j = J_l(e)^-1 Ad(M^-1),     J_i = -J_l(e)^-1 Ad(E),

with Ad the 7x7 adjoint of a Sim3 and J_l(x) = sum_k ad(x)^k / (k+1)! the
left Jacobian (evaluated here as a block of the matrix exponential of
[[ad(x), I], [0, 0]]).  Each Levenberg-Marquardt iteration solves
(H + lambda diag H) d = -g over the free nodes (Marquardt's scaling),
evaluates F at the candidate exp(d_i) S_i and accepts it if F decreases
(lambda / 10) or rejects it (lambda x 10, the linearisation is kept).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from . import sim3

LAMBDA_MIN, LAMBDA_MAX = 1e-12, 1e12


def edge_error(S_i, S_j, M) -> np.ndarray:
    return sim3.log(sim3.compose(sim3.inverse(M), sim3.compose(S_j, sim3.inverse(S_i))))


def adjoint(S) -> np.ndarray:
    """Ad(S) with exp(Ad(S) x) = S exp(x) S^-1, tangent order (omega, upsilon, sigma):
    S (x)^ S^-1 for S = [[sR, t], [0, 1]] maps omega to R omega, sigma to
    sigma and upsilon to s R upsilon + [t]x R omega - sigma t."""
    S = np.asarray(S, np.float64)
    R, t, s = S[:9].reshape(3, 3), S[9:12], S[12]
    A = np.zeros((7, 7))
    A[:3, :3] = R
    A[3:6, :3] = sim3.hat(t) @ R
    A[3:6, 3:6] = s * R
    A[3:6, 6] = -t
    A[6, 6] = 1.0
    return A


def ad(x) -> np.ndarray:
    """ad(x) y = [x^, y^] for the 4x4 generators (tangent order omega, upsilon, sigma)."""
    x = np.asarray(x, np.float64)
    A = np.zeros((7, 7))
    A[:3, :3] = sim3.hat(x[:3])
    A[3:6, :3] = sim3.hat(x[3:6])
    A[3:6, 3:6] = sim3.hat(x[:3]) + x[6] * np.eye(3)
    A[3:6, 6] = -x[3:6]
    return A


def left_jacobian(x) -> np.ndarray:
    """J_l(x) = sum_k ad(x)^k / (k+1)!: the top-right block of
    expm([[ad(x), I], [0, 0]])."""
    B = np.zeros((14, 14))
    B[:7, :7] = ad(x)
    B[:7, 7:] = np.eye(7)
    return expm(B)[:7, 7:]


def edge_jacobians(S_i, S_j, M):
    """(J_i, J_j), each 7x7: d e_ij / d d_i and d e_ij / d d_j, exact."""
    E = sim3.compose(sim3.inverse(M), sim3.compose(S_j, sim3.inverse(S_i)))
    Jinv = np.linalg.inv(left_jacobian(sim3.log(E)))
    return -Jinv @ adjoint(E), Jinv @ adjoint(sim3.inverse(M))


def cost(S, edges, M) -> float:
    return float(sum(np.dot(e, e) for e in (edge_error(S[i], S[j], M[k]) for k, (i, j) in enumerate(edges))))


def normal_equations(S, edges, M, col, n_free):
    """(g, H, F) at S over the free nodes (col[i] = block column, -1 held)."""
    H = np.zeros((7 * n_free, 7 * n_free))
    g = np.zeros(7 * n_free)
    F = 0.0
    for k, (i, j) in enumerate(edges):
        e = edge_error(S[i], S[j], M[k])
        F += float(e @ e)
        Ji, Jj = edge_jacobians(S[i], S[j], M[k])
        for a, Ja in ((i, Ji), (j, Jj)):
            if col[a] < 0:
                continue
            ra = slice(7 * col[a], 7 * col[a] + 7)
            g[ra] += Ja.T @ e
            for b, Jb in ((i, Ji), (j, Jj)):
                if col[b] >= 0:
                    H[ra, 7 * col[b]:7 * col[b] + 7] += Ja.T @ Jb
    return g, H, F


def optimize(S0, edges, M, fixed, iters=10, lam=1e-4, history=None, lambdas=None, accepted=None, candidates=None):
    """`iters` Levenberg-Marquardt iterations from damping `lam` over the
    free nodes (fixed[i] true holds node i).  lam = 0 takes plain
    Gauss-Newton steps, every one accepted.  Returns the poses.  Optional
    lists receive: `history` F of the accepted poses before every iteration
    and at the end, `lambdas` the damping each iteration solved with,
    `accepted` whether each iteration's candidate was taken, `candidates`
    F of each iteration's candidate."""
    S = np.array(S0, np.float64, copy=True)
    n = len(S)
    free = np.nonzero(~np.asarray(fixed, bool))[0]
    col = -np.ones(n, np.int64)
    col[free] = np.arange(len(free))
    lin = None
    F = None   # F of the accepted poses: evaluated once, at the start or as the accepted candidate
    for _ in range(iters):
        if lin is None:
            lin = normal_equations(S, edges, M, col, len(free))
            if F is None:
                F = lin[2]
        g, H, _ = lin
        if history is not None:
            history.append(F)
        if lambdas is not None:
            lambdas.append(lam)
        d = np.linalg.solve(H + lam * np.diag(np.diag(H)), -g)
        C = S.copy()
        for a in free:
            C[a] = sim3.compose(sim3.exp(d[7 * col[a]:7 * col[a] + 7]), S[a])
        Fc = cost(C, edges, M)
        if candidates is not None:
            candidates.append(Fc)
        take = lam == 0.0 or Fc < F
        if accepted is not None:
            accepted.append(bool(take))
        if take:
            S = C
            F = Fc
            lin = None
            lam = max(lam / 10.0, LAMBDA_MIN) if lam > 0.0 else 0.0
        else:
            lam = min(lam * 10.0, LAMBDA_MAX)
    if history is not None:
        history.append(cost(S, edges, M) if F is None else F)
    return S
