"""Sim3 reprojection residual, its gradient and Gauss-Newton, in float64
(test infrastructure only).

After matching, the loop Sim3 is refined from the matched pairs (the Sim(3)
optimisation between the two projection searches of Sec. IV-C).  For a
matched pair (map point X, observation uv, keyframe pose T_k = (R_k, t_k)):

    p = s R X + t             (the loop Sim3 S applied to the point)
    q = R_k p + t_k           (into keyframe k)
    r = pi(q) - uv,  pi(q) = (fx q0/q2 + cx, fy q1/q2 + cy)
    e = |r|,  rho(e) = e^2/2 if e <= delta else delta e - delta^2/2
    L = sum rho(e)            (pairs with q2 <= 0 contribute nothing)

The gradient is taken with respect to a left perturbation S <- exp(xi) S at
xi = 0, xi = (omega, upsilon, sigma).  With w = min(1, delta/e) the Huber
weight, g = sum w J^T r and the Gauss-Newton matrix H = sum w J^T J where
J = d r / d xi.  Here J is obtained by the chain rule written out term by
term; the tests pin it against central finite differences of L.
"""
from __future__ import annotations

import numpy as np

from . import sim3


def _kf_RT(kf_idx, kf_T, n):
    if kf_T is None:
        R = np.broadcast_to(np.eye(3), (n, 3, 3))
        t = np.zeros((n, 3))
    else:
        T = np.asarray(kf_T, np.float64)[np.asarray(kf_idx)]
        R = T[:, :9].reshape(-1, 3, 3)
        t = T[:, 9:12]
    return R, t


def project(S, xyz, kf_idx, kf_T, cam):
    X = np.asarray(xyz, np.float64)
    p = sim3.act(S, X)
    R, t = _kf_RT(kf_idx, kf_T, len(X))
    q = np.einsum("nij,nj->ni", R, p) + t
    fx, fy, cx, cy = (float(c) for c in cam[:4])
    with np.errstate(divide="ignore", invalid="ignore"):
        uv = np.stack([fx * q[:, 0] / q[:, 2] + cx, fy * q[:, 1] / q[:, 2] + cy], axis=1)
    return p, q, uv, R


def huber(e, delta):
    e = np.asarray(e, np.float64)
    rho = np.where(e <= delta, 0.5 * e * e, delta * e - 0.5 * delta * delta)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(e <= delta, 1.0, delta / e)
    return rho, w


def forward(S, xyz, uv, kf_idx, kf_T, cam, delta):
    """Per-pair residual r [n,2], Huber weight w [n] (0 for pairs behind the
    camera), and the loss L."""
    _, q, uvp, _ = project(S, xyz, kf_idx, kf_T, cam)
    valid = q[:, 2] > 0
    r = np.where(valid[:, None], uvp - np.asarray(uv, np.float64), 0.0)
    e = np.linalg.norm(r, axis=1)
    rho, w = huber(e, delta)
    rho = np.where(valid, rho, 0.0)
    w = np.where(valid, w, 0.0)
    return r, w, float(rho.sum())


def jacobian(S, xyz, kf_idx, kf_T, cam):
    """J [n, 2, 7] = d pi(q) / d q  .  R_k  .  [ -[p]x | I | p ]."""
    p, q, _, R = project(S, xyz, kf_idx, kf_T, cam)
    fx, fy = float(cam[0]), float(cam[1])
    n = len(p)
    dpi = np.zeros((n, 2, 3))
    with np.errstate(divide="ignore", invalid="ignore"):
        iz = 1.0 / q[:, 2]
        dpi[:, 0, 0] = fx * iz
        dpi[:, 0, 2] = -fx * q[:, 0] * iz * iz
        dpi[:, 1, 1] = fy * iz
        dpi[:, 1, 2] = -fy * q[:, 1] * iz * iz
    dp = np.zeros((n, 3, 7))
    # d(exp(xi) p)/d xi at 0: omega x p = -[p]x omega, upsilon, sigma p
    dp[:, 0, 1], dp[:, 0, 2] = p[:, 2], -p[:, 1]
    dp[:, 1, 0], dp[:, 1, 2] = -p[:, 2], p[:, 0]
    dp[:, 2, 0], dp[:, 2, 1] = p[:, 1], -p[:, 0]
    dp[:, 0, 3] = dp[:, 1, 4] = dp[:, 2, 5] = 1.0
    dp[:, :, 6] = p
    J = np.einsum("nab,nbc,ncd->nad", dpi, R, dp)
    J[q[:, 2] <= 0] = 0.0
    return J


def grad_hess(S, xyz, uv, kf_idx, kf_T, cam, delta):
    """g [7] = sum w J^T r, H [7,7] = sum w J^T J, and L."""
    r, w, L = forward(S, xyz, uv, kf_idx, kf_T, cam, delta)
    J = jacobian(S, xyz, kf_idx, kf_T, cam)
    g = np.einsum("n,nai,na->i", w, J, r)
    H = np.einsum("n,nai,naj->ij", w, J, J)
    return g, H, L


def loss_at(xi, S0, xyz, uv, kf_idx, kf_T, cam, delta):
    return forward(sim3.compose(sim3.exp(xi), S0), xyz, uv, kf_idx, kf_T, cam, delta)[2]


def fd_grad(S0, xyz, uv, kf_idx, kf_T, cam, delta, h=1e-4):
    """Central differences of L(exp(xi) S0) at xi = 0."""
    g = np.zeros(7)
    for i in range(7):
        e = np.zeros(7)
        e[i] = h
        g[i] = (loss_at(e, S0, xyz, uv, kf_idx, kf_T, cam, delta)
                - loss_at(-e, S0, xyz, uv, kf_idx, kf_T, cam, delta)) / (2 * h)
    return g


def H_upper(H) -> np.ndarray:
    """The 28 entries of the upper triangle of a symmetric 7x7, row by row."""
    return np.asarray(H)[np.triu_indices(7)]


def gauss_newton(S0, xyz, uv, kf_idx, kf_T, cam, delta, iters=10):
    """Undamped IRLS Gauss-Newton: solve H dxi = -g, S <- exp(dxi) S."""
    S = np.asarray(S0, np.float64).copy()
    for _ in range(iters):
        g, H, _ = grad_hess(S, xyz, uv, kf_idx, kf_T, cam, delta)
        dxi = np.linalg.solve(H, -g)
        S = sim3.compose(sim3.exp(dxi), S)
    return S


def _marquardt_solve(g, H, lam):
    """Solve (H + lam diag H) dxi = -g."""
    return np.linalg.solve(H + lam * np.diag(np.diag(H)), -g)


LM_CONVERGED = 1e-6   # relative loss change that ends a Levenberg-Marquardt round


def refine_robust(S0, xyz, uv, kf_idx, kf_T, cam, delta, iters=5, rounds=2, outlier_px=np.inf, lm_lambda=0.0,
                  history=None):
    """Robust refinement of the loop Sim3 in rounds (the Sim(3) optimisation
    around the projection searches of Sec. IV-C; the paper gives no
    algorithm, so the steps below are readings).

    Round 0 uses every pair.  Each later round uses the pairs that lie in
    front of their keyframe with reprojection error e <= outlier_px at the
    Sim3 the previous round ended with (the set is chosen afresh each round).
    A round is `iters` evaluations of g, H and the Huber loss L on its pairs:
      * lm_lambda == 0: undamped Gauss-Newton, S <- exp(dxi) S after every
        evaluation, dxi = -H^-1 g;
      * lm_lambda > 0: Levenberg-Marquardt with Marquardt's scaling.  The
        first evaluation of a round is at the round's starting Sim3; each
        later one is at the candidate exp(dxi) S_acc, dxi solving
        (H + lambda diag H) dxi = -g with g, H of S_acc.  With
        rho = (L(S_acc) - L_c) / L(S_acc): rho > 1e-6 accepts the candidate
        (S_acc moves there, lambda / 10); |rho| <= 1e-6 ends the round
        (converged: the loss no longer changes beyond what its rounding can
        decide); rho < -1e-6 rejects it (lambda * 10).  lambda is kept in
        [1e-12, 1e16] and reset to lm_lambda at each round.  The round ends
        at S_acc; a candidate solved after the last evaluation is not taken.
    Returns (S, n_used): n_used counts the round's pairs in front of their
    keyframe at the last evaluation that produced the result (GN: the last
    evaluation; LM: the evaluation of the final S_acc).
    `history`, if a list, receives (round, L, status) per evaluation, status
    "step" (GN), "start" (LM, a round's first), "accept", "reject" or
    "converged".
    """
    S = np.asarray(S0, np.float64).copy()
    X = np.asarray(xyz, np.float64)
    U = np.asarray(uv, np.float64)
    kf_idx = None if kf_idx is None else np.asarray(kf_idx)
    n_used = 0
    for rnd in range(rounds):
        if rnd == 0:
            sel = np.ones(len(X), bool)
        else:
            _, q, uvp, _ = project(S, X, kf_idx, kf_T, cam)
            with np.errstate(invalid="ignore"):
                e = np.linalg.norm(uvp - U, axis=1)
                sel = (q[:, 2] > 0) & (e <= outlier_px)
        Xs, Us = X[sel], U[sel]
        ks = None if kf_idx is None else kf_idx[sel]

        def evaluate(S_at):
            g, H, L = grad_hess(S_at, Xs, Us, ks, kf_T, cam, delta)
            _, q, _, _ = project(S_at, Xs, ks, kf_T, cam)
            return g, H, L, int((q[:, 2] > 0).sum())

        if lm_lambda <= 0.0:
            for _ in range(iters):
                g, H, L, n_used = evaluate(S)
                if history is not None:
                    history.append((rnd, L, "step"))
                S = sim3.compose(sim3.exp(np.linalg.solve(H, -g)), S)
        else:
            lam = float(lm_lambda)
            g, H, L, n_used = evaluate(S)
            if history is not None:
                history.append((rnd, L, "start"))
            for _ in range(1, iters):
                S_c = sim3.compose(sim3.exp(_marquardt_solve(g, H, lam)), S)
                g_c, H_c, L_c, n_c = evaluate(S_c)
                rho = (L - L_c) / L if L > 0 else 0.0
                ok = rho > LM_CONVERGED
                if history is not None:
                    history.append((rnd, L_c, "accept" if ok else "reject" if rho < -LM_CONVERGED else "converged"))
                if ok:
                    S, g, H, L, n_used = S_c, g_c, H_c, L_c, n_c
                    lam = max(lam / 10.0, 1e-12)
                elif rho >= -LM_CONVERGED:
                    break
                else:
                    lam = min(lam * 10.0, 1e16)
    return S, n_used


# ---------------------------------------------------------------------------
# The other direction of a loop match: a point X of the current side, mapped
# into the loop side by S^-1 and observed in a keyframe k there,
#     r = pi(T_k S^-1 X) - uv.
# Its gradient is still taken with respect to the left perturbation of S:
# S^-1 <- S^-1 exp(-xi), so d(S^-1 X)/dxi = -(1/s) R^T [ -[X]x | I | X ].


def forward_inv(S, xyz, uv, kf_idx, kf_T, cam, delta):
    """r, w, L of the other direction (forward() at S^-1)."""
    return forward(sim3.inverse(S), xyz, uv, kf_idx, kf_T, cam, delta)


def jacobian_inv(S, xyz, kf_idx, kf_T, cam):
    """J [n, 2, 7] = d pi(q)/d q . R_k . (-(1/s) R^T) . [ -[X]x | I | X ]."""
    X = np.asarray(xyz, np.float64)
    _, q, _, Rk = project(sim3.inverse(S), X, kf_idx, kf_T, cam)
    fx, fy = float(cam[0]), float(cam[1])
    n = len(X)
    dpi = np.zeros((n, 2, 3))
    with np.errstate(divide="ignore", invalid="ignore"):
        iz = 1.0 / q[:, 2]
        dpi[:, 0, 0] = fx * iz
        dpi[:, 0, 2] = -fx * q[:, 0] * iz * iz
        dpi[:, 1, 1] = fy * iz
        dpi[:, 1, 2] = -fy * q[:, 1] * iz * iz
    R, s = np.asarray(S[:9], np.float64).reshape(3, 3), float(S[12])
    G = np.zeros((n, 3, 7))
    G[:, 0, 1], G[:, 0, 2] = X[:, 2], -X[:, 1]
    G[:, 1, 0], G[:, 1, 2] = -X[:, 2], X[:, 0]
    G[:, 2, 0], G[:, 2, 1] = X[:, 1], -X[:, 0]
    G[:, 0, 3] = G[:, 1, 4] = G[:, 2, 5] = 1.0
    G[:, :, 6] = X
    J = np.einsum("nab,nbc,cd,nde->nae", dpi, Rk, -R.T / s, G)
    J[q[:, 2] <= 0] = 0.0
    return J


def grad_hess_inv(S, xyz, uv, kf_idx, kf_T, cam, delta):
    r, w, L = forward_inv(S, xyz, uv, kf_idx, kf_T, cam, delta)
    J = jacobian_inv(S, xyz, kf_idx, kf_T, cam)
    return np.einsum("n,nai,na->i", w, J, r), np.einsum("n,nai,naj->ij", w, J, J), L


def gauss_newton_bidir(S0, fwd, bwd, cam, delta, iters=10, cam_bwd=None):
    """Undamped IRLS Gauss-Newton on both directions: g and H are the sums of
    the two sets' (fwd = (xyz, uv, kf_idx, kf_T) observed through S, bwd the
    same observed through S^-1; cam_bwd: the bwd set's camera, default
    cam)."""
    S = np.asarray(S0, np.float64).copy()
    cb = cam if cam_bwd is None else cam_bwd
    for _ in range(iters):
        g1, H1, _ = grad_hess(S, *fwd, cam, delta)
        g2, H2, _ = grad_hess_inv(S, *bwd, cb, delta)
        S = sim3.compose(sim3.exp(np.linalg.solve(H1 + H2, -(g1 + g2))), S)
    return S
