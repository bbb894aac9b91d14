"""Pins of the float64 Sim3 reprojection residual oracle: analytic gradient
vs central finite differences, the all-inlier least-squares case, the
zero-noise optimum and Gauss-Newton recovery of the planted Sim3."""
import numpy as np
import pytest

import synth
from oracle import residual, sim3


@pytest.fixture(scope="module")
def c4():
    return synth.gen_c4(n=20000)


def _S0(d):
    return sim3.compose(sim3.exp(d["xi0"]), d["S_true"])


def test_gradient_matches_central_differences(c4):
    S0 = _S0(c4)
    g, H, L = residual.grad_hess(S0, c4["xyz"], c4["uv"], None, None, c4["cam"], c4["huber_delta"])
    # h = 1e-4: O(h^2) truncation plus O(h) from the pairs near the Huber kink
    fd = residual.fd_grad(S0, c4["xyz"], c4["uv"], None, None, c4["cam"], c4["huber_delta"], h=1e-4)
    assert np.max(np.abs(g - fd)) / np.max(np.abs(fd)) < 1e-4
    # and the difference keeps shrinking with h
    fd6 = residual.fd_grad(S0, c4["xyz"], c4["uv"], None, None, c4["cam"], c4["huber_delta"], h=1e-6)
    assert np.max(np.abs(g - fd6)) / np.max(np.abs(fd6)) < 1e-7
    assert L > 0
    # one camera at the origin of the Sim3's target frame cannot see scale:
    # the sigma component of the gradient vanishes and H is singular there
    assert abs(g[6]) < 1e-9 * np.max(np.abs(g))
    assert np.min(np.linalg.eigvalsh(H)) < 1e-12 * np.max(np.linalg.eigvalsh(H))


def test_gradient_with_keyframe_poses():
    # several keyframes with their own SE3 pose
    d = synth.gen_c4(n=3000, seed=9)
    rng = np.random.default_rng(4)
    T = []
    for _ in range(4):
        S = sim3.exp(np.concatenate([rng.normal(size=3) * 0.05, rng.normal(size=3) * 0.1, [0.0]]))
        T.append(S[:12])
    T = np.array(T)
    kf = rng.integers(0, 4, len(d["xyz"]))
    S0 = _S0(d)
    g, _, _ = residual.grad_hess(S0, d["xyz"], d["uv"], kf, T, d["cam"], 2.45)
    fd = residual.fd_grad(S0, d["xyz"], d["uv"], kf, T, d["cam"], 2.45, h=1e-6)
    assert np.max(np.abs(g - fd)) / np.max(np.abs(fd)) < 1e-7


def test_all_inlier_is_least_squares(c4):
    # delta -> infinity: every weight is 1 and L = 1/2 sum |r|^2
    S0 = _S0(c4)
    r, w, L = residual.forward(S0, c4["xyz"], c4["uv"], None, None, c4["cam"], 1e9)
    assert np.all(w == 1.0)
    assert np.isclose(L, 0.5 * np.sum(r * r), rtol=1e-12)
    g, H, _ = residual.grad_hess(S0, c4["xyz"], c4["uv"], None, None, c4["cam"], 1e9)
    fd = residual.fd_grad(S0, c4["xyz"], c4["uv"], None, None, c4["cam"], 1e9, h=1e-6)
    assert np.max(np.abs(g - fd)) / np.max(np.abs(fd)) < 1e-7
    # H is symmetric positive semi-definite
    assert np.allclose(H, H.T) and np.all(np.linalg.eigvalsh(H) > -1e-9 * np.max(np.abs(H)))


def test_zero_noise_optimum():
    d = synth.gen_c4(n=5000, seed=12, outlier_frac=0.0, pix_sigma=0.0)
    S = d["S_true"]
    # observations computed from the float32 points are exact projections
    r, w, L = residual.forward(S, d["xyz"], d["uv"], None, None, d["cam"], 2.45)
    assert L < 1e-6
    g, H, _ = residual.grad_hess(S, d["xyz"], d["uv"], None, None, d["cam"], 2.45)
    assert np.max(np.abs(g)) < 1e-2 * np.sqrt(np.max(np.diag(H))) * 1e-3


def _multi_view(n, seed):
    """C4-style observations seen from 6 keyframes placed around the scene,
    so that the Sim3 scale is observable."""
    rng = np.random.default_rng(seed)
    d = synth.gen_c4(n=n, seed=seed, pix_sigma=0.0, outlier_frac=0.0)
    T = np.array([sim3.exp(np.concatenate([rng.normal(size=3) * 0.1, rng.normal(size=3) * 0.5, [0.0]]))[:12]
                  for _ in range(6)])
    kf = rng.integers(0, 6, n)
    S = d["S_true"]
    _, q, uv, _ = residual.project(S, d["xyz"], kf, T, d["cam"])
    uv = uv + rng.normal(0, 1.0, uv.shape)
    out = rng.random(n) < 0.1
    th = rng.uniform(0, 2 * np.pi, n)
    uv[out] += 20 * np.stack([np.cos(th[out]), np.sin(th[out])], 1)
    keep = q[:, 2] > 0.1
    return d, d["xyz"][keep], uv[keep], kf[keep], T


def test_gauss_newton_recovers_planted_sim3():
    d, xyz, uv, kf, T = _multi_view(20000, 31)
    S0 = _S0(d)
    S = residual.gauss_newton(S0, xyz, uv, kf, T, d["cam"], 2.45, iters=10)
    err = np.linalg.norm(sim3.log(sim3.compose(S, sim3.inverse(d["S_true"]))))
    err0 = np.linalg.norm(sim3.log(sim3.compose(S0, sim3.inverse(d["S_true"]))))
    assert err < 1e-3 < err0


def test_behind_camera_pairs_contribute_nothing(c4):
    xyz = c4["xyz"][:100].copy()
    xyz[:10, 2] = -50.0
    S0 = _S0(c4)
    r, w, L = residual.forward(S0, xyz, c4["uv"][:100], None, None, c4["cam"], 2.45)
    _, q, _, _ = residual.project(S0, xyz, None, None, c4["cam"])
    behind = q[:, 2] <= 0
    assert behind.sum() >= 10
    assert np.all(w[behind] == 0) and np.all(r[behind] == 0)


def _views_with_outliers(n, seed, sigma):
    """Observations of C4's points from 6 keyframes, pixel noise `sigma`, and
    10% of them moved 20 px in a random direction (the planted outliers)."""
    rng = np.random.default_rng(seed)
    d = synth.gen_c4(n=n, seed=seed, pix_sigma=0.0, outlier_frac=0.0)
    T = np.array([sim3.exp(np.concatenate([rng.normal(size=3) * 0.1, rng.normal(size=3) * 0.5, [0.0]]))[:12]
                  for _ in range(6)])
    kf = rng.integers(0, 6, n)
    _, q, uv, _ = residual.project(d["S_true"], d["xyz"], kf, T, d["cam"])
    uv = uv + rng.normal(0, sigma, uv.shape) if sigma > 0 else uv
    out = rng.random(n) < 0.1
    th = rng.uniform(0, 2 * np.pi, n)
    uv[out] += 20 * np.stack([np.cos(th[out]), np.sin(th[out])], 1)
    keep = q[:, 2] > 0.1
    return d, d["xyz"][keep], uv[keep], kf[keep], T, out[keep]


def _err(S, S_ref):
    return np.linalg.norm(sim3.log(sim3.compose(S, sim3.inverse(S_ref))))


@pytest.mark.parametrize("lm", [0.0, 1e-3])
def test_robust_rounds_recover_exact_sim3_despite_outliers(lm):
    """Noise-free inliers and 10% gross outliers: the second round drops
    exactly the outliers and converges to the planted Sim3, which the Huber
    weights alone (one round) do not."""
    d, xyz, uv, kf, T, out = _views_with_outliers(6000, 41, 0.0)
    S0 = _S0(d)
    S1, _ = residual.refine_robust(S0, xyz, uv, kf, T, d["cam"], 2.45, iters=10, rounds=1, lm_lambda=lm)
    S2, n2 = residual.refine_robust(S0, xyz, uv, kf, T, d["cam"], 2.45, iters=10, rounds=2, outlier_px=3.035,
                                    lm_lambda=lm)
    assert _err(S2, d["S_true"]) < 1e-9
    assert _err(S1, d["S_true"]) > 1e-6
    assert n2 == int((~out).sum())


def test_robust_round_zero_is_gauss_newton():
    d, xyz, uv, kf, T, _ = _views_with_outliers(4000, 43, 1.0)
    S0 = _S0(d)
    S, n = residual.refine_robust(S0, xyz, uv, kf, T, d["cam"], 2.45, iters=7, rounds=1)
    assert np.array_equal(S, residual.gauss_newton(S0, xyz, uv, kf, T, d["cam"], 2.45, iters=7))
    assert n == len(xyz)


def test_lm_with_vanishing_damping_is_gauss_newton_one_step_behind():
    """With lambda -> 0 every step that lowers the loss is the Gauss-Newton
    step: m accepted candidates are m Gauss-Newton updates."""
    d, xyz, uv, kf, T, _ = _views_with_outliers(4000, 45, 1.0)
    S0 = _S0(d)
    h = []
    S, _ = residual.refine_robust(S0, xyz, uv, kf, T, d["cam"], 2.45, iters=8, rounds=1, lm_lambda=1e-14,
                                  history=h)
    status = [st for _, _, st in h]
    m = status.count("accept")
    assert m >= 2 and status[:m + 1] == ["start"] + ["accept"] * m
    assert _err(S, residual.gauss_newton(S0, xyz, uv, kf, T, d["cam"], 2.45, iters=m)) < 1e-10


def test_lm_accepted_loss_decreases_and_rejections_do_not_move():
    d, xyz, uv, kf, T, _ = _views_with_outliers(6000, 47, 1.0)
    S0 = _S0(d)
    h = []
    S, _ = residual.refine_robust(S0, xyz, uv, kf, T, d["cam"], 2.45, iters=8, rounds=2, outlier_px=3.035,
                                  lm_lambda=1e-3, history=h)
    for rnd in (0, 1):
        acc = [L for r, L, st in h if r == rnd and st in ("start", "accept")]
        assert all(b < a * (1 - residual.LM_CONVERGED) for a, b in zip(acc, acc[1:])), acc
        assert all(L > min(acc) for r, L, st in h if r == rnd and st == "reject")
        last = [st for r, _, st in h if r == rnd][-1]
        assert last in ("accept", "converged")   # a round ends accepting or converged
    assert h[0][1] > 10 * h[-1][1]
    # a huge damping barely moves: each step is a tiny gradient step
    S_big, _ = residual.refine_robust(S0, xyz, uv, kf, T, d["cam"], 2.45, iters=3, rounds=1, lm_lambda=1e12)
    assert _err(S_big, S0) < 1e-8


@pytest.fixture(scope="module")
def bidir():
    return synth.gen_bidir(n_fwd=4000, n_bwd=4000)


def test_inverse_direction_gradient_matches_central_differences(bidir):
    """The other direction's analytic gradient (chain rule through S^-1)
    against central differences of its loss under S <- exp(xi) S."""
    S0 = bidir["S0"]
    xyz, uv, kf, T = bidir["bwd"]
    T = T.astype(np.float64)
    g, H, _ = residual.grad_hess_inv(S0, xyz, uv, kf, T, bidir["cam"], 2.45)
    fd = np.zeros(7)
    for i in range(7):
        e = np.zeros(7)
        e[i] = 1e-6   # central differences: truncation ~h^2 (2e-9 relative here)
        fd[i] = (residual.forward_inv(sim3.compose(sim3.exp(e), S0), xyz, uv, kf, T, bidir["cam"], 2.45)[2]
                 - residual.forward_inv(sim3.compose(sim3.exp(-e), S0), xyz, uv, kf, T, bidir["cam"], 2.45)[2]) / 2e-6
    assert np.max(np.abs(g - fd)) / np.max(np.abs(fd)) < 1e-7
    assert np.allclose(H, H.T) and np.all(np.linalg.eigvalsh(H) > -1e-9 * np.max(np.abs(H)))


def test_inverse_direction_of_the_inverse_is_the_forward_residual(bidir):
    """Observing X through S^-1 with S replaced by its inverse is the forward
    residual: the two directions agree on the residual itself."""
    S0 = bidir["S0"]
    xyz, uv, kf, T = bidir["fwd"]
    T = T.astype(np.float64)
    r1, w1, L1 = residual.forward(S0, xyz, uv, kf, T, bidir["cam"], 2.45)
    r2, w2, L2 = residual.forward_inv(sim3.inverse(S0), xyz, uv, kf, T, bidir["cam"], 2.45)
    assert np.max(np.abs(r1 - r2)) < 1e-9 and abs(L1 - L2) < 1e-9 * L1


def test_bidirectional_gauss_newton_recovers_exact_sim3():
    d = synth.gen_bidir(seed=506, n_fwd=3000, n_bwd=3000, pix_sigma=0.0, outlier_frac=0.0)
    fwd = d["fwd"][:3] + (d["fwd"][3].astype(np.float64),)
    bwd = d["bwd"][:3] + (d["bwd"][3].astype(np.float64),)
    S = residual.gauss_newton_bidir(d["S0"], fwd, bwd, d["cam"], 2.45, iters=10)
    assert _err(S, d["S_true"]) < 1e-7 < _err(d["S0"], d["S_true"])
    # each direction alone also pins the truth: the sets are consistent
    S1 = residual.gauss_newton(d["S0"], *fwd, d["cam"], 2.45, iters=10)
    assert _err(S1, d["S_true"]) < 1e-7
