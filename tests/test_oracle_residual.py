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
