"""Pins of the float64 Sim3 algebra: closed forms of special cases, group
laws and the one-parameter-subgroup property."""
import numpy as np
import pytest

from oracle import sim3


def rodrigues(w):
    th = np.linalg.norm(w)
    if th == 0:
        return np.eye(3)
    K = sim3.hat(w / th)
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K


RNG = np.random.default_rng(21)
XIS = [RNG.normal(size=7) * np.array([0.3, 0.3, 0.3, 1, 1, 1, 0.2]) for _ in range(6)]


def test_pure_scale_translation():
    # omega = 0: R = I, s = e^sigma, t = upsilon (e^sigma - 1) / sigma
    for sig in (0.3, -0.2, 1e-3):
        ups = np.array([0.4, -1.0, 2.0])
        S = sim3.exp(np.concatenate([[0, 0, 0], ups, [sig]]))
        assert np.allclose(S[:9], np.eye(3).reshape(9), atol=1e-14)
        assert np.isclose(S[12], np.exp(sig), rtol=1e-13)
        assert np.allclose(S[9:12], ups * np.expm1(sig) / sig, rtol=1e-12)


def test_rigid_motion_is_se3_exponential():
    # sigma = 0: the textbook SE(3) exponential (Rodrigues rotation and
    # V = I + (1 - cos th)/th^2 W + (th - sin th)/th^3 W^2)
    w = np.array([0.3, -0.5, 0.2])
    ups = np.array([1.0, 2.0, -0.5])
    S = sim3.exp(np.concatenate([w, ups, [0.0]]))
    th = np.linalg.norm(w)
    W = sim3.hat(w)
    V = np.eye(3) + (1 - np.cos(th)) / th**2 * W + (th - np.sin(th)) / th**3 * W @ W
    assert np.allclose(S[:9].reshape(3, 3), rodrigues(w), atol=1e-13)
    assert np.allclose(S[9:12], V @ ups, atol=1e-13)
    assert np.isclose(S[12], 1.0, atol=1e-14)


@pytest.mark.parametrize("xi", XIS)
def test_group_laws(xi):
    S = sim3.exp(xi)
    R = S[:9].reshape(3, 3)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-12) and np.isclose(np.linalg.det(R), 1.0)
    I = sim3.compose(S, sim3.inverse(S))
    assert np.allclose(I, sim3.identity(), atol=1e-12)
    assert np.allclose(sim3.log(S), xi, atol=1e-10)
    # one-parameter subgroup: exp(a xi) exp(b xi) = exp((a + b) xi)
    assert np.allclose(sim3.compose(sim3.exp(0.3 * xi), sim3.exp(0.7 * xi)), S, atol=1e-12)


def test_action_and_composition():
    A, B = sim3.exp(XIS[0]), sim3.exp(XIS[1])
    X = RNG.normal(size=(5, 3))
    assert np.allclose(sim3.act(sim3.compose(A, B), X), sim3.act(A, sim3.act(B, X)), atol=1e-12)
    # action is s R X + t
    R, t, s = A[:9].reshape(3, 3), A[9:12], A[12]
    assert np.allclose(sim3.act(A, X), s * X @ R.T + t, atol=1e-12)
