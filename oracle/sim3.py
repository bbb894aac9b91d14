"""Sim(3) algebra in float64 (test infrastructure only).

The paper corrects keyframe poses with an estimated Sim3 (Sec. III-B) and
refines that Sim3 after projection search (Sec. IV-C).  A Sim3 here is the
13-vector ``[R (row-major 9), t (3), s]`` acting as ``X -> s R X + t``.  The
tangent is ``xi = (omega, upsilon, sigma)`` and the exponential is, by
definition, the matrix exponential of the 4x4 generator
``[[sigma I + [omega]x, upsilon], [0, 0]]``; this module evaluates exactly that
with ``scipy.linalg.expm`` instead of a closed form.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm, logm


def hat(w) -> np.ndarray:
    w = np.asarray(w, np.float64)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def generator(xi) -> np.ndarray:
    xi = np.asarray(xi, np.float64)
    G = np.zeros((4, 4))
    G[:3, :3] = xi[6] * np.eye(3) + hat(xi[:3])
    G[:3, 3] = xi[3:6]
    return G


def to_matrix(S) -> np.ndarray:
    S = np.asarray(S, np.float64)
    M = np.eye(4)
    M[:3, :3] = S[12] * S[:9].reshape(3, 3)
    M[:3, 3] = S[9:12]
    return M


def from_matrix(M) -> np.ndarray:
    A = M[:3, :3]
    s = np.cbrt(np.linalg.det(A))
    return np.concatenate([(A / s).reshape(9), M[:3, 3], [s]])


def exp(xi) -> np.ndarray:
    return from_matrix(expm(generator(xi)))


def log(S) -> np.ndarray:
    L = np.real(logm(to_matrix(S)))
    return np.array([L[2, 1], L[0, 2], L[1, 0], L[0, 3], L[1, 3], L[2, 3], np.trace(L[:3, :3]) / 3.0])


def compose(A, B) -> np.ndarray:
    """(A o B)(X) = A(B(X))."""
    return from_matrix(to_matrix(A) @ to_matrix(B))


def inverse(S) -> np.ndarray:
    return from_matrix(np.linalg.inv(to_matrix(S)))


def act(S, X) -> np.ndarray:
    S = np.asarray(S, np.float64)
    return np.asarray(X, np.float64) @ (S[12] * S[:9].reshape(3, 3)).T + S[9:12]


def identity() -> np.ndarray:
    return np.concatenate([np.eye(3).reshape(9), np.zeros(3), [1.0]])


def to_f32_rows(S) -> np.ndarray:
    """Float32 search form ``[sR (9), t (3), 1/s, 0, 0, 0]`` of a Sim3."""
    S = np.asarray(S, np.float64)
    out = np.zeros(16, np.float32)
    out[:9] = (S[12] * S[:9]).astype(np.float32)
    out[9:12] = S[9:12].astype(np.float32)
    out[12] = np.float32(1.0 / S[12])
    return out
