"""Quintic guiding trajectories, Sec. IV-B-3, eq. (polynomial).

Each axis is f(t) = sum_{i=0..5} a_i t^i on [0, T], T = N dt, with the six
coefficients fixed by position, velocity and acceleration at both ends.
The oracle forms that 6 x 6 linear system literally and solves it.

Reading of the end conditions (the paper gives none): start at the current
(p0, v0, a0); end at the anchor with velocity |v0| times the unit vector
from p0 to the anchor and zero acceleration, unless given explicitly.
"""
import numpy as np


def boundary_matrix(T):
    T = float(T)
    return np.array([
        [1, 0, 0, 0, 0, 0],
        [0, 1, 0, 0, 0, 0],
        [0, 0, 2, 0, 0, 0],
        [1, T, T ** 2, T ** 3, T ** 4, T ** 5],
        [0, 1, 2 * T, 3 * T ** 2, 4 * T ** 3, 5 * T ** 4],
        [0, 0, 2, 6 * T, 12 * T ** 2, 20 * T ** 3],
    ], np.float64)


def default_end_velocity(p0, v0, anchors):
    p0 = np.asarray(p0, np.float64)
    a = np.asarray(anchors, np.float64).reshape(-1, 3)
    d = a - p0[None, :]
    n = np.linalg.norm(d, axis=1, keepdims=True)
    unit = np.where(n > 0.0, d / np.where(n > 0.0, n, 1.0), 0.0)
    return np.linalg.norm(np.asarray(v0, np.float64)) * unit


def build_guides(p0, v0, a0, anchors, T, end_vel=None, end_acc=None):
    """Coefficients a[m, axis, i] (float64 (M, 3, 6)) of every guide."""
    p0 = np.asarray(p0, np.float32).astype(np.float64)
    v0 = np.asarray(v0, np.float32).astype(np.float64)
    a0 = np.asarray(a0, np.float32).astype(np.float64)
    anc = np.asarray(anchors, np.float32).astype(np.float64).reshape(-1, 3)
    M = len(anc)
    vT = default_end_velocity(p0, v0, anc) if end_vel is None else \
        np.asarray(end_vel, np.float32).astype(np.float64).reshape(M, 3)
    aT = np.zeros((M, 3)) if end_acc is None else \
        np.asarray(end_acc, np.float32).astype(np.float64).reshape(M, 3)
    A = boundary_matrix(np.float64(np.float32(T)))
    coef = np.empty((M, 3, 6))
    for m in range(M):
        for ax in range(3):
            rhs = np.array([p0[ax], v0[ax], a0[ax], anc[m, ax], vT[m, ax], aT[m, ax]])
            coef[m, ax] = np.linalg.solve(A, rhs)
    return coef


def evaluate(coef, t, deriv=0):
    """f^(deriv)(t) for coef (..., 6) at times t (array) -> (..., len(t))."""
    coef = np.asarray(coef, np.float64)
    t = np.asarray(t, np.float64)
    out = np.zeros(coef.shape[:-1] + t.shape)
    for i in range(deriv, 6):
        fac = 1.0
        for r in range(deriv):
            fac *= (i - r)
        out = out + fac * coef[..., i, None] * t ** (i - deriv)
    return out


def guide_positions(coef, N, dt):
    """p_traj(t) = f((t+1) dt), t = 0..N-1 (reading: the cost of step t is
    taken at the state after control t); returns (M, N, 3)."""
    tt = (np.arange(N, dtype=np.float64) + 1.0) * np.float64(np.float32(dt))
    return np.moveaxis(evaluate(coef, tt), -1, -2)
