"""Pins for the oracle's guides (Sec. IV-B-3) and quadrotor model (Sec. III-A).

Guides are checked against their six boundary conditions (evaluated by
differentiating the polynomial, not by the solver) and a textbook closed
form; the RK4 model against motions whose exact solution is known.
"""
import math

import numpy as np
import pytest

from oracle import dynamics as D
from oracle import guides as G


def test_guide_boundary_conditions():
    rng = np.random.default_rng(1)
    for _ in range(20):
        p0, v0, a0 = rng.normal(size=3), rng.normal(size=3) * 3, rng.normal(size=3)
        anc = rng.normal(size=(6, 3)) * 5
        vT, aT = rng.normal(size=(6, 3)), rng.normal(size=(6, 3))
        T = float(rng.uniform(0.5, 4.0))
        f32 = lambda x: np.asarray(x, np.float32).astype(np.float64)
        coef = G.build_guides(p0, v0, a0, anc, T, end_vel=vT, end_acc=aT)
        T64 = float(np.float32(T))
        for m in range(6):
            at0 = [G.evaluate(coef[m], [0.0], k)[:, 0] for k in range(3)]
            atT = [G.evaluate(coef[m], [T64], k)[:, 0] for k in range(3)]
            np.testing.assert_allclose(at0[0], f32(p0), atol=1e-12)
            np.testing.assert_allclose(at0[1], f32(v0), atol=1e-12)
            np.testing.assert_allclose(at0[2], f32(a0), atol=1e-12)
            np.testing.assert_allclose(atT[0], f32(anc[m]), atol=1e-9)
            np.testing.assert_allclose(atT[1], f32(vT[m]), atol=1e-9)
            np.testing.assert_allclose(atT[2], f32(aT[m]), atol=1e-9)


def test_guide_closed_form():
    """Textbook minimum-jerk style closed form for the quintic coefficients."""
    rng = np.random.default_rng(2)
    p0, v0, a0 = rng.normal(size=3), rng.normal(size=3), rng.normal(size=3)
    pT, vT, aT = rng.normal(size=3) * 4, rng.normal(size=3), rng.normal(size=3)
    T = 2.0
    coef = G.build_guides(p0, v0, a0, pT[None], T, end_vel=vT[None], end_acc=aT[None])[0]
    f = lambda x: np.asarray(x, np.float32).astype(np.float64)
    p0, v0, a0, pT, vT, aT = map(f, (p0, v0, a0, pT, vT, aT))
    dP = pT - (p0 + v0 * T + 0.5 * a0 * T * T)
    dV = (vT - v0 - a0 * T) * T
    dA = (aT - a0) * T * T
    expect = np.stack([p0, v0, 0.5 * a0,
                       (10 * dP - 4 * dV + 0.5 * dA) / T ** 3,
                       (-15 * dP + 7 * dV - dA) / T ** 4,
                       (6 * dP - 3 * dV + 0.5 * dA) / T ** 5], -1)
    np.testing.assert_allclose(coef, expect, rtol=1e-10, atol=1e-12)


def test_rest_to_rest_guide_is_straight_and_monotone():
    anchor = np.array([[3.0, 4.0, 1.0]])
    coef = G.build_guides(np.zeros(3), np.zeros(3), np.zeros(3), anchor, 1.0)
    pos = G.guide_positions(coef, 20, 0.05)[0]
    a = np.asarray(anchor[0], np.float32).astype(np.float64)
    cross = np.cross(pos, a)
    assert np.abs(cross).max() < 1e-12
    s = pos @ a / (a @ a)
    assert np.all(np.diff(s) > 0) and abs(s[-1] - 1.0) < 1e-12


def test_default_end_velocity():
    coef = G.build_guides(np.zeros(3), [2.0, 0, 0], np.zeros(3), [[0.0, 5.0, 0.0]], 2.0)
    vT = G.evaluate(coef[0], [2.0], 1)[:, 0]
    np.testing.assert_allclose(vT, [0.0, 2.0, 0.0], atol=1e-12)


HOVER = dict(mass=1.0, gravity=9.81)


def test_hover_is_an_equilibrium():
    x0 = np.array([1.0, -2.0, 3.0, 1, 0, 0, 0, 0, 0, 0])
    u = np.tile([9.81, 0, 0, 0], (30, 1))
    xs = D.rollout(x0, u, 0.05, 1.0, 9.81)
    assert np.array_equal(xs, np.broadcast_to(x0, xs.shape))


@pytest.mark.parametrize("F", [0.0, 4.0, 16.35])
def test_constant_thrust_is_exact_parabola(F):
    """RK4 is exact for p'' = const: p = p0 + v0 t + a t^2 / 2."""
    x0 = np.array([0.3, 0.2, -1.0, 1, 0, 0, 0, 1.5, -0.5, 2.0])
    dt, N = 0.05, 40
    xs = D.rollout(x0, np.tile([F, 0, 0, 0], (N, 1)), dt, 1.0, 9.81)
    t = dt * np.arange(N + 1)
    acc = np.array([0.0, 0.0, F - 9.81])
    p = x0[:3] + np.outer(t, x0[7:10]) + 0.5 * np.outer(t * t, acc)
    v = x0[7:10] + np.outer(t, acc)
    np.testing.assert_allclose(xs[:, 0:3], p, atol=1e-12)
    np.testing.assert_allclose(xs[:, 7:10], v, atol=1e-12)


def test_body_rate_step_is_truncated_exponential():
    """For q' = q (x) [0, w]/2 with constant w, one RK4 step equals the
    degree-4 Taylor polynomial of the exponential, then normalised."""
    rng = np.random.default_rng(3)
    for _ in range(10):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w = rng.normal(size=3) * 2
        dt = 0.05
        x = np.concatenate([[0, 0, 0], q, [0, 0, 0]])
        x1 = D.rk4_step(x, np.concatenate([[0.0], w]), dt, 1.0, 9.81)
        th = dt * np.linalg.norm(w)
        qw = np.concatenate([[0.0], w])
        # Hamilton product q (x) (0, w) written for this check
        a = q
        b = qw
        prod = np.array([a[0]*b[0]-a[1]*b[1]-a[2]*b[2]-a[3]*b[3],
                         a[0]*b[1]+a[1]*b[0]+a[2]*b[3]-a[3]*b[2],
                         a[0]*b[2]-a[1]*b[3]+a[2]*b[0]+a[3]*b[1],
                         a[0]*b[3]+a[1]*b[2]-a[2]*b[1]+a[3]*b[0]])
        expect = (1 - th ** 2 / 8 + th ** 4 / 384) * q + dt * (1 - th ** 2 / 24) * 0.5 * prod
        expect /= np.linalg.norm(expect)
        np.testing.assert_allclose(x1[3:7], expect, atol=3e-16)


def test_yaw_rate_keeps_hover():
    """Rotation about the body z axis leaves the thrust direction vertical."""
    x0 = np.array([0, 0, 0, 1, 0, 0, 0, 0, 0, 0.0])
    xs = D.rollout(x0, np.tile([9.81, 0, 0, 1.3], (20, 1)), 0.05, 1.0, 9.81)
    assert np.abs(xs[:, 7:10]).max() < 1e-13
    ang = 2 * np.arctan2(xs[-1, 6], xs[-1, 3])
    th = 0.05 * 1.3
    step = 2 * math.atan2((1 - th ** 2 / 24) * th / 2, 1 - th ** 2 / 8 + th ** 4 / 384)
    assert abs(ang - 20 * step) < 1e-12 and abs(ang - 1.3) < 2e-8
    np.testing.assert_allclose(np.linalg.norm(xs[:, 3:7], axis=1), 1.0, atol=1e-15)


def test_tilted_thrust_direction():
    """With q a rotation of theta about +x, thrust points along R e3 =
    (0, -sin theta, cos theta): the velocity after one step is exact."""
    th = 0.3
    q = np.array([math.cos(th / 2), math.sin(th / 2), 0, 0])
    x0 = np.concatenate([[0, 0, 0], q, [0, 0, 0]])
    x1 = D.rk4_step(x0, np.array([10.0, 0, 0, 0]), 0.1, 1.0, 9.81)
    np.testing.assert_allclose(x1[7:10], [0.0, -10 * math.sin(th) * 0.1,
                                          (10 * math.cos(th) - 9.81) * 0.1], atol=1e-14)
