"""Pins for the oracle's costs (Sec. IV-C), MPPI weights/update (Sec. III-B),
Stage-II selection and the noise generator.
"""
import math

import numpy as np
import pytest

from fixtures import make_plain_problem, table1_params
from oracle import cost as C
from oracle import mppi as MP
from oracle import philox as PH
from oracle.guides import build_guides


def test_collision_penalty_branches():
    prm = table1_params()
    f = lambda d: C.collision_penalty(d, 1e6, 5.0, 0.4, 1.0)
    assert f(0.0) == 1e6 and f(0.3999) == 1e6
    assert f(np.float64(np.float32(0.4))) == pytest.approx(1e6, rel=1e-7)
    assert f(0.9999999) == pytest.approx(1e6 * math.exp(-5 * 0.5999999), rel=1e-12)
    assert f(np.nextafter(1.0, 0)) == pytest.approx(4.9787068e4, rel=1e-7)
    assert f(1.0) == 0.0 and f(np.inf) == 0.0
    assert prm["C"] == 1e6


def _random_quat(rng, n):
    q = rng.normal(size=(n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def test_attitude_error_identity():
    """|R(q) R(q_g)^T - I|_F = 2 sqrt(2) |vec(q_g^* (x) q)| = 2 sqrt(2) |sin(angle/2)|."""
    rng = np.random.default_rng(0)
    q, qg = _random_quat(rng, 500), _random_quat(rng, 500)
    e = C.attitude_error(q, qg)
    qgc = qg * np.array([1, -1, -1, -1])
    w = qgc[:, 0:1] * q[:, 1:] + q[:, 0:1] * qgc[:, 1:] + np.cross(qgc[:, 1:], q[:, 1:])
    np.testing.assert_allclose(e, 2 * math.sqrt(2) * np.linalg.norm(w, axis=1), atol=1e-12)
    assert np.abs(C.attitude_error(q, q)).max() < 1e-7
    th = 0.7
    e1 = C.attitude_error(np.array([math.cos(th / 2), 0, math.sin(th / 2), 0]), np.array([1.0, 0, 0, 0]))
    assert e1 == pytest.approx(2 * math.sqrt(2) * math.sin(th / 2), rel=1e-12)


def test_nearest_brute_vs_loops_and_kdtree():
    rng = np.random.default_rng(1)
    cloud = (rng.normal(size=(300, 3)) * 4).astype(np.float32)
    cloud[17] = cloud[5]                       # exact duplicate: lowest index wins
    q = rng.normal(size=(40, 3)) * 4
    q[0] = cloud[5].astype(np.float64)
    d, idx = C.nearest(cloud, q, chunk=7)
    for a in range(len(q)):
        best, bi = math.inf, -1
        for b in range(len(cloud)):
            o = cloud[b].astype(np.float64)
            s = (q[a, 0] - o[0]) ** 2 + (q[a, 1] - o[1]) ** 2 + (q[a, 2] - o[2]) ** 2
            if s < best:
                best, bi = s, b
        assert idx[a] == bi and d[a] == math.sqrt(best)
    assert idx[0] == 5 and d[0] == 0.0
    big = (rng.normal(size=(20000, 3)) * 10).astype(np.float32)
    qq = rng.normal(size=(500, 3)) * 10
    d1, _ = C.nearest(big, qq)
    d2, _ = C.nearest_kdtree(big, qq)
    np.testing.assert_allclose(d1, d2, rtol=1e-13)
    de, ie = C.nearest(np.zeros((0, 3), np.float32), qq[:3])
    assert np.all(np.isinf(de)) and np.all(ie == -1)


def test_nearest_single_obstacle_straight_line():
    """Straight-line rollout past one point: d_t = distance to the line point."""
    o = np.array([[2.0, 1.5, 0.0]], np.float32)
    t = np.arange(1, 21) * 0.25
    path = np.stack([t, np.zeros_like(t), np.zeros_like(t)], 1)
    d, _ = C.nearest(o, path)
    np.testing.assert_allclose(d, np.sqrt((t - 2.0) ** 2 + 1.5 ** 2), rtol=1e-15)


def _hover_problem(K=4, N=6, M=2):
    prob = make_plain_problem()
    prob = dict(prob)
    prob["M"], prob["K"], prob["N"] = M, K, N
    prob["u_nom"] = np.tile(np.float32([9.81, 0, 0, 0]), (M, N, 1)).astype(np.float32)
    prob["cloud"] = np.zeros((0, 3), np.float32)
    prm = dict(prob["params"])
    prm["sigma"] = np.zeros(4, np.float32)
    prob["params"] = prm
    return prob


def test_hover_rollout_cost_closed_form():
    prob = _hover_problem()
    prm = prob["params"]
    N, M = prob["N"], prob["M"]
    coef = np.zeros((M, 3, 6))                       # guide held at the origin
    st = MP.mppi_step(prob, coef)
    g = np.asarray(prob["p_goal"], np.float32).astype(np.float64)
    t = st["terms"]
    assert np.allclose(t["goal"], N * (3.0 * np.linalg.norm(g) + 0.25 * 0.0), rtol=1e-14)
    assert np.all(t["vnorm"] == 0.0) and np.all(t["track"] == 0.0) and np.all(t["col"] == 0.0)
    mg = float(np.float32(9.81))
    assert np.allclose(t["ctrl"], (N - 1) * 0.5 * mg * mg, rtol=1e-14)


def test_zero_noise_gives_nominal():
    """sigma = 0: every sample is the nominal rollout, S equal, eps = 1/K, no update."""
    prob = make_plain_problem()
    prob = dict(prob)
    prm = dict(prob["params"])
    prm["sigma"] = np.zeros(4, np.float32)
    prob["params"] = prm
    prob["K"] = 8
    coef = build_guides(prob["x0"][:3], prob["x0"][7:10], np.zeros(3), prob["anchors"], 1.0)
    rng = np.random.default_rng(0)
    u0 = prob["u_nom"].copy()
    u0[..., 1:] = rng.uniform(-1, 1, u0[..., 1:].shape).astype(np.float32)
    st = MP.mppi_step(prob, coef, u_nom=u0)
    assert np.all(st["S1"] == st["S1"][:, :1])
    assert np.all(st["eps"] == 1.0 / 8)
    assert np.array_equal(st["u_new"], u0.astype(np.float64))
    assert np.all(st["states"] == st["states"][:, :1])


def test_weights_properties():
    rng = np.random.default_rng(4)
    S = rng.uniform(0, 50, size=(3, 200))
    e = MP.mppi_weights(S, 0.1)
    assert np.all(e >= 0) and np.allclose(e.sum(1), 1.0, atol=1e-12)
    np.testing.assert_allclose(MP.mppi_weights(S + 1234.5, 0.1), e, atol=1e-13)
    one = MP.mppi_weights(S, 1e-9)
    assert np.array_equal(np.argmax(one, 1), np.argmin(S, 1)) and np.allclose(one.max(1), 1.0)
    flat = MP.mppi_weights(S, 1e9)
    np.testing.assert_allclose(flat, 1.0 / 200, rtol=1e-6)


def test_update_stays_in_box_and_single_sample():
    prob = dict(make_plain_problem())
    prob["K"] = 1
    prob["N"] = 20
    coef = build_guides(prob["x0"][:3], prob["x0"][7:10], np.zeros(3), prob["anchors"], 1.0)
    st = MP.mppi_step(prob, coef)
    prm = prob["params"]
    n = PH.normals(prm["seed"], prob["problem_id"], 1, 1, 20)
    expect = np.clip(prob["u_nom"].astype(np.float64) + prm["sigma"].astype(np.float64) * n[:, 0],
                     prm["u_min"].astype(np.float64), prm["u_max"].astype(np.float64))
    np.testing.assert_allclose(st["u_new"], expect, atol=1e-14)
    prob["K"] = 64
    prm2 = dict(prm)
    prm2["sigma"] = np.float32([8.0, 6.0, 6.0, 6.0])
    prob["params"] = prm2
    st = MP.mppi_step(prob, coef)
    lo, hi = prm["u_min"].astype(np.float64), prm["u_max"].astype(np.float64)
    assert np.all(st["u_new"] >= lo - 1e-12) and np.all(st["u_new"] <= hi + 1e-12)
    assert np.any(st["u"] == lo) and np.any(st["u"] == hi)


def test_ctrl_sum_bounds():
    """J_ctrl sums |u_t|^2 over t = 0..N-2 and |u_t - u_{t-1}|^2 over t = 1..N-2."""
    rng = np.random.default_rng(9)
    N = 7
    u = rng.normal(size=(N, 4))
    states = np.zeros((N + 1, 10))
    states[:, 3] = 1.0
    prm = table1_params()
    t = C.cost_terms(states, u, None, (np.zeros(3), np.zeros(3), [1, 0, 0, 0]), prm,
                     np.full(N, np.inf))
    ref = 0.0
    for k in range(0, N - 1):
        ref += 0.5 * sum(u[k] ** 2)
    for k in range(1, N - 1):
        ref += 0.5 * sum((u[k] - u[k - 1]) ** 2)
    assert t["ctrl"] == pytest.approx(ref, rel=1e-14)


def test_stage2_rejects_guide_through_obstacle():
    """An instance whose nominal path crosses a cylinder costs >= C and loses."""
    prob = dict(make_plain_problem())
    rng = np.random.default_rng(0)
    th = rng.uniform(-np.pi, np.pi, 4000)
    z = rng.uniform(-2, 6, 4000)
    cyl = np.stack([3.0 + 0.3 * np.cos(th), 0.3 * np.sin(th), z], 1).astype(np.float32)
    prob["cloud"] = cyl
    N = 40
    u = np.zeros((2, N, 4), np.float32)
    u[:, :, 0] = 9.81
    prob["x0"] = np.float32([0, 0, 0, 1, 0, 0, 0, 4.0, 0, 0])      # flying at +x, 4 m/s
    u[1, :, 3] = 0.0
    u[1, :10, 1] = -0.5                                            # roll: turn away (+y)
    sel = MP.select_best(prob, u)
    assert sel["terms"]["col"][0] >= 1e6
    assert sel["best"] == 1


def test_philox_statistics():
    """Uniform words and standard normals (the only property the method needs)."""
    w = PH.raw_words(0, 0, 4, 256, 64)
    top = (w >> 28).ravel()
    counts = np.bincount(top, minlength=16)
    exp = top.size / 16
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 40.0                        # 15 dof, p ~ 5e-4
    n = PH.normals(0, 0, 4, 256, 64).reshape(-1, 4)
    assert np.abs(n.mean(0)).max() < 0.02
    assert np.abs(n.var(0) - 1.0).max() < 0.02
    c = np.corrcoef(n.T)
    assert np.abs(c - np.eye(4)).max() < 0.02
    from scipy import stats
    for ch in range(4):
        assert stats.kstest(n[:, ch], "norm").pvalue > 1e-3
    # different key / counter word -> unrelated streams
    n2 = PH.normals(0, 1, 4, 256, 64).reshape(-1, 4)
    n3 = PH.normals(0, 0, 4, 256, 64, iteration=1).reshape(-1, 4)
    assert abs(np.corrcoef(n[:, 0], n2[:, 0])[0, 1]) < 0.02
    assert abs(np.corrcoef(n[:, 0], n3[:, 0])[0, 1]) < 0.02


def test_philox_is_a_bijection_on_a_counter_block():
    m, k, t = np.meshgrid(np.arange(4), np.arange(1024), np.arange(16), indexing="ij")
    out = PH.philox4x32_10((k, t, m, np.zeros_like(k)), (12345, 678))
    packed = (out[0].astype(np.uint64) << np.uint64(32)) | out[1].astype(np.uint64)
    assert len(np.unique(packed)) == packed.size


def test_stage1_terms_on_exact_parabola():
    """Constant thrust, level attitude, no noise: every state is a parabola
    in closed form, so J_track, J_vnorm and J_goal follow without RK4."""
    prob = dict(make_plain_problem())
    prm = dict(prob["params"])
    prm["sigma"] = np.zeros(4, np.float32)
    prob["params"] = prm
    M, K, N = 1, 2, 20
    prob.update(M=M, K=K, N=N, cloud=np.zeros((0, 3), np.float32))
    prob["x0"] = np.float32([0.5, -1.0, 2.0, 1, 0, 0, 0, 3.0, 1.0, -0.5])
    F = np.float32(12.0)
    prob["u_nom"] = np.tile(np.float32([F, 0, 0, 0]), (M, N, 1))
    coef = np.zeros((M, 3, 6))
    coef[0, :, 0] = [1.0, 0.0, 2.0]
    coef[0, :, 1] = [2.5, 0.5, 0.0]               # guide f(tau) = c0 + c1 tau
    st = MP.mppi_step(prob, coef)
    dt = float(np.float32(0.05))
    tau = (np.arange(N) + 1) * dt
    x0 = prob["x0"].astype(np.float64)
    acc = np.array([0, 0, float(F) - float(np.float32(9.81))])   # parameters enter as float32
    p = x0[:3] + np.outer(tau, x0[7:10]) + 0.5 * np.outer(tau ** 2, acc)
    v = x0[7:10] + np.outer(tau, acc)
    f = coef[0, :, 0] + np.outer(tau, coef[0, :, 1])
    g = prob["p_goal"].astype(np.float64)
    t = st["terms"]
    assert t["track"][0, 0] == pytest.approx(15.0 * np.linalg.norm(p - f, axis=1).sum(), rel=1e-12)
    assert t["vnorm"][0, 0] == pytest.approx(float(np.float32(0.15)) * (v * v).sum(), rel=1e-12)
    goal = 3.0 * np.linalg.norm(p - g, axis=1).sum() + 0.25 * np.linalg.norm(v, axis=1).sum()
    assert t["goal"][0, 0] == pytest.approx(goal, rel=1e-12)
    w = np.float32([2.0, 3.0, 0.5, 1.5, 7.0])
    prm["w"] = w
    st2 = MP.mppi_step(prob, coef)
    tot = sum(float(w[i]) * st2["terms"][n][0, 0] for i, n in enumerate(C.TERMS))
    assert st2["S1"][0, 0] == pytest.approx(tot, rel=1e-14)


def test_iterations_chain_noise_and_controls():
    """Several iterations per step: with K = 1 each iteration is u <- clip(u + sigma n_i)
    with n_i drawn at counter word iter_base + i, u_nom held in float32 between
    iterations; sigma = 0 leaves u unchanged."""
    prob = dict(make_plain_problem())
    prob.update(K=1, N=12)
    prob["u_nom"] = prob["u_nom"][:, :12].copy()
    prm = dict(prob["params"])
    prm["iter_base"] = 5
    prob["params"] = prm
    coef = build_guides(prob["x0"][:3], prob["x0"][7:10], np.zeros(3), prob["anchors"], 0.6)
    its = MP.mppi_iterations(prob, coef, 3)
    lo, hi = prm["u_min"].astype(np.float64), prm["u_max"].astype(np.float64)
    u = prob["u_nom"].astype(np.float64)
    for i, st in enumerate(its):
        n = PH.normals(prm["seed"], prob["problem_id"], 1, 1, 12, iteration=5 + i)
        u = u.astype(np.float32).astype(np.float64)
        u = np.clip(u + prm["sigma"].astype(np.float64) * n[:, 0], lo, hi)
        np.testing.assert_allclose(st["u_new"], u, atol=1e-13)
    assert not np.allclose(its[0]["u_new"] - prob["u_nom"], its[1]["u_new"] - its[0]["u_new"])
    prm0 = dict(prm)
    prm0["sigma"] = np.zeros(4, np.float32)
    prob["params"] = prm0
    prob["K"] = 6
    its = MP.mppi_iterations(prob, coef, 4)
    assert np.array_equal(its[-1]["u_new"], prob["u_nom"].astype(np.float64))
