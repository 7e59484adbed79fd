"""Pins for the oracle's gradient (frozen active set), PyTorch float64 autograd.

The frozen forward must reproduce the NumPy oracle's costs; its autograd gradient
must agree with central finite differences of the same frozen function; the
weight gradient is the vector of summed terms; clipped controls get no gradient.
"""
import numpy as np
import pytest
import torch

from fixtures import make_plain_problem
from oracle import adjoint as A
from oracle import mppi as OM
from oracle.guides import build_guides


def small_problem(K=24, N=12, M=2, seed=0):
    prob = dict(make_plain_problem())
    rng = np.random.default_rng(seed)
    prob.update(M=M, K=K, N=N)
    prob["x0"] = np.float32([0, 0, 0, 1, 0, 0, 0, 2.0, 0.3, 0.0])
    prob["u_nom"] = (np.float32([9.81, 0, 0, 0]) + rng.normal(size=(M, N, 4)) * 0.3).astype(np.float32)
    # keep the cloud near the rollouts so every collision branch occurs
    th = rng.uniform(-np.pi, np.pi, 600)
    z = rng.uniform(-1, 2, 600)
    prob["cloud"] = np.stack([1.6 + 0.3 * np.cos(th), 0.55 + 0.3 * np.sin(th), z], 1).astype(np.float32)
    anchors = np.float32([[4, 0.5, 0.3], [4, -0.5, -0.2]])[:M]
    coef = build_guides(prob["x0"][:3], prob["x0"][7:10], np.zeros(3), anchors, N * 0.05)
    return prob, coef


def test_frozen_forward_matches_numpy_oracle():
    prob, coef = small_problem()
    act = A.active_set(prob, coef)
    J = A.frozen_terms(prob, coef, torch.tensor(prob["u_nom"].astype(np.float64)), act)
    st = OM.mppi_step(prob, coef)
    for name in A.TERMS:
        np.testing.assert_allclose(J[name].numpy(), st["terms"][name], rtol=1e-12, atol=1e-9)
    assert set(np.unique(act["branch"])) == {0, 1, 2}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_autograd_matches_central_differences(seed):
    prob, coef = small_problem(seed=seed)
    act = A.active_set(prob, coef)
    gu, gw, L = A.grad(prob, coef, act)
    rng = np.random.default_rng(100 + seed)
    for _ in range(6):
        dirn = rng.normal(size=gu.shape)
        fd = A.fd_directional(prob, coef, act, dirn, h=1e-4)
        an = float((gu * dirn).sum())
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3 * np.abs(gu).sum())
    # L is linear in w: only the rounding of L itself (~eps |L| / h) limits the quotient
    np.testing.assert_allclose(A.fd_grad_w(prob, coef, act), gw, rtol=1e-8,
                               atol=8 * np.finfo(float).eps * abs(L) / 1e-4)


def test_weight_gradient_is_summed_terms():
    prob, coef = small_problem()
    act = A.active_set(prob, coef)
    _, gw, _ = A.grad(prob, coef, act, scale=0.5)
    st = OM.mppi_step(prob, coef)
    ref = [0.5 * st["terms"][n].sum() for n in A.TERMS]
    np.testing.assert_allclose(gw, ref, rtol=1e-12)


def test_clipped_control_has_no_gradient():
    prob, coef = small_problem(K=1, N=6, M=1)
    prob["u_nom"][0, 2, 0] = 16.35           # thrust at the upper limit
    prob["u_nom"][0, 4, 1] = -3.0            # roll rate at the lower limit
    act = A.active_set(prob, coef)
    gu, _, _ = A.grad(prob, coef, act)
    for (t, c) in [(2, 0), (4, 1)]:
        if not act["mask"][0, 0, t, c]:
            assert gu[0, t, c] == 0.0
    assert np.count_nonzero(~act["mask"]) >= 1
    assert np.abs(gu).sum() > 0


def test_collision_gradient_points_away_from_obstacle():
    """A single hovering sample next to one point: dL/dthrust follows the
    distance derivative sign of the middle collision branch."""
    prob, coef = small_problem(K=1, N=4, M=1)
    prm = dict(prob["params"])
    prm["sigma"] = np.zeros(4, np.float32)
    prm["w"] = np.float32([0, 0, 0, 0, 1])
    prob["params"] = prm
    prob["x0"] = np.float32([0, 0, 0, 1, 0, 0, 0, 0, 0, 0])
    prob["u_nom"] = np.tile(np.float32([9.81, 0, 0, 0]), (1, 4, 1))
    prob["cloud"] = np.float32([[0.0, 0.0, 0.7]])       # 0.7 m above: middle branch
    act = A.active_set(prob, coef)
    assert np.all(act["branch"] == 1)
    gu, _, _ = A.grad(prob, coef, act)
    # more thrust moves the drone up, closer to the point: cost increases
    assert np.all(gu[0, :-1, 0] > 0)


def test_empty_cloud_has_no_collision_gradient():
    prob, coef = small_problem(K=8, N=5, M=1)
    prob["cloud"] = np.zeros((0, 3), np.float32)
    act = A.active_set(prob, coef)
    assert np.all(act["branch"] == 2) and np.all(act["idx"] == -1)
    act2 = A.active_set(prob, coef, nearest_idx=np.full((1, 8, 5), -1))
    assert np.all(act2["branch"] == 2)
    prm = dict(prob["params"])
    prm["w"] = np.float32([0, 0, 0, 0, 1])
    prob["params"] = prm
    gu, gw, L = A.grad(prob, coef, act)
    assert L == 0.0 and np.all(gu == 0.0)
