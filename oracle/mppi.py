"""One MPPI iteration per instance and the Stage-II selection.

Sec. III-B: perturbed controls u^k_j = u^nom_j + delta^k_j (delta ~ N(0,
Sigma)), RK4 rollouts, per-rollout cost S_k, then eq. (mppi_weights)

  rho = min_k S_k,  eta = sum_k exp(-(S_k - rho)/lambda),
  eps_k = exp(-(S_k - rho)/lambda) / eta

and eq. (mppi_update): u^nom <- u^nom + sum_k eps_k delta u^k.

Sec. IV-C: M instances run in parallel, instance m tracking guide m with
the Stage-I cost S1; Stage II rolls the M updated sequences out without
noise, scores them with S2 = J_goal + J_col and keeps the cheapest.

Readings: perturbed controls are clipped to the Table I box and the
update uses the clipped perturbation delta_eff = clip(u^nom + delta) - u^nom
(so u^nom stays inside the box); one iteration per planning step; Stage-II
ties go to the lowest instance index.
"""
import numpy as np

from . import philox
from .cost import cost_terms, f64, nearest, weighted_sum
from .dynamics import rollout
from .guides import guide_positions


def perturb(u_nom, normals, prm):
    """u = clip(u_nom + sigma * n, u_min, u_max) and delta_eff = u - u_nom.

    u_nom (M, N, 4); normals (M, K, N, 4) -> both (M, K, N, 4) float64."""
    un = f64(u_nom)[:, None]
    u = np.clip(un + f64(prm["sigma"]) * np.asarray(normals, np.float64),
                f64(prm["u_min"]), f64(prm["u_max"]))
    return u, u - un


def mppi_weights(S, lam):
    """eq. (mppi_weights) along the last axis."""
    S = np.asarray(S, np.float64)
    rho = S.min(-1, keepdims=True)
    e = np.exp(-(S - rho) / f64(lam))
    return e / e.sum(-1, keepdims=True)


def mppi_update(u_nom, eps, delta_eff):
    """eq. (mppi_update): u_nom (M,N,4) + sum_k eps[m,k] delta_eff[m,k]."""
    return f64(u_nom) + np.einsum("mk,mknc->mnc", eps, delta_eff)


def goal_of(prob):
    return prob["p_goal"], prob["v_goal"], prob["q_goal"]


def mppi_step(prob, coef, u_nom=None, normals=None, nearest_fn=nearest,
              S1_override=None, iteration=0):
    """One Stage-I MPPI iteration for all M instances of a problem.

    Returns dict with u (M,K,N,4), delta_eff, states (M,K,N+1,10), d (M,K,N),
    nearest index, terms, S1 (M,K), eps (M,K), u_new (M,N,4).  With
    `S1_override` the weights use the given costs (teacher forcing).
    """
    prm = prob["params"]
    M, K, N = prob["M"], prob["K"], prob["N"]
    u_nom = prob["u_nom"] if u_nom is None else u_nom
    if normals is None:
        normals = philox.normals(prm["seed"], prob["problem_id"], M, K, N,
                                 int(prm["iter_base"]) + iteration)
    u, delta_eff = perturb(u_nom, normals, prm)
    dt = f64(prm["dt"])
    states = rollout(f64(prob["x0"]), u, dt, f64(prm["mass"]), f64(prm["gravity"]))
    p_traj = guide_positions(coef, N, prm["dt"])[:, None]
    d, idx = nearest_fn(prob["cloud"], states[..., 1:, 0:3].reshape(-1, 3))
    d, idx = d.reshape(M, K, N), idx.reshape(M, K, N)
    terms = cost_terms(states, u, p_traj, goal_of(prob), prm, d)
    S1 = weighted_sum(terms, prm["w"])
    S_used = S1 if S1_override is None else np.asarray(S1_override, np.float64)
    eps = mppi_weights(S_used, prm["lam"])
    return dict(u=u, delta_eff=delta_eff, states=states, d=d, nearest=idx,
                terms=terms, S1=S1, eps=eps, u_new=mppi_update(u_nom, eps, delta_eff))


def select_best(prob, u_nom, nearest_fn=nearest):
    """Stage II: noise-free rollout of each instance, S2 = J_goal + J_col."""
    prm = prob["params"]
    u = f64(u_nom)
    M, N = u.shape[0], u.shape[1]
    states = rollout(f64(prob["x0"]), u, f64(prm["dt"]), f64(prm["mass"]), f64(prm["gravity"]))
    d, _ = nearest_fn(prob["cloud"], states[..., 1:, 0:3].reshape(-1, 3))
    terms = cost_terms(states, u, None, goal_of(prob), prm, d.reshape(M, N))
    S2 = weighted_sum(terms, prm["w"], names=("goal", "col"))
    return dict(S2=S2, best=int(np.argmin(S2)), states=states, d=d.reshape(M, N), terms=terms)


def mppi_iterations(prob, coef, n_iter, nearest_fn=nearest):
    """Several Stage-I iterations in a row (Sec. III-B iterates sampling and update;
    iteration i draws its noise at counter word iter_base + i and starts from the
    previous iteration's u_nom).  Returns the list of per-iteration results."""
    out, u = [], prob["u_nom"]
    for i in range(int(n_iter)):
        st = mppi_step(prob, coef, u_nom=u, nearest_fn=nearest_fn, iteration=i)
        out.append(st)
        u = st["u_new"]
    return out


def plan_step(prob, nearest_fn=nearest):
    """Partition -> anchors -> guides -> Stage I -> Stage II for one problem."""
    from .guides import build_guides
    from .partition import partition_anchors
    part = prob["partition"]
    pa = partition_anchors(prob["cloud"], prob["goal_dir"], part["n_az_c"], part["n_el_c"],
                           part["f_a"], part["f_e"], part["r_max"], part["ell"],
                           prob["M_h"], prob["M_v"], p0=prob["x0"][:3])
    T = np.float32(prob["N"] * np.float32(prob["params"]["dt"]))
    coef = build_guides(prob["x0"][:3], prob["x0"][7:10], np.zeros(3, np.float32),
                        pa["anchors"].astype(np.float32), T)
    its = mppi_iterations(prob, coef, prob.get("n_iter", 1), nearest_fn=nearest_fn)
    sel = select_best(prob, its[-1]["u_new"], nearest_fn=nearest_fn)
    return dict(partition=pa, coef=coef, stage1=its[-1], iterations=its, stage2=sel)
