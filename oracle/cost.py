"""Two-stage cost, Sec. IV-C eq. (total cost) and its five terms.

  S1 = J_track + J_vnorm + J_ctrl + S2,   S2 = J_goal + J_col

Terms (scalar weights; the paper's Q matrices are given as scalars):
  J_track = sum_{t=0}^{N-1} Q_track |p_t - p_traj(t)|
  J_vnorm = sum_{t=0}^{N-1} Q_vnorm |v_t|^2
  J_ctrl  = sum_{t=0}^{N-2} Q_c |u_t|^2 + sum_{t=1}^{N-2} Q_cdelta |u_t - u_{t-1}|^2
  J_goal  = sum_{t=0}^{N-1} Q_p |p_t - p_g| + Q_v |v_t - v_g| + Q_q |R(q_t) R(q_g)^T - I|_F
  J_col   = sum_{t=0}^{N-1} phi(d_t),  d_t = min_o |p_t - o|
  phi(d)  = C if d < d_min;  C exp(-a (d - d_min)) if d_min <= d < d_max;  0 otherwise

Readings: (p_t, v_t, q_t) is the state after control t (x_{t+1}); u_t is
the perturbed, clipped control of the same sample and u_{t-1} its own
previous control; the sums keep the paper's bounds literally; the
collision set is the raw cloud unless a filtered set is passed; an empty
collision set gives d = +inf.  Each term may be scaled by a weight w_i
(default 1) in the order (track, vnorm, ctrl, goal, col).
"""
import numpy as np

from .dynamics import rotation_matrix

TERMS = ("track", "vnorm", "ctrl", "goal", "col")


def nearest(cloud, queries, chunk=256):
    """Brute force d = min_o |q - o| and the lowest index attaining min |q-o|^2.

    cloud float32 (P, 3); queries (Q, 3) (any float dtype).  Distances are
    computed as sqrt((qx-ox)^2 + (qy-oy)^2 + (qz-oz)^2) in float64.
    """
    o = np.asarray(cloud, np.float32).reshape(-1, 3).astype(np.float64)
    q = np.asarray(queries, np.float64).reshape(-1, 3)
    d2 = np.full(len(q), np.inf)
    idx = np.full(len(q), -1, np.int64)
    if len(o) == 0:
        return np.sqrt(d2), idx
    for s in range(0, len(q), chunk):
        qc = q[s:s + chunk]
        acc = (qc[:, None, 0] - o[None, :, 0]) ** 2
        acc += (qc[:, None, 1] - o[None, :, 1]) ** 2
        acc += (qc[:, None, 2] - o[None, :, 2]) ** 2
        i = np.argmin(acc, axis=1)
        idx[s:s + chunk] = i
        d2[s:s + chunk] = acc[np.arange(len(qc)), i]
    return np.sqrt(d2), idx


def nearest_kdtree(cloud, queries):
    """Exact nearest distance through a k-d tree (scipy); the index is any
    point attaining the minimum.  Used where brute force is too slow."""
    from scipy.spatial import cKDTree
    o = np.asarray(cloud, np.float32).reshape(-1, 3).astype(np.float64)
    q = np.asarray(queries, np.float64).reshape(-1, 3)
    if len(o) == 0:
        return np.full(len(q), np.inf), np.full(len(q), -1, np.int64)
    d, i = cKDTree(o).query(q, k=1)
    return d, i.astype(np.int64)


def collision_penalty(d, C, a, d_min, d_max):
    d = np.asarray(d, np.float64)
    return np.where(d < d_min, C, np.where(d < d_max, C * np.exp(-a * (d - d_min)), 0.0))


def attitude_error(q, q_goal):
    """|R(q) R(q_g)^T - I|_F, the matrix formula written out."""
    R = rotation_matrix(np.asarray(q, np.float64))
    Rg = rotation_matrix(np.asarray(q_goal, np.float64))
    E = R @ np.swapaxes(Rg, -1, -2) - np.eye(3)
    return np.sqrt((E * E).sum((-1, -2)))


def f64(v):
    return np.asarray(v, np.float32).astype(np.float64)


def cost_terms(states, u, p_traj, goal, prm, d):
    """Unweighted J terms for rollouts.

    states (..., N+1, 10), u (..., N, 4), p_traj (..., N, 3) or None,
    goal = (p_g, v_g, q_g), d (..., N) nearest distances of p_t.
    Returns dict name -> (...) float64.
    """
    p = states[..., 1:, 0:3]
    q = states[..., 1:, 3:7]
    v = states[..., 1:, 7:10]
    p_g, v_g, q_g = (f64(x) for x in goal)
    out = {}
    if p_traj is not None:
        out["track"] = f64(prm["Q_track"]) * np.linalg.norm(p - p_traj, axis=-1).sum(-1)
    out["vnorm"] = f64(prm["Q_vnorm"]) * (v * v).sum(-1).sum(-1)
    u = np.asarray(u, np.float64)
    N = u.shape[-2]
    ctrl = f64(prm["Q_c"]) * (u[..., 0:N - 1, :] ** 2).sum(-1).sum(-1)
    du = u[..., 1:N - 1, :] - u[..., 0:N - 2, :]
    ctrl = ctrl + f64(prm["Q_cdelta"]) * (du * du).sum(-1).sum(-1)
    out["ctrl"] = ctrl
    goal_t = (f64(prm["Q_p"]) * np.linalg.norm(p - p_g, axis=-1)
              + f64(prm["Q_v"]) * np.linalg.norm(v - v_g, axis=-1)
              + f64(prm["Q_q"]) * attitude_error(q, q_g))
    out["goal"] = goal_t.sum(-1)
    out["col"] = collision_penalty(d, f64(prm["C"]), f64(prm["a"]), f64(prm["d_min"]),
                                   f64(prm["d_max"])).sum(-1)
    return out


def weighted_sum(terms, w, names=TERMS):
    w = f64(w)
    total = 0.0
    for i, name in enumerate(TERMS):
        if name in names and name in terms:
            total = total + w[i] * terms[name]
    return total
