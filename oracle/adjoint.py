"""Gradient of the summed Stage-I cost, L = scale * sum_{m,k} S1[m,k], with
respect to the nominal controls u_nom[m, t, c] and the five term weights.

The cost is piecewise smooth (control clipping, the three collision branches,
the nearest-point switch).  The derivative computed here is the exact one of the
active smooth piece: the clip mask, the collision branch of every (m, k, t) and
the nearest cloud point o* (lowest index on ties) are frozen at the evaluation
point.  The forward model is the same definition as `oracle.mppi` (Sec. III-A
eq. (dynamics), RK4 of eq. (mppi_rollout), the Stage-I terms of Sec. IV-C),
written a second time in PyTorch float64 so that autograd supplies the
derivative; `fd_directional` / `fd_grad_w` give central finite differences of the same frozen
function for an independent check.
"""
import numpy as np
import torch

from . import philox
from .cost import f64, nearest
from .dynamics import rollout
from .guides import guide_positions
from .mppi import perturb

T = torch.float64


def active_set(prob, coef, u_nom=None, normals=None, nearest_fn=nearest, nearest_idx=None):
    """Clip mask, nearest points and collision branches at the evaluation point.

    `nearest_idx` (M, K, N) int, when given, replaces the oracle's own nearest
    search (to evaluate on another implementation's active set)."""
    prm = prob["params"]
    M, K, N = prob["M"], prob["K"], prob["N"]
    u_nom = prob["u_nom"] if u_nom is None else u_nom
    if normals is None:
        normals = philox.normals(prm["seed"], prob["problem_id"], M, K, N, prm["iter_base"])
    raw = f64(u_nom)[:, None] + f64(prm["sigma"]) * np.asarray(normals, np.float64)
    lo, hi = f64(prm["u_min"]), f64(prm["u_max"])
    mask = (raw >= lo) & (raw <= hi)
    u, _ = perturb(u_nom, normals, prm)
    states = rollout(f64(prob["x0"]), u, f64(prm["dt"]), f64(prm["mass"]), f64(prm["gravity"]))
    pos = states[..., 1:, 0:3]
    cloud = np.asarray(prob["cloud"], np.float32).astype(np.float64).reshape(-1, 3)
    if nearest_idx is None:
        d, idx = nearest_fn(prob["cloud"], pos.reshape(-1, 3))
        d, idx = d.reshape(M, K, N), idx.reshape(M, K, N)
    else:
        idx = np.asarray(nearest_idx, np.int64)
    # an empty collision set has no nearest point: d = +inf (zero penalty)
    pad = np.concatenate([cloud, np.zeros((1, 3))])          # row -1 (= last) is a dummy
    o_star = np.where((idx >= 0)[..., None], pad[np.where(idx >= 0, idx, -1)], 0.0)
    if nearest_idx is not None:
        d = np.where(idx >= 0, np.linalg.norm(pos - o_star, axis=-1), np.inf)
    d_min, d_max = f64(prm["d_min"]), f64(prm["d_max"])
    branch = np.where(d < d_min, 0, np.where(d < d_max, 1, 2))
    return dict(mask=mask, clipped=u, normals=np.asarray(normals, np.float64), branch=branch,
                o_star=o_star, d=d, idx=idx)


def _quat_mul(a, b):
    aw, ax, ay, az = a.unbind(-1)
    bw, bx, by, bz = b.unbind(-1)
    return torch.stack([aw * bw - ax * bx - ay * by - az * bz,
                        aw * bx + ax * bw + ay * bz - az * by,
                        aw * by - ax * bz + ay * bw + az * bx,
                        aw * bz + ax * by - ay * bx + az * bw], -1)


def _rot(q):
    w, x, y, z = q.unbind(-1)
    r0 = torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1)
    r1 = torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1)
    r2 = torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)
    return torch.stack([r0, r1, r2], -2)


def _f(x, u, mass, g):
    v = x[..., 7:10]
    q = x[..., 3:7]
    om = torch.cat([torch.zeros_like(u[..., :1]), u[..., 1:4]], -1)
    dq = 0.5 * _quat_mul(q, om)
    thrust = torch.cat([torch.zeros_like(u[..., :2]), u[..., :1]], -1)
    dv = torch.einsum("...ij,...j->...i", _rot(q), thrust) / mass
    dv = dv - torch.tensor([0.0, 0.0, g], dtype=T)
    return torch.cat([v, dq, dv], -1)


def _rk4(x, u, dt, mass, g):
    k1 = _f(x, u, mass, g)
    k2 = _f(x + 0.5 * dt * k1, u, mass, g)
    k3 = _f(x + 0.5 * dt * k2, u, mass, g)
    k4 = _f(x + dt * k3, u, mass, g)
    xn = x + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    q = xn[..., 3:7]
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    return torch.cat([xn[..., 0:3], q, xn[..., 7:10]], -1)


def _norm(v):
    """|v| with a zero subgradient at v = 0."""
    n2 = (v * v).sum(-1)
    safe = torch.where(n2 > 0, n2, torch.ones_like(n2))
    return torch.where(n2 > 0, torch.sqrt(safe), torch.zeros_like(n2))


def frozen_terms(prob, coef, u_nom, act):
    """Unweighted J terms (M, K) of the frozen piece; u_nom is a torch tensor."""
    prm = prob["params"]
    M, K, N = prob["M"], prob["K"], prob["N"]
    sc = lambda key: float(f64(prm[key]))  # noqa: E731  (float32 parameter as a float)
    sig = torch.tensor(f64(prm["sigma"]), dtype=T)
    n = torch.tensor(act["normals"], dtype=T)
    mask = torch.tensor(act["mask"])
    clipped = torch.tensor(act["clipped"], dtype=T)
    u = torch.where(mask, u_nom[:, None] + sig * n, clipped)           # (M,K,N,4)
    dt, mass, g = sc("dt"), sc("mass"), sc("gravity")
    x = torch.tensor(f64(prob["x0"]), dtype=T).expand(M, K, 10)
    xs = []
    for j in range(N):
        x = _rk4(x, u[:, :, j], dt, mass, g)
        xs.append(x)
    X = torch.stack(xs, 2)                                             # (M,K,N,10)
    p, q, v = X[..., 0:3], X[..., 3:7], X[..., 7:10]
    ptraj = torch.tensor(guide_positions(np.asarray(coef, np.float64), N, prm["dt"]), dtype=T)
    pg = torch.tensor(f64(prob["p_goal"]), dtype=T)
    vg = torch.tensor(f64(prob["v_goal"]), dtype=T)
    Rg = _rot(torch.tensor(f64(prob["q_goal"]), dtype=T))
    J = {}
    J["track"] = sc("Q_track") * _norm(p - ptraj[:, None]).sum(-1)
    J["vnorm"] = sc("Q_vnorm") * (v * v).sum(-1).sum(-1)
    J["ctrl"] = (sc("Q_c") * (u[:, :, 0:N - 1] ** 2).sum(-1).sum(-1)
                 + sc("Q_cdelta") * ((u[:, :, 1:N - 1] - u[:, :, 0:N - 2]) ** 2).sum(-1).sum(-1))
    E = _rot(q) @ Rg.transpose(-1, -2) - torch.eye(3, dtype=T)
    att = _norm(E.reshape(E.shape[:-2] + (9,)))
    J["goal"] = (sc("Q_p") * _norm(p - pg) + sc("Q_v") * _norm(v - vg)
                 + sc("Q_q") * att).sum(-1)
    C, a, dmin = sc("C"), sc("a"), sc("d_min")
    d = _norm(p - torch.tensor(act["o_star"], dtype=T))
    br = torch.tensor(act["branch"])
    phi = torch.where(br == 0, torch.full_like(d, C),
                      torch.where(br == 1, C * torch.exp(-a * (d - dmin)), torch.zeros_like(d)))
    J["col"] = phi.sum(-1)
    return J


TERMS = ("track", "vnorm", "ctrl", "goal", "col")


def loss(prob, coef, u_nom, w, act, scale=1.0):
    J = frozen_terms(prob, coef, u_nom, act)
    return scale * sum(w[i] * J[name].sum() for i, name in enumerate(TERMS))


def grad(prob, coef, act, u_nom=None, scale=1.0):
    """(dL/du_nom (M,N,4), dL/dw (5,), L) by autograd on the frozen piece."""
    u0 = prob["u_nom"] if u_nom is None else u_nom
    u = torch.tensor(f64(u0), dtype=T, requires_grad=True)
    w = torch.tensor(f64(prob["params"]["w"]), dtype=T, requires_grad=True)
    L = loss(prob, coef, u, w, act, scale)
    gu, gw = torch.autograd.grad(L, [u, w])
    return gu.numpy(), gw.numpy(), float(L.detach())


def fd_directional(prob, coef, act, direction, h=1e-4, u_nom=None, scale=1.0):
    """Central difference of the frozen L along `direction` (M, N, 4)."""
    u0 = f64(prob["u_nom"] if u_nom is None else u_nom)
    w = torch.tensor(f64(prob["params"]["w"]), dtype=T)
    dirn = np.asarray(direction, np.float64)
    with torch.no_grad():
        lp = loss(prob, coef, torch.tensor(u0 + h * dirn, dtype=T), w, act, scale)
        lm = loss(prob, coef, torch.tensor(u0 - h * dirn, dtype=T), w, act, scale)
    return float(lp - lm) / (2.0 * h)


def fd_grad_w(prob, coef, act, h=1e-4, scale=1.0):
    u0 = torch.tensor(f64(prob["u_nom"]), dtype=T)
    w0 = f64(prob["params"]["w"])
    out = np.zeros(5)
    with torch.no_grad():
        for i in range(5):
            e = np.zeros(5)
            e[i] = h
            lp = loss(prob, coef, u0, torch.tensor(w0 + e, dtype=T), act, scale)
            lm = loss(prob, coef, u0, torch.tensor(w0 - e, dtype=T), act, scale)
            out[i] = float(lp - lm) / (2 * h)
    return out
