"""Seeded planning problems for the five benchmark workloads.

Each builder returns plain dicts of NumPy arrays (float32 where the planner
sees float32) so that the HIP path and the CPU oracle read identical inputs.
Fixture randomness is NumPy PCG64 seeded with the workload number; the
planner's own sampling noise is drawn inside each implementation from the
counter-based generator keyed by `seed`/`problem_id`/`iter_base`.
"""
import functools
import math

import numpy as np

from .scenes import (Cylinder, _empty_boxes, cylinders_surface_points,
                     forest_scene, incline_scene, lidar_sweep, verticals_scene)

GRAVITY = 9.81


def table1_params(sigma=(1.0, 1.0, 1.0, math.sqrt(0.5)), dt=0.05, lam=0.1):
    """Parameter values of Table I (mass, limits, weights, collision shape).

    `sigma` is the per-channel standard deviation of the control noise in
    the order (thrust, omega_x, omega_y, omega_z).  Table I lists
    Sigma = (1.0, 1.0, 0.5); the default reads those as variances.
    """
    return dict(
        dt=float(dt), lam=float(lam), mass=1.0, gravity=GRAVITY,
        sigma=np.asarray(sigma, np.float32),
        u_min=np.asarray([0.3, -3.0, -3.0, -2.0], np.float32),
        u_max=np.asarray([16.35, 3.0, 3.0, 2.0], np.float32),
        Q_track=15.0, Q_vnorm=0.15, Q_c=0.5, Q_cdelta=0.5,
        Q_p=3.0, Q_v=0.25, Q_q=1.0,
        C=1.0e6, a=5.0, d_min=0.4, d_max=1.0,
        w=np.ones(5, np.float32),
        seed=0, iter_base=0,
    )


def split_instances(M):
    """(M_h, M_v): M_v is the largest divisor of M not above min(3, sqrt M)."""
    best = 1
    for mv in range(1, M + 1):
        if M % mv == 0 and mv <= min(3.0, math.sqrt(M)):
            best = mv
    return M // best, best


def hover_controls(M, N, mass=1.0, gravity=GRAVITY):
    u = np.zeros((M, N, 4), np.float32)
    u[..., 0] = np.float32(mass * gravity)
    return u


def _state(p=(0.0, 0.0, 0.0), v=(0.0, 0.0, 0.0), q=(1.0, 0.0, 0.0, 0.0)):
    return np.asarray(list(p) + list(q) + list(v), np.float32)


def _problem(cloud, M, K, N, params, p_goal, x0=None, partition=None,
             problem_id=0, name=""):
    x0 = _state() if x0 is None else np.asarray(x0, np.float32)
    M_h, M_v = split_instances(M)
    part = dict(n_az_c=32, n_el_c=8, f_a=4, f_e=4, r_max=30.0, ell=5.0)
    if partition:
        part.update(partition)
    p_goal = np.asarray(p_goal, np.float32)
    return dict(
        name=name,
        cloud=np.ascontiguousarray(cloud, np.float32).reshape(-1, 3),
        x0=x0, p_goal=p_goal,
        v_goal=np.zeros(3, np.float32),
        q_goal=np.asarray([1.0, 0.0, 0.0, 0.0], np.float32),
        goal_dir=(p_goal - x0[:3]).astype(np.float32),
        M=int(M), K=int(K), N=int(N), M_h=M_h, M_v=M_v,
        partition=part, params=params,
        u_nom=hover_controls(M, N, params["mass"], params["gravity"]),
        problem_id=int(problem_id),
    )


def make_plain_problem(seed=1):
    """Single MPPI instance over 40 vertical cylinders (5,000 surface points).

    K=256, N=20, dt=0.05, sigma=(1.0, 0.5, 0.5, 0.5); start at rest at the
    origin, goal (18, 0, 1.5); one rest-to-rest straight-line guide.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    start, goal = np.array([0.0, 0.0]), np.array([18.0, 0.0])
    cx, cy, r = [], [], []
    while len(r) < 40:
        x, y, rr = rng.uniform(0, 20), rng.uniform(-10, 10), rng.uniform(0.2, 0.5)
        if np.hypot(x - start[0], y - start[1]) <= rr + 0.5:
            continue
        if np.hypot(x - goal[0], y - goal[1]) <= rr + 0.5:
            continue
        cx.append(x), cy.append(y), r.append(rr)
    n = 40
    cyl = Cylinder(np.stack([cx, cy, np.full(n, -2.0)], 1),
                   np.tile([0.0, 0.0, 1.0], (n, 1)), np.asarray(r), np.full(n, 8.0))
    cloud = cylinders_surface_points(rng, cyl, 5000, 20.0)
    params = table1_params(sigma=(1.0, 0.5, 0.5, 0.5))
    prob = _problem(cloud, 1, 256, 20, params, (18.0, 0.0, 1.5),
                    name="plain-cylinders-5k")
    g = prob["goal_dir"].astype(np.float64)
    prob["anchors"] = (prob["x0"][:3] + 5.0 * g / np.linalg.norm(g)).astype(np.float32)[None, :]
    return prob


def _subsample(rng, pts, n):
    idx = np.sort(rng.choice(len(pts), size=n, replace=False))
    return pts[idx]


def make_ensemble_problem(seed=2, n_points=50000, K=1024, N=40, M=8):
    """One planning step of the anchor-guided ensemble in a forest.

    Trunks at 0.15 per m^2 over [-32, 32]^2, radii U[0.15, 0.4], sensor at
    (0, 0, 1.5); 1,800 x 32 beams (0.2 deg azimuth, elevation -15..15 deg),
    30 m range, 2 cm range noise, subsampled to exactly `n_points`.
    Partition 32 x 8 coarse cells refined 4 x 4, r_max = 30 m; M = 8
    instances (4 x 2), K = 1024, N = 40, dt = 0.05; goal (18, 0, 0).
    """
    s = seed
    while True:
        rng = np.random.Generator(np.random.PCG64(s))
        cyl, boxes = forest_scene(rng)
        pts = lidar_sweep(rng, cyl, boxes, (0.0, 0.0, 1.5), 1800,
                          np.linspace(-15.0, 15.0, 32), 30.0, 0.02)
        if len(pts) >= n_points:
            break
        s += 1000
    cloud = _subsample(rng, pts, n_points)
    return _problem(cloud, M, K, N, table1_params(), (18.0, 0.0, 0.0),
                    name=f"ensemble-forest-{n_points // 1000}k")


def make_paper_point_problem(seed=6, n_points=200000, K=128, N=25, M=15):
    """The paper's own operating point (Sec. IV-A, Sec. V-A, Table I).

    An accumulated LiDAR cloud of 200,000 points within r_max = 10 m (Livox-like
    vertical field of view -7..52 deg) in a dense "Verticals" scene (0.625 per m^2,
    radii 0.4-1.1 m, 6 m tall); 3 deg partition, 120 x 60 fine cells pooled 6 x 6
    into 20 x 10 coarse cells; M = 15 (5 x 3) instances, K = 128, N = 25,
    dt = 0.05; the collision set is the filtered cloud P_f.
    """
    s = seed
    n_az = 4000
    while True:
        rng = np.random.Generator(np.random.PCG64(s))
        cyl, boxes = verticals_scene(rng, half=16.0, wall=False)
        pts = lidar_sweep(rng, cyl, boxes, (0.0, 0.0, 1.5), n_az,
                          np.linspace(-7.0, 52.0, 96), 10.0, 0.02)
        if len(pts) >= n_points:
            break
        n_az = int(n_az * 1.5)
    cloud = _subsample(rng, pts, n_points)
    prob = _problem(cloud, M, K, N, table1_params(), (18.0, 0.0, 0.0),
                    partition=dict(n_az_c=20, n_el_c=10, f_a=6, f_e=6, r_max=10.0, ell=5.0),
                    name=f"paper-point-verticals-{n_points // 1000}k")
    prob["collision"] = "filtered"
    return prob


@functools.lru_cache(maxsize=4)
def _batched_cached(seed, n_problems):
    rng = np.random.Generator(np.random.PCG64(seed))
    probs = []
    for b in range(n_problems):
        kind = int(rng.integers(0, 3))
        P = int(np.clip(round(rng.lognormal(math.log(5.0e4), 0.5)), 10000, 200000))
        M = int(rng.integers(4, 17))
        K = int(rng.choice([512, 1024, 2048, 4096]))
        N = int(rng.choice([30, 40, 60]))
        srng = np.random.Generator(np.random.PCG64(seed * 1000 + b))
        if kind == 0:
            cyl, boxes = forest_scene(srng)
            name = "forest"
        elif kind == 1:
            cyl, boxes = verticals_scene(srng)
            name = "verticals"
        else:
            cyl, boxes = incline_scene(srng)
            name = "incline"
        n_el = 64
        n_az = max(1800, int(math.ceil(1.6 * P / n_el)))
        while True:
            pts = lidar_sweep(srng, cyl, boxes, (0.0, 0.0, 1.5), n_az,
                              np.linspace(-15.0, 15.0, n_el), 30.0, 0.02)
            if len(pts) >= P:
                break
            n_az *= 2
        cloud = _subsample(srng, pts, P)
        goal_az = srng.uniform(-0.6, 0.6)
        goal = (18.0 * math.cos(goal_az), 18.0 * math.sin(goal_az), srng.uniform(-1.0, 1.0))
        probs.append(_problem(cloud, M, K, N, table1_params(), goal,
                              problem_id=b, name=f"{name}-{P}"))
    return probs


def make_batched_problems(seed=3, n_problems=64):
    """64 uneven problems over forest / verticals+wall / incline scenes.

    Cloud size round(LogNormal(ln 5e4, 0.5)) clipped to [1e4, 2e5];
    M ~ U{4..16}, K ~ U{512, 1024, 2048, 4096}, N ~ U{30, 40, 60}.
    """
    return [dict(p) for p in _batched_cached(seed, n_problems)]


def make_loop_step(step, seed=5, n_points=1_000_000):
    """One replayed pose of the closed-loop incline flight.

    Pose p_s = (0.28 s, 0, 2.0), v = (7, 0, 0), q = identity; the cloud is
    sweeps of 1024 x 128 beams (el +-15 deg, 40 m, 2 cm noise) with azimuth
    jitter, accumulated until there are `n_points` hits (8 sweeps nominally)
    and truncated to exactly that; M = 16 (8 x 2), K = 8192,
    N = 60, dt = 0.04.  Expressed in the drone-centred frame.
    """
    scene = _loop_scene(seed)
    rng = np.random.Generator(np.random.PCG64(seed * 100000 + step))
    pose = np.array([0.28 * step, 0.0, 2.0])
    chunks, have = [], 0
    for _ in range(16):
        pts = lidar_sweep(rng, scene, _empty_boxes(), pose, 1024,
                          np.linspace(-15.0, 15.0, 128), 40.0, 0.02,
                          az_jitter=math.pi / 1024)
        chunks.append(pts)
        have += len(pts)
        if have >= n_points:
            break
    cloud = np.concatenate(chunks)[:n_points]
    x0 = _state(v=(7.0, 0.0, 0.0))
    goal = (80.0 - pose[0], 0.0, 0.0)
    return _problem(cloud, 16, 8192, 60, table1_params(dt=0.04), goal, x0=x0,
                    problem_id=0, name=f"loop-incline-step{step}")


@functools.lru_cache(maxsize=1)
def _loop_scene(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    cyl, _ = incline_scene(rng, x_lo=-10.0, x_hi=80.0, y_lo=-15.0, y_hi=15.0,
                           keep_out_points=[(0.28 * s, 0.0, 2.0) for s in range(0, 200, 5)])
    return cyl
