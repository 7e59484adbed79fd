"""Quadrotor model, Sec. III-A eq. (dynamics), and its RK4 discretisation,
Sec. III-B eq. (mppi_rollout).

State x = [p (3), q (4, Hamilton, scalar first, body -> world), v (3)],
input u = (F_t, omega) with omega in the body frame.

  p' = v
  q' = 1/2 q (x) [0, omega]
  v' = (1/m) R(q) [0, 0, F_t]^T + g,   g = (0, 0, -gravity)

Readings: R(q) is the unit-quaternion rotation matrix evaluated on the
raw (unnormalised) RK4 stage quaternion; the quaternion is renormalised
after every full RK4 step; the control is held constant over a step.
"""
import numpy as np


def quat_mul(a, b):
    """Hamilton product a (x) b for (..., 4) arrays, scalar first."""
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], -1)


def rotation_matrix(q):
    """R(q) (..., 3, 3) of a unit quaternion (..., 4)."""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def f(x, u, mass, gravity):
    """Continuous-time right-hand side for (..., 10) states, (..., 4) inputs."""
    v = x[..., 7:10]
    q = x[..., 3:7]
    omega = np.concatenate([np.zeros(u.shape[:-1] + (1,)), u[..., 1:4]], -1)
    dq = 0.5 * quat_mul(q, omega)
    thrust = np.zeros(u.shape[:-1] + (3,))
    thrust[..., 2] = u[..., 0]
    dv = np.einsum("...ij,...j->...i", rotation_matrix(q), thrust) / mass
    dv[..., 2] -= gravity
    return np.concatenate([v, dq, dv], -1)


def rk4_step(x, u, dt, mass, gravity):
    k1 = f(x, u, mass, gravity)
    k2 = f(x + 0.5 * dt * k1, u, mass, gravity)
    k3 = f(x + 0.5 * dt * k2, u, mass, gravity)
    k4 = f(x + dt * k3, u, mass, gravity)
    xn = x + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    q = xn[..., 3:7]
    xn[..., 3:7] = q / np.linalg.norm(q, axis=-1, keepdims=True)
    return xn


def rollout(x0, u, dt, mass, gravity):
    """x_{j+1} = x_j + f_RK4(x_j, u_j, dt), j = 0..N-1.

    x0 (10,) or (..., 10); u (..., N, 4).  Returns states (..., N+1, 10).
    """
    u = np.asarray(u, np.float64)
    N = u.shape[-2]
    x = np.broadcast_to(np.asarray(x0, np.float64), u.shape[:-2] + (10,)).copy()
    out = np.empty(u.shape[:-2] + (N + 1, 10))
    out[..., 0, :] = x
    for j in range(N):
        x = rk4_step(x, u[..., j, :], dt, mass, gravity)
        out[..., j + 1, :] = x
    return out
