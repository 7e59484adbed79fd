"""Cloud accumulation and the vehicle step of a closed loop (test infrastructure
only: tests, the smoke check and the benchmark's CPU baseline use it; the
product path never does).

The planner's cloud is several recent LiDAR frames (Sec. IV-A accumulates
scans), each recorded in the sensor frame at its own pose and brought into the
drone-centred frame with world axes in which the partition is read (origin at
the current position).  Between planning steps the vehicle follows the model of
Sec. III-A for one control period under the first control of the executed plan,
integrated with the RK4 step of Sec. III-B.
"""
import numpy as np

from .cost import f64
from .dynamics import rk4_step, rotation_matrix


def to_local(frames, frame_start, frame_offsets, poses, origin):
    """Frame f holds n_f = offsets[f+1] - offsets[f] points starting at row
    frame_start[f] of `frames`, in that frame's sensor coordinates; output rows
    offsets[f] .. offsets[f+1] are R(q_f/|q_f|) x + p_f - origin.

    frames (R, 3) float32; frame_start (F,) int; frame_offsets (F+1,) int;
    poses (F, 7) float32 rows (p_x, p_y, p_z, q_w, q_x, q_y, q_z), sensor to world;
    origin (3,).  Returns (offsets[F], 3) float64."""
    src = f64(frames).reshape(-1, 3)
    start = np.asarray(frame_start, np.int64)
    off = np.asarray(frame_offsets, np.int64)
    poses = f64(poses).reshape(-1, 7)
    o = f64(origin)
    out = np.empty((int(off[-1]), 3))
    for f in range(len(poses)):
        lo, hi = int(off[f]), int(off[f + 1])
        x = src[int(start[f]):int(start[f]) + (hi - lo)]
        q = poses[f, 3:7] / np.linalg.norm(poses[f, 3:7])
        R = rotation_matrix(q)
        out[lo:hi] = (x @ R.T + poses[f, 0:3]) - o
    return out


def advance_state(x0, u_plans, index, dt, mass, gravity):
    """x1 = RK4(x0, u_plans[i][0]) with i = index clamped to [0, M)."""
    u = f64(u_plans)
    i = min(max(int(index), 0), u.shape[0] - 1)
    return rk4_step(f64(x0), u[i, 0], f64(dt), f64(mass), f64(gravity))
