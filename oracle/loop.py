"""Receding-horizon helpers of the closed-loop workload (test infrastructure only).

MPPI is executed in receding horizon (Sec. III-B): after each planning step the
selected sequence, advanced by one step with its last control held, seeds the
next step.  The closed-loop workload also refines the selected sequence once by
a gradient step on its Stage-II cost, choosing the step length among a few
candidates by that same cost.
"""
import numpy as np

from .cost import f64


def shift_controls(src, index, shift, M_dst):
    """dst[m][t] = src[index][min(t + shift, N - 1)] for m < M_dst."""
    src = f64(src)
    M, N = src.shape[0], src.shape[1]
    sel = min(max(int(index), 0), M - 1)
    t = np.minimum(np.arange(N) + int(shift), N - 1)
    return np.broadcast_to(src[sel][t], (M_dst, N, 4)).copy()


def step_candidates(u, g, s0, beta, n, u_min, u_max):
    """out[0] = u; out[i] = clip(u - s0 beta^(i-1) g / max|g|), i = 1..n-1."""
    u, g = f64(u), f64(g)
    gmax = np.abs(g).max()
    out = np.empty((n,) + u.shape)
    out[0] = u
    for i in range(1, n):
        if gmax > 0:
            s = float(np.float32(s0)) * float(np.float32(beta)) ** (i - 1)
            out[i] = np.clip(u - s * g / gmax, f64(u_min), f64(u_max))
        else:
            out[i] = u
    return out
