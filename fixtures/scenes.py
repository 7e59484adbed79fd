"""Obstacle scenes and a simulated spinning LiDAR.

The scenes follow the statistics the paper gives for its simulated
environments (Sec. V-B: forests of trunks, "Verticals" of 6 m cylinders
with radii 0.4-1.1 m, "Inclines" of 10 m cylinders tilted 0-30 deg with
radii 0.06-0.3 m; the real-world "Wall" scene for the wall box).  The
LiDAR casts rays from a sensor origin and returns the first hit along each
beam, with Gaussian range noise, expressed in the sensor-centred frame
(world axes, origin at the sensor).
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Cylinder:
    """Finite cylinders: base point, unit axis, radius, length (arrays)."""
    base: np.ndarray    # (n, 3)
    axis: np.ndarray    # (n, 3) unit
    radius: np.ndarray  # (n,)
    length: np.ndarray  # (n,)

    def __len__(self):
        return len(self.radius)


@dataclass
class Box:
    lo: np.ndarray  # (n, 3)
    hi: np.ndarray  # (n, 3)

    def __len__(self):
        return len(self.lo)


def _empty_boxes():
    return Box(np.zeros((0, 3)), np.zeros((0, 3)))


def forest_scene(rng, half=32.0, density=0.15, r_lo=0.15, r_hi=0.4,
                 z_lo=-8.0, z_hi=12.0, keep_out=1.0, sensor_xy=(0.0, 0.0)):
    """Vertical trunks with Poisson-distributed centres over a square."""
    area = (2 * half) ** 2
    n = rng.poisson(density * area)
    cx = rng.uniform(-half, half, n)
    cy = rng.uniform(-half, half, n)
    r = rng.uniform(r_lo, r_hi, n)
    d = np.hypot(cx - sensor_xy[0], cy - sensor_xy[1])
    keep = d > r + keep_out
    cx, cy, r = cx[keep], cy[keep], r[keep]
    n = len(r)
    base = np.stack([cx, cy, np.full(n, z_lo)], 1)
    axis = np.tile([0.0, 0.0, 1.0], (n, 1))
    return Cylinder(base, axis, r, np.full(n, z_hi - z_lo)), _empty_boxes()


def verticals_scene(rng, half=32.0, density=0.625, r_lo=0.4, r_hi=1.1,
                    height=6.0, z_ground=-1.5, keep_out=1.0, wall=True):
    """Dense 6 m cylinders plus an optional wall box 8 m ahead (+x)."""
    area = (2 * half) ** 2
    n = rng.poisson(density * area)
    cx = rng.uniform(-half, half, n)
    cy = rng.uniform(-half, half, n)
    r = rng.uniform(r_lo, r_hi, n)
    keep = np.hypot(cx, cy) > r + keep_out
    if wall:
        # keep the wall face itself unobstructed in front of the sensor
        keep &= ~((cx > 2.0) & (cx < 8.0) & (np.abs(cy) < 3.0 + r))
    cx, cy, r = cx[keep], cy[keep], r[keep]
    n = len(r)
    base = np.stack([cx, cy, np.full(n, z_ground)], 1)
    axis = np.tile([0.0, 0.0, 1.0], (n, 1))
    cyl = Cylinder(base, axis, r, np.full(n, height))
    if wall:
        boxes = Box(np.array([[8.0, -3.0, z_ground]]),
                    np.array([[8.5, 3.0, z_ground + 6.0]]))
    else:
        boxes = _empty_boxes()
    return cyl, boxes


def incline_scene(rng, x_lo=-32.0, x_hi=32.0, y_lo=-32.0, y_hi=32.0,
                  density=0.5, r_lo=0.06, r_hi=0.3, length=10.0,
                  tilt_max_deg=30.0, z_ground=-2.0, keep_out=1.0,
                  keep_out_points=((0.0, 0.0, 0.0),)):
    """Tilted thin cylinders; tilt uniform in [0, 30 deg], random heading."""
    area = (x_hi - x_lo) * (y_hi - y_lo)
    n = rng.poisson(density * area)
    cx = rng.uniform(x_lo, x_hi, n)
    cy = rng.uniform(y_lo, y_hi, n)
    r = rng.uniform(r_lo, r_hi, n)
    tilt = np.deg2rad(rng.uniform(0.0, tilt_max_deg, n))
    head = rng.uniform(-np.pi, np.pi, n)
    axis = np.stack([np.sin(tilt) * np.cos(head), np.sin(tilt) * np.sin(head),
                     np.cos(tilt)], 1)
    base = np.stack([cx, cy, np.full(n, z_ground)], 1)
    keep = np.ones(n, bool)
    for kp in keep_out_points:
        kp = np.asarray(kp, float)
        keep &= _segment_point_distance(base, axis, np.full(n, length), kp) > r + keep_out
    cyl = Cylinder(base[keep], axis[keep], r[keep], np.full(int(keep.sum()), length))
    return cyl, _empty_boxes()


def _segment_point_distance(base, axis, length, p):
    w = p[None, :] - base
    s = np.clip((w * axis).sum(1), 0.0, length)
    closest = base + s[:, None] * axis
    return np.linalg.norm(p[None, :] - closest, axis=1)


def _ray_cylinders(dirs, origin, cyl, tmax):
    """First-hit distance along unit rays `dirs` (B,3) from `origin`."""
    B = len(dirs)
    best = np.full(B, np.inf)
    if len(cyl) == 0 or B == 0:
        return best
    w = origin[None, :] - cyl.base                          # (C,3)
    wa = (w * cyl.axis).sum(1)                              # (C,)
    wp = w - wa[:, None] * cyl.axis                          # (C,3)
    cpar = (wp * wp).sum(1) - cyl.radius ** 2               # (C,)
    for s in range(0, B, 2048):
        d = dirs[s:s + 2048]                                 # (b,3)
        da = d @ cyl.axis.T                                  # (b,C)
        # d_perp = d - da*axis ; A = |d_perp|^2 = 1 - da^2
        A = 1.0 - da * da
        Bq = 2.0 * (d @ wp.T)                                # d_perp . w_perp = d . w_perp
        disc = Bq * Bq - 4.0 * A * cpar[None, :]
        ok = (disc >= 0.0) & (A > 1e-12)
        sq = np.sqrt(np.where(ok, disc, 0.0))
        t1 = (-Bq - sq) / np.where(ok, 2.0 * A, 1.0)
        h = wa[None, :] + t1 * da
        hit = ok & (t1 > 0.0) & (h >= 0.0) & (h <= cyl.length[None, :])
        t = np.where(hit, t1, np.inf)
        best[s:s + 2048] = t.min(1)
    return best


def _ray_boxes(dirs, origin, boxes):
    B = len(dirs)
    best = np.full(B, np.inf)
    for lo, hi in zip(boxes.lo, boxes.hi):
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / dirs
            t0 = (lo[None, :] - origin[None, :]) * inv
            t1 = (hi[None, :] - origin[None, :]) * inv
        tn = np.nanmax(np.minimum(t0, t1), 1)
        tf = np.nanmin(np.maximum(t0, t1), 1)
        hit = (tf >= tn) & (tn > 0.0)
        best = np.minimum(best, np.where(hit, tn, np.inf))
    return best


def lidar_sweep(rng, cyl, boxes, origin, n_az, el_deg, max_range, noise_std,
                az_jitter=0.0):
    """Cast n_az x len(el_deg) beams; return hits in the sensor frame.

    Azimuth beams are evenly spaced over [-180, 180) deg (optionally
    jittered), elevations are given in degrees.  Each returned point is
    (range + N(0, noise_std^2)) * beam direction, float64 (n, 3), in beam
    order (azimuth-major).
    """
    origin = np.asarray(origin, float)
    az = -np.pi + 2.0 * np.pi * (np.arange(n_az) + 0.5) / n_az
    if az_jitter:
        az = az + rng.uniform(-az_jitter, az_jitter, n_az)
    el = np.deg2rad(np.asarray(el_deg, float))
    ce, se = np.cos(el), np.sin(el)
    dirs = np.stack([np.outer(np.cos(az), ce).ravel(),
                     np.outer(np.sin(az), ce).ravel(),
                     np.tile(se, n_az)], 1)
    # Cull cylinders per azimuth sector using a bounding circle in xy.
    rng_t = np.full(len(dirs), np.inf)
    if len(cyl):
        mid = cyl.base + 0.5 * cyl.length[:, None] * cyl.axis
        half_xy = 0.5 * cyl.length * np.hypot(cyl.axis[:, 0], cyl.axis[:, 1])
        rad = half_xy + cyl.radius + 1e-3
        rel = mid[:, :2] - origin[None, :2]
        dist = np.hypot(rel[:, 0], rel[:, 1])
        ang = np.arctan2(rel[:, 1], rel[:, 0])
        near = dist <= rad
        half_w = np.where(near, np.pi, np.arcsin(np.clip(rad / np.maximum(dist, 1e-9), 0, 1)))
        reach = dist - rad <= max_range
        n_sec = 64
        sec_w = 2.0 * np.pi / n_sec
        beam_sec = np.clip(((np.repeat(az, len(el)) + np.pi) // sec_w).astype(int), 0, n_sec - 1)
        for s in range(n_sec):
            lo = -np.pi + s * sec_w
            hi = lo + sec_w
            c = 0.5 * (lo + hi)
            dang = np.abs((ang - c + np.pi) % (2 * np.pi) - np.pi)
            sel = reach & (near | (dang <= half_w + 0.5 * sec_w + 2.0 * az_jitter + 1e-3))
            bsel = np.nonzero(beam_sec == s)[0]
            if len(bsel) == 0 or not sel.any():
                continue
            sub = Cylinder(cyl.base[sel], cyl.axis[sel], cyl.radius[sel], cyl.length[sel])
            rng_t[bsel] = _ray_cylinders(dirs[bsel], origin, sub, max_range)
    if len(boxes):
        rng_t = np.minimum(rng_t, _ray_boxes(dirs, origin, boxes))
    hit = rng_t <= max_range
    r = rng_t[hit] + rng.normal(0.0, noise_std, int(hit.sum()))
    return r[:, None] * dirs[hit]


def cylinders_surface_points(rng, cyl, n, max_norm, center=(0.0, 0.0, 0.0)):
    """Points uniform on the lateral surfaces (area-weighted), |p| <= max_norm."""
    center = np.asarray(center, float)
    area = 2 * np.pi * cyl.radius * cyl.length
    prob = area / area.sum()
    out = []
    have = 0
    while have < n:
        m = 2 * (n - have) + 64
        ci = rng.choice(len(cyl), size=m, p=prob)
        th = rng.uniform(-np.pi, np.pi, m)
        h = rng.uniform(0.0, 1.0, m) * cyl.length[ci]
        a = cyl.axis[ci]
        # orthonormal frame around the axis
        ref = np.where(np.abs(a[:, 2:3]) < 0.9, [[0.0, 0.0, 1.0]], [[1.0, 0.0, 0.0]])
        e1 = np.cross(a, ref)
        e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
        e2 = np.cross(a, e1)
        p = (cyl.base[ci] + h[:, None] * a
             + cyl.radius[ci, None] * (np.cos(th)[:, None] * e1 + np.sin(th)[:, None] * e2))
        p = p - center[None, :]
        p = p[np.linalg.norm(p, axis=1) <= max_norm]
        out.append(p)
        have += len(p)
    return np.concatenate(out)[:n]


def _axis_angle_matrix(q):
    """Rotation of a unit quaternion via its axis and angle (Rodrigues' formula)."""
    q = np.asarray(q, float)
    q = q / np.linalg.norm(q)
    s = np.linalg.norm(q[1:])
    if s == 0.0:
        return np.eye(3)
    ang = 2.0 * np.arctan2(s, q[0])
    k = q[1:] / s
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + np.sin(ang) * K + (1.0 - np.cos(ang)) * (K @ K)


def record_frame(rng, cyl, boxes, x, n_az, el_deg, max_range, noise_std):
    """One LiDAR frame recorded by a vehicle in state x = (p, q, v): the hits of a
    sweep from p (beams spread in world azimuth/elevation), expressed in the body
    axes of attitude q.  Returns (points float32 (n, 3), pose float32 (7,) = (p, q))."""
    x = np.asarray(x, float)
    p, q = x[0:3], x[3:7]
    hits = lidar_sweep(rng, cyl, boxes, p, n_az, el_deg, max_range, noise_std)
    body = hits @ _axis_angle_matrix(q)       # R^T h for every row h
    return body.astype(np.float32), np.concatenate([p, q]).astype(np.float32)
