"""Multi-resolution partition and anchors (Sec. IV-A, Sec. IV-B-1/2).

Readings (the paper leaves these open):
  * Frame: the cloud is given relative to the drone with world axes
    (z up); azimuth is measured from +x, elevation from the xy-plane.
  * Grid: azimuth cells cover [-pi, pi) in n_az equal wedges, elevation
    cells cover [-pi/2, pi/2] in n_el equal bands (120 x 60 at 3 deg in the
    paper; any n_az x n_el here).
  * Binning is decided by exact predicates on the float32 boundary
    directions so that integer outputs are reproducible bit for bit: a
    point is in azimuth wedge i iff it lies on or counter-clockwise of
    boundary i and strictly clockwise of boundary i+1; it is in elevation
    band j for the highest j >= 1 whose lower boundary it lies on or
    above (band 0 otherwise).  All predicate arithmetic is IEEE binary64
    add/sub/mul on float32 operands (no fused multiply-add).
  * A cone with no point has r = r_max ("unobserved is free"); the
    nearest point of a cone is the lowest point index attaining the
    minimum; coarse argmax ties go to the lowest flat fine index
    c = j * n_az + i.
  * Anchors: the goal direction is binned with the same predicates; the
    M_h x M_v block of coarse cells is centred on the goal's coarse cell
    (wrapping in azimuth, clamped in elevation), m = o_v * M_h + o_h.
"""
import math

import numpy as np


def partition_tables(n_az, n_el):
    """Float32 direction tables for an n_az x n_el angular grid.

    Returns dict with
      az_bound (n_az, 2): (cos, sin) of theta_i = -pi + 2 pi i / n_az
      el_bound (n_el+1, 2): (cos, sin) of beta_j = -pi/2 + pi j / n_el
      az_centre (n_az, 2), el_centre (n_el, 2): the same at half steps.
    Angles are formed in binary64 and cos/sin taken with the C library
    (math module), then rounded to float32.
    """
    def cs(t):
        return (math.cos(t), math.sin(t))

    az_b = [cs(-math.pi + 2.0 * math.pi * i / n_az) for i in range(n_az)]
    az_c = [cs(-math.pi + 2.0 * math.pi * (i + 0.5) / n_az) for i in range(n_az)]
    el_b = [cs(-0.5 * math.pi + math.pi * j / n_el) for j in range(n_el + 1)]
    el_c = [cs(-0.5 * math.pi + math.pi * (j + 0.5) / n_el) for j in range(n_el)]
    f = lambda a: np.asarray(a, np.float64).astype(np.float32)
    return dict(az_bound=f(az_b), el_bound=f(el_b), az_centre=f(az_c), el_centre=f(el_c))


def cell_directions(tab):
    """Unit direction of every fine cell, eq. (unit direction).

    d_ij = [cos b_j cos a_i, cos b_j sin a_i, sin b_j] from the centre
    tables; returned float64 (n_el * n_az, 3) in flat order c = j*n_az + i.
    """
    ca, sa = tab["az_centre"][:, 0].astype(np.float64), tab["az_centre"][:, 1].astype(np.float64)
    cb, sb = tab["el_centre"][:, 0].astype(np.float64), tab["el_centre"][:, 1].astype(np.float64)
    d = np.stack([np.outer(cb, ca), np.outer(cb, sa), np.outer(sb, np.ones_like(ca))], -1)
    return d.reshape(-1, 3)


def azimuth_bin(x, y, tab):
    """Azimuth wedge of each (x, y) (float64 arrays of float32 values)."""
    c = tab["az_bound"][:, 0].astype(np.float64)
    s = tab["az_bound"][:, 1].astype(np.float64)
    cross = c[None, :] * y[:, None] - s[None, :] * x[:, None]
    ge = cross >= 0.0
    inside = ge & ~np.roll(ge, -1, axis=1)
    n_in = inside.sum(1)
    on_axis = (x == 0.0) & (y == 0.0)
    assert np.all((n_in == 1) | on_axis), "azimuth wedges must partition the plane"
    return np.where(on_axis, 0, np.argmax(inside, axis=1))


def elevation_at_or_above(x, y, z, cb, sb):
    """Predicate 'direction (x,y,z) is at or above elevation boundary (cb, sb)'.

    z / |p| >= sin(beta)  <=>  z cb >= sb sqrt(x^2+y^2), evaluated on
    squares with the sign cases split.  Broadcasts points against boundaries.
    """
    zc = z * cb
    A = zc * zc
    xs = x * sb
    ys = y * sb
    B = xs * xs + ys * ys
    up = z >= 0.0
    return np.where(sb >= 0.0, up & (A >= B), up | (A <= B))


def elevation_bin(x, y, z, tab, n_el):
    cb = tab["el_bound"][1:n_el, 0].astype(np.float64)[None, :]
    sb = tab["el_bound"][1:n_el, 1].astype(np.float64)[None, :]
    pred = elevation_at_or_above(x[:, None], y[:, None], z[:, None], cb, sb)
    if n_el == 1:
        return np.zeros(len(x), np.int64)
    highest = (n_el - 1) - np.argmax(pred[:, ::-1], axis=1)  # highest true j in 1..n_el-1
    return np.where(pred.any(1), highest, 0)


def bin_directions(v, tab, n_az, n_el):
    """Fine cell (i, j) of each row of v (float32 (n, 3))."""
    v = np.asarray(v, np.float32).reshape(-1, 3).astype(np.float64)
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    return azimuth_bin(x, y, tab), elevation_bin(x, y, z, tab, n_el)


def range_key(cloud):
    """r^2 = (x*x + y*y) + z*z in binary64 for float32 points."""
    p = np.asarray(cloud, np.float32).astype(np.float64)
    return (p[:, 0] * p[:, 0] + p[:, 1] * p[:, 1]) + p[:, 2] * p[:, 2]


def fine_partition(cloud, tab, n_az, n_el, r_max, chunk=65536):
    """Nearest range per cone, Sec. IV-A-1: r_ij = min |p_c| over the cone.

    Returns (fine_key float64 (n_el*n_az,), fine_idx int32): fine_key holds
    r^2 (r_max^2 for an empty cone) and fine_idx the lowest point index
    attaining it (-1 for an empty cone).  Points at the origin or beyond
    r_max are ignored.
    """
    cloud = np.asarray(cloud, np.float32).reshape(-1, 3)
    n_fine = n_az * n_el
    rmax2 = np.float64(np.float32(r_max)) * np.float64(np.float32(r_max))
    key = np.full(n_fine, rmax2)
    idx = np.full(n_fine, -1, np.int64)
    r2 = range_key(cloud)
    valid = (r2 > 0.0) & (r2 <= rmax2)
    cell = np.full(len(cloud), -1, np.int64)
    for s in range(0, len(cloud), chunk):
        i, j = bin_directions(cloud[s:s + chunk], tab, n_az, n_el)
        cell[s:s + chunk] = j * n_az + i
    vi = np.nonzero(valid)[0]
    np.minimum.at(key, cell[vi], r2[vi])
    match = vi[r2[vi] == key[cell[vi]]]           # increasing point index
    cells, first = np.unique(cell[match], return_index=True)
    idx[cells] = match[first]
    return key, idx.astype(np.int32)


def coarse_best(fine_key, n_az, n_el, f_a, f_e):
    """Coarse safe direction, eq. (safe-vector): argmax r_ij over Omega_IJ.

    Returns int32 (n_el//f_e * n_az//f_a,) flat fine index of the argmax for
    each coarse cell in flat order C = J * (n_az//f_a) + I.
    """
    n_az_c, n_el_c = n_az // f_a, n_el // f_e
    k = fine_key.reshape(n_el, n_az)
    out = np.empty(n_az_c * n_el_c, np.int32)
    for J in range(n_el_c):
        for I in range(n_az_c):
            block = k[J * f_e:(J + 1) * f_e, I * f_a:(I + 1) * f_a]
            jj, ii = np.unravel_index(np.argmax(block), block.shape)  # first max in c order
            out[J * n_az_c + I] = (J * f_e + jj) * n_az + (I * f_a + ii)
    return out


def anchors(coarse, goal_dir, tab, n_az, n_el, f_a, f_e, M_h, M_v, ell, p0):
    """Anchor cells and refined endpoints, Sec. IV-B-1/2, eq. (anchor-point).

    Returns (anchor_cell int32 (M,), anchor_fine int32 (M,), p_ref float64 (M,3)).
    """
    n_az_c, n_el_c = n_az // f_a, n_el // f_e
    g = np.asarray(goal_dir, np.float32).reshape(1, 3)
    if not np.any(g != 0.0):
        g = np.asarray([[1.0, 0.0, 0.0]], np.float32)      # current heading
    ig, jg = bin_directions(g, tab, n_az, n_el)
    Ig, Jg = int(ig[0]) // f_a, int(jg[0]) // f_e
    d = cell_directions(tab)
    M = M_h * M_v
    cell = np.empty(M, np.int32)
    fine = np.empty(M, np.int32)
    pref = np.empty((M, 3))
    J0 = min(max(Jg - (M_v - 1) // 2, 0), n_el_c - M_v)
    for ov in range(M_v):
        for oh in range(M_h):
            m = ov * M_h + oh
            I = (Ig - (M_h - 1) // 2 + oh) % n_az_c
            J = J0 + ov
            cell[m] = J * n_az_c + I
            fine[m] = coarse[cell[m]]
            pref[m] = np.asarray(p0, np.float32).astype(np.float64) + np.float64(np.float32(ell)) * d[fine[m]]
    return cell, fine, pref


def partition_anchors(cloud, goal_dir, n_az_c, n_el_c, f_a, f_e, r_max, ell, M_h, M_v,
                      p0=(0.0, 0.0, 0.0)):
    """The whole perception/guidance front end of one planning step."""
    n_az, n_el = n_az_c * f_a, n_el_c * f_e
    tab = partition_tables(n_az, n_el)
    key, idx = fine_partition(cloud, tab, n_az, n_el, r_max)
    cb = coarse_best(key, n_az, n_el, f_a, f_e)
    cell, fine, pref = anchors(cb, goal_dir, tab, n_az, n_el, f_a, f_e, M_h, M_v, ell, p0)
    return dict(fine_key=key, fine_idx=idx, coarse_best=cb, anchor_cell=cell,
                anchor_fine=fine, anchors=pref, tables=tab)
