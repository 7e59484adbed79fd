"""Pins for the oracle's partition and anchors (Sec. IV-A, IV-B-1/2).

Each check compares against something other than the oracle's own
formulas: angles from atan2 (the paper's definition of the cells),
explicit per-point loops, closed-form geometry and invariances.
"""
import math

import numpy as np
import pytest

from oracle import partition as P


def angle_cell(x, y, z, n_az, n_el):
    """Cell from the angles themselves (the paper's definition)."""
    az = math.atan2(y, x)
    el = math.atan2(z, math.hypot(x, y))
    i = int(math.floor((az + math.pi) / (2 * math.pi / n_az)))
    j = int(math.floor((el + math.pi / 2) / (math.pi / n_el)))
    return min(max(i, 0), n_az - 1), min(max(j, 0), n_el - 1), az, el


def margin(az, el, n_az, n_el):
    wa = 2 * math.pi / n_az
    we = math.pi / n_el
    fa = ((az + math.pi) / wa) % 1.0
    fe = ((el + math.pi / 2) / we) % 1.0
    return min(fa, 1 - fa) * wa, min(fe, 1 - fe) * we


@pytest.mark.parametrize("n_az,n_el", [(128, 32), (120, 60), (7, 5), (3, 1)])
def test_bins_match_angles(n_az, n_el):
    rng = np.random.default_rng(11)
    v = rng.normal(size=(4000, 3)).astype(np.float32) * rng.uniform(0.1, 30, (4000, 1)).astype(np.float32)
    tab = P.partition_tables(n_az, n_el)
    i, j = P.bin_directions(v, tab, n_az, n_el)
    checked = 0
    for k in range(len(v)):
        x, y, z = (float(c) for c in v[k])
        ia, ja, az, el = angle_cell(x, y, z, n_az, n_el)
        ma, me = margin(az, el, n_az, n_el)
        if ma > 1e-6:
            assert i[k] == ia
            checked += 1
        if me > 1e-6 and abs(el) < math.pi / 2 - 1e-6:
            assert j[k] == ja
    assert checked > 3900


def test_tables_unit_and_centres_bin_to_themselves():
    n_az, n_el = 128, 32
    tab = P.partition_tables(n_az, n_el)
    d = P.cell_directions(tab)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=2e-7)
    i, j = P.bin_directions(d.astype(np.float32), tab, n_az, n_el)
    c = j * n_az + i
    assert np.array_equal(c, np.arange(n_az * n_el))


def test_elevation_predicate_monotone():
    n_el = 60
    tab = P.partition_tables(120, n_el)
    rng = np.random.default_rng(3)
    v = rng.normal(size=(3000, 3))
    cb = tab["el_bound"][1:n_el, 0].astype(np.float64)[None, :]
    sb = tab["el_bound"][1:n_el, 1].astype(np.float64)[None, :]
    v = v.astype(np.float32).astype(np.float64)
    pred = P.elevation_at_or_above(v[:, 0:1], v[:, 1:2], v[:, 2:3], cb, sb)
    # true on a prefix of boundaries, false after
    assert np.all(np.diff(pred.astype(int), axis=1) <= 0)


def test_axis_points_and_poles():
    tab = P.partition_tables(16, 8)
    v = np.array([[0, 0, 1], [0, 0, -1], [0, 0, 5e-3], [1e-30, 0, 1]], np.float32)
    i, j = P.bin_directions(v, tab, 16, 8)
    assert list(i[:3]) == [0, 0, 0]
    assert j[0] == 7 and j[1] == 0 and j[2] == 7


def brute_partition(cloud, n_az, n_el, r_max, tab):
    """Per-point loop: cell from the oracle's bin, min r^2, lowest index."""
    n = n_az * n_el
    rmax2 = float(np.float32(r_max)) ** 2
    key = [rmax2] * n
    idx = [-1] * n
    i_all, j_all = P.bin_directions(cloud, tab, n_az, n_el)
    for k, p in enumerate(cloud.astype(np.float64)):
        r2 = (p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]
        if r2 == 0.0 or r2 > rmax2:
            continue
        c = int(j_all[k]) * n_az + int(i_all[k])
        if r2 < key[c]:
            key[c], idx[c] = r2, k
        elif r2 == key[c] and idx[c] == -1:
            idx[c] = k
    return np.array(key), np.array(idx)


def test_fine_partition_brute_force_small():
    rng = np.random.default_rng(5)
    n_az, n_el = 12, 6
    tab = P.partition_tables(n_az, n_el)
    for trial in range(20):
        n = int(rng.integers(0, 65))
        cloud = (rng.normal(size=(n, 3)) * rng.uniform(0.5, 8.0)).astype(np.float32)
        if n > 4 and trial % 3 == 0:
            cloud[1] = cloud[0]            # exact duplicate: tie on key
            cloud[3] = 0.0                 # origin point: ignored
            cloud[2] = cloud[0] * 100.0    # beyond r_max: ignored
        key, idx = P.fine_partition(cloud, tab, n_az, n_el, 10.0)
        bkey, bidx = brute_partition(cloud, n_az, n_el, 10.0, tab)
        assert np.array_equal(key, bkey)
        assert np.array_equal(idx, bidx)


def test_single_point_and_empty():
    tab = P.partition_tables(32, 16)
    key, idx = P.fine_partition(np.zeros((0, 3), np.float32), tab, 32, 16, 10.0)
    assert np.all(idx == -1) and np.all(key == 100.0)
    pt = np.array([[3.0, 4.0, 0.5]], np.float32)
    key, idx = P.fine_partition(pt, tab, 32, 16, 10.0)
    assert (idx >= 0).sum() == 1
    c = int(np.nonzero(idx >= 0)[0][0])
    assert idx[c] == 0 and key[c] == 3.0 ** 2 + 4.0 ** 2 + 0.25


def test_permutation_invariance():
    rng = np.random.default_rng(8)
    cloud = (rng.normal(size=(2000, 3)) * 6).astype(np.float32)
    tab = P.partition_tables(64, 16)
    key, idx = P.fine_partition(cloud, tab, 64, 16, 30.0)
    perm = rng.permutation(len(cloud))
    key2, idx2 = P.fine_partition(cloud[perm], tab, 64, 16, 30.0)
    assert np.array_equal(key, key2)
    has = idx >= 0
    assert np.array_equal(has, idx2 >= 0)
    assert np.array_equal(idx[has], perm[idx2[has]])


def test_coarse_argmax_loops_and_ties():
    rng = np.random.default_rng(2)
    n_az, n_el, fa, fe = 16, 8, 4, 2
    key = rng.integers(0, 5, n_az * n_el).astype(np.float64)   # many ties
    out = P.coarse_best(key, n_az, n_el, fa, fe)
    for J in range(n_el // fe):
        for I in range(n_az // fa):
            best_c, best_v = None, -1.0
            for j in range(J * fe, (J + 1) * fe):
                for i in range(I * fa, (I + 1) * fa):
                    c = j * n_az + i
                    if key[c] > best_v or (key[c] == best_v and c < best_c):
                        best_c, best_v = c, key[c]
            assert out[J * (n_az // fa) + I] == best_c


@pytest.mark.parametrize("goal", [(18.0, 0.0, 0.0), (-3.0, -7.0, 2.0), (0.0, 0.0, 0.0),
                                  (1.0, 1.0, 40.0), (0.2, -5.0, -9.0)])
def test_anchor_geometry(goal):
    rng = np.random.default_rng(4)
    cloud = (rng.normal(size=(3000, 3)) * 8).astype(np.float32)
    n_az_c, n_el_c, fa, fe = 32, 8, 4, 4
    Mh, Mv = 5, 3
    p0 = np.array([0.5, -1.0, 2.0], np.float32)
    out = P.partition_anchors(cloud, goal, n_az_c, n_el_c, fa, fe, 30.0, 5.0, Mh, Mv, p0=p0)
    tab = out["tables"]
    # |p_ref - p0| = ell (eq. anchor-point, unit d)
    r = np.linalg.norm(out["anchors"] - p0.astype(np.float64), axis=1)
    assert np.allclose(r, 5.0, rtol=1e-6)
    # each anchor direction lies in its assigned coarse cell
    d = P.cell_directions(tab)[out["anchor_fine"]]
    i, j = P.bin_directions(d.astype(np.float32), tab, n_az_c * fa, n_el_c * fe)
    assert np.array_equal((j // fe) * n_az_c + (i // fa), out["anchor_cell"])
    # the block is contiguous and contains the goal's coarse cell in azimuth
    g = np.asarray(goal, np.float32) if any(goal) else np.array([1, 0, 0], np.float32)
    gi, gj = P.bin_directions(g[None], tab, n_az_c * fa, n_el_c * fe)
    I = out["anchor_cell"] % n_az_c
    J = out["anchor_cell"] // n_az_c
    assert int(gi[0]) // fa in set(I.tolist())
    assert len(set(J.tolist())) == Mv and max(J) - min(J) == Mv - 1
    assert I.reshape(Mv, Mh).tolist() == [I[:Mh].tolist()] * Mv
    # the anchor is the coarse cell's maximum-range fine cell
    key = out["fine_key"]
    for m in range(Mh * Mv):
        Cc = out["anchor_cell"][m]
        Ic, Jc = Cc % n_az_c, Cc // n_az_c
        blk = [(jj * n_az_c * fa + ii) for jj in range(Jc * fe, (Jc + 1) * fe)
               for ii in range(Ic * fa, (Ic + 1) * fa)]
        assert key[out["anchor_fine"][m]] == max(key[b] for b in blk)


def test_nearest_range_matches_definition_on_forest():
    """r_ij = min |p| over the cone, checked with atan2 cells away from edges."""
    from fixtures import make_ensemble_problem
    prob = make_ensemble_problem(n_points=50000)
    cloud = prob["cloud"][::8]
    n_az, n_el = 128, 32
    tab = P.partition_tables(n_az, n_el)
    key, idx = P.fine_partition(cloud, tab, n_az, n_el, 30.0)
    best = {}
    for k, p in enumerate(cloud.astype(np.float64)):
        ia, ja, az, el = angle_cell(*p, n_az, n_el)
        r = math.sqrt(p[0] ** 2 + p[1] ** 2 + p[2] ** 2)
        if r > 30.0:
            continue
        c = ja * n_az + ia
        if c not in best or r < best[c][0]:
            best[c] = (r, k)
    i, j = P.bin_directions(cloud, tab, n_az, n_el)
    unsafe = set()
    for k, p in enumerate(cloud.astype(np.float64)):
        ia, ja, az, el = angle_cell(*p, n_az, n_el)
        ma, me = margin(az, el, n_az, n_el)
        if ma < 1e-6 or me < 1e-6:
            unsafe.add(int(j[k]) * n_az + int(i[k]))
            unsafe.add(ja * n_az + ia)
    checked = 0
    for c, (r, k) in best.items():
        if c in unsafe:
            continue
        assert abs(math.sqrt(key[c]) - r) <= 1e-12 * r
        assert idx[c] == k
        checked += 1
    assert checked > 500
