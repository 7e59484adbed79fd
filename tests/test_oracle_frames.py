"""Pins of the cloud accumulation and the vehicle step (oracle/frames.py)."""
import math

import numpy as np

from fixtures import table1_params
from oracle import frames as FR
from oracle.dynamics import quat_mul


def _rz(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _ry(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def _qz(a):
    return np.array([math.cos(a / 2), 0.0, 0.0, math.sin(a / 2)])


def _qy(a):
    return np.array([math.cos(a / 2), 0.0, math.sin(a / 2), 0.0])


def test_identity_pose_is_a_translation():
    rng = np.random.default_rng(0)
    pts = rng.normal(size=(50, 3)).astype(np.float32)
    pose = np.float32([[1.5, -2.0, 0.25, 1, 0, 0, 0]])
    out = FR.to_local(pts, [0], [0, 50], pose, np.float32([0.5, 0.5, 0.5]))
    exp = pts.astype(np.float64) + np.float64([1.0, -2.5, -0.25])
    np.testing.assert_array_equal(out, exp)


def test_yaw_then_pitch_matches_elementary_rotations():
    """q = q_z(psi) (x) q_y(theta) acts as Rz(psi) Ry(theta) (textbook elementary
    rotations); an unnormalised quaternion gives the same map."""
    rng = np.random.default_rng(1)
    pts = rng.normal(size=(40, 3)) * 5
    psi, th = 0.7, -0.3
    q = quat_mul(_qz(psi), _qy(th))
    pose = np.concatenate([[2.0, 1.0, -1.0], 3.0 * q])
    out = FR.to_local(pts.astype(np.float32), [0], [0, 40], pose.astype(np.float32), np.zeros(3))
    R = _rz(psi) @ _ry(th)
    exp = pts.astype(np.float32).astype(np.float64) @ R.T + np.float32([2.0, 1.0, -1.0])
    np.testing.assert_allclose(out, exp, atol=1e-6)    # pose rounded to float32


def test_frames_keep_shape_and_order():
    """A rigid map per frame: distances inside a frame are preserved, and swapping
    two frames (points and poses) swaps their outputs."""
    rng = np.random.default_rng(2)
    a = rng.normal(size=(30, 3)).astype(np.float32)
    b = rng.normal(size=(20, 3)).astype(np.float32)
    qa = _qz(1.1)
    qb = quat_mul(_qy(0.4), _qz(-2.0))
    pa = np.concatenate([[0.5, 0, 0], qa]).astype(np.float32)
    pb = np.concatenate([[0, 3.0, 1.0], qb]).astype(np.float32)
    org = np.float32([0.1, 0.2, 0.3])
    out = FR.to_local(np.concatenate([a, b]), [0, 30], [0, 30, 50], np.stack([pa, pb]), org)
    sw = FR.to_local(np.concatenate([b, a]), [0, 20], [0, 20, 50], np.stack([pb, pa]), org)
    # frames read from a ring in any slot order give the same output
    ring = np.zeros((100, 3), np.float32)
    ring[60:90], ring[5:25] = a, b
    np.testing.assert_array_equal(FR.to_local(ring, [60, 5], [0, 30, 50], np.stack([pa, pb]), org), out)
    np.testing.assert_array_equal(out[:30], sw[20:])
    np.testing.assert_array_equal(out[30:], sw[:20])
    da = np.linalg.norm(a[:, None].astype(np.float64) - a[None].astype(np.float64), axis=-1)
    do = np.linalg.norm(out[:30, None] - out[None, :30], axis=-1)
    np.testing.assert_allclose(do, da, atol=1e-6)
    # the frame origin maps to p - origin
    z = FR.to_local(np.zeros((1, 3), np.float32), [0], [0, 1], pb[None], org)
    np.testing.assert_allclose(z[0], pb[:3].astype(np.float64) - org, atol=1e-15)


def test_empty_frames_and_empty_cloud():
    pose = np.float32([[0, 0, 0, 1, 0, 0, 0]] * 3)
    pts = np.ones((4, 3), np.float32)
    out = FR.to_local(pts, [0, 0, 4], [0, 0, 4, 4], pose, np.zeros(3))
    np.testing.assert_array_equal(out, np.ones((4, 3)))
    assert FR.to_local(np.zeros((0, 3), np.float32), [0], [0, 0], pose[:1], np.zeros(3)).shape == (0, 3)


def test_advance_state_hover_and_selected_plan():
    prm = table1_params()
    mg = float(np.float32(prm["mass"]) * np.float32(prm["gravity"]))
    x0 = np.float32([1, 2, 3, 1, 0, 0, 0, 0, 0, 0])
    u = np.zeros((3, 5, 4), np.float32)
    u[:, :, 0] = 2 * mg
    u[1, 0] = [mg, 0, 0, 0]
    # hover is an equilibrium: only the selected plan's first control matters
    x1 = FR.advance_state(x0, u, 1, prm["dt"], prm["mass"], prm["gravity"])
    np.testing.assert_allclose(x1, x0.astype(np.float64), atol=1e-12)
    # index clamped; thrust 2mg with q = I is exact constant acceleration g upward
    x1 = FR.advance_state(x0, u, 7, prm["dt"], prm["mass"], prm["gravity"])
    dt = float(np.float32(prm["dt"]))
    a = 2 * mg / float(np.float32(prm["mass"])) - float(np.float32(prm["gravity"]))
    np.testing.assert_allclose(x1[2], 3 + 0.5 * a * dt * dt, rtol=1e-14)
    np.testing.assert_allclose(x1[9], a * dt, rtol=1e-14)


def test_recorded_frame_maps_back_to_the_world_hits():
    """A frame recorded in the body axes of a tilted vehicle, mapped with its pose
    (origin at the sensor), gives back the world-axis hits of the same sweep."""
    from fixtures import forest_scene, lidar_sweep, record_frame
    rng = np.random.Generator(np.random.PCG64(4))
    cyl, boxes = forest_scene(rng, half=15.0)
    q = quat_mul(_qz(0.8), quat_mul(_qy(0.2), np.array([np.cos(0.05), np.sin(0.05), 0, 0])))
    x = np.concatenate([[1.0, -2.0, 1.5], q, [0, 0, 0]])
    el = np.linspace(-15, 15, 8)
    pts, pose = record_frame(np.random.Generator(np.random.PCG64(9)), cyl, boxes, x, 180, el, 20.0, 0.0)
    hits = lidar_sweep(np.random.Generator(np.random.PCG64(9)), cyl, boxes, x[:3], 180, el, 20.0, 0.0)
    assert len(pts) == len(hits) > 100
    back = FR.to_local(pts, [0], [0, len(pts)], pose, pose[:3])
    np.testing.assert_allclose(back, hits, atol=2e-5)
