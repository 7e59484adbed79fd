"""Pins for the receding-horizon helpers."""
import numpy as np

from oracle import loop as L


def test_shift_holds_last_control_and_copies_selected():
    src = np.arange(3 * 5 * 4, dtype=np.float32).reshape(3, 5, 4)
    out = L.shift_controls(src, 1, 1, 4)
    assert out.shape == (4, 5, 4)
    for m in range(4):
        assert np.array_equal(out[m, :4], src[1, 1:])
        assert np.array_equal(out[m, 4], src[1, 4])
    assert np.array_equal(L.shift_controls(src, 7, 0, 1)[0], src[2])      # clamped index
    assert np.array_equal(L.shift_controls(src, 0, 9, 1)[0], np.tile(src[0, 4], (5, 1)))


def test_candidates_descend_and_respect_the_box():
    rng = np.random.default_rng(0)
    u = (np.float32([9.81, 0, 0, 0]) + rng.normal(size=(6, 4))).astype(np.float32)
    g = rng.normal(size=(6, 4)).astype(np.float32)
    lo, hi = np.float32([0.3, -3, -3, -2]), np.float32([16.35, 3, 3, 2])
    c = L.step_candidates(u, g, 0.5, 0.5, 4, lo, hi)
    assert np.array_equal(c[0], u.astype(np.float64))
    u64, g64 = u.astype(np.float64), g.astype(np.float64)
    gm = np.abs(g64).max()
    np.testing.assert_allclose(c[1], np.clip(u64 - 0.5 * g64 / gm, lo.astype(np.float64),
                                             hi.astype(np.float64)), rtol=1e-15)
    for i in range(1, 4):
        assert np.all(c[i] >= lo - 1e-12) and np.all(c[i] <= hi + 1e-12)
        # an unclipped entry moves against the gradient by exactly s_i g / max|g|
        s = 0.5 * 0.5 ** (i - 1)
        free = (c[i] > lo) & (c[i] < hi)
        np.testing.assert_allclose((u64 - c[i])[free], (s * g64 / gm)[free], rtol=1e-9, atol=1e-12)
    z = L.step_candidates(u, np.zeros_like(g), 0.5, 0.5, 3, lo, hi)
    assert np.all(z == u.astype(np.float64))
