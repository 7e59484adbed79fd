"""Host-side checks of the C ABI: exports, tables, workspace sizes and argument
validation (no device work is enqueued by any call here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2509_17340_amd as aero
from oracle import partition as OP

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "aero.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(aero_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 9
    lib = ctypes.CDLL(aero.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    lib = aero.lib()
    for s in range(6):
        assert lib.aero_status_string(s).decode().startswith("AERO_")
    assert b"unknown" in lib.aero_status_string(99)


@pytest.mark.parametrize("n_az,n_el", [(128, 32), (120, 60), (3, 1), (360, 90), (8192, 16)])
def test_tables_match_oracle_bitwise(n_az, n_el):
    t = aero.partition_tables(n_az, n_el)
    o = OP.partition_tables(n_az, n_el)
    ref = np.concatenate([o["az_bound"].ravel(), o["el_bound"].ravel(),
                          o["az_centre"].ravel(), o["el_centre"].ravel()])
    assert t.dtype == np.float32 and t.shape == ref.shape
    assert np.array_equal(t.view(np.uint32), ref.view(np.uint32))


def test_tables_errors():
    lib = aero.lib()
    buf = np.zeros(8, np.float32)
    assert lib.aero_partition_tables(2, 4, buf.ctypes.data, buf.size) == 2
    assert lib.aero_partition_tables(16, 4, None, 100) == 1
    assert lib.aero_partition_tables(16, 4, buf.ctypes.data, buf.size) == 2


class FakeTensor:
    """Stands in for a device tensor: only an address and a shape."""

    def __init__(self, shape, addr=0x1000):
        self.shape = shape
        self._addr = addr

    def data_ptr(self):
        return self._addr

    def numel(self):
        return int(np.prod(self.shape))

    def element_size(self):
        return 1


def make_problem(M=2, K=64, N=10, P=100, **kw):
    return aero.Problem(FakeTensor((P, 3)), M, K, N, [0, 0, 0, 1, 0, 0, 0, 0, 0, 0],
                        [5, 0, 0], FakeTensor((M, N, 4)), coef=FakeTensor((M, 3, 6)), **kw)


def params(**over):
    from fixtures import table1_params
    p = table1_params()
    p.update(over)
    return p


def test_workspace_size_arithmetic():
    p = make_problem(M=3, K=100, N=7, P=50)
    a = aero.workspace_size(aero.CALL_MPPI_STEP, [p])
    MK, MNK = 3 * 100, 3 * 7 * 100
    assert a >= 8 * MK * 2 + 4 * MNK * 4 + 4 * MNK * 3 + 4 * MNK
    b = aero.workspace_size(aero.CALL_MPPI_STEP, [p, p])
    # the problems of a call share its hit-word array (at least 4 MiB)
    assert b >= 2 * a - 4096 - (1 << 22)
    assert b > a
    p2 = make_problem(M=3, K=100, N=7, P=50, S1=FakeTensor((3, 100)),
                      delta_eff=FakeTensor((3, 7, 4, 100)), min_dist2=FakeTensor((3, 7, 100)))
    assert aero.workspace_size(aero.CALL_MPPI_STEP, [p2]) < a
    assert aero.workspace_size(aero.CALL_SELECT_BEST, [p]) > 0
    assert aero.workspace_size(aero.CALL_MPPI_STEP, []) == 0
    assert aero.workspace_size(7, [p]) == 0
    bad = make_problem(K=0)
    assert aero.workspace_size(aero.CALL_MPPI_STEP, [bad]) == 0


def expect_status(code, fn, *a, **k):
    with pytest.raises(aero.AeroError) as e:
        fn(*a, **k)
    assert e.value.status == code


def test_mppi_step_validation_without_device():
    ws = FakeTensor((1 << 30,))
    ok = make_problem()
    expect_status(2, aero.mppi_step, params(), [make_problem(K=0)], ws)
    expect_status(2, aero.mppi_step, params(), [make_problem(N=1)], ws)
    expect_status(2, aero.mppi_step, params(), [make_problem(N=513)], ws)
    expect_status(2, aero.mppi_step, params(), [make_problem(M=0)], ws)
    expect_status(2, aero.mppi_step, params(), [make_problem(P=-1)], ws)
    expect_status(3, aero.mppi_step, params(lam=0.0), [ok], ws)
    expect_status(3, aero.mppi_step, params(dt=-0.1), [ok], ws)
    expect_status(3, aero.mppi_step, params(d_min=1.0, d_max=1.0), [ok], ws)
    expect_status(3, aero.mppi_step, params(sigma=np.float32([1, -1, 1, 1])), [ok], ws)
    expect_status(3, aero.mppi_step, params(u_min=np.float32([20, -3, -3, -2])), [ok], ws)
    expect_status(3, aero.mppi_step, params(C=float("nan")), [ok], ws)
    bad = make_problem()
    bad.x0 = np.float32([0, 0, 0, 0, 0, 0, 0, 0, 0, 0])
    expect_status(3, aero.mppi_step, params(), [bad], ws)
    bad = make_problem()
    bad.p_goal = np.float32([np.inf, 0, 0])
    expect_status(3, aero.mppi_step, params(), [bad], ws)
    bad = make_problem()
    bad.coef = None
    expect_status(1, aero.mppi_step, params(), [bad], ws)
    bad = make_problem()
    bad.u_nom = None
    expect_status(1, aero.mppi_step, params(), [bad], ws)
    expect_status(4, aero.mppi_step, params(), [ok], FakeTensor((16,)))
    expect_status(4, aero.mppi_step, params(), [ok], None, ws_bytes=1 << 30)
    lib = aero.lib()
    assert lib.aero_mppi_step(None, None, 1, None, 0, None) == 1
    arr = (aero.ProblemStruct * 1)()
    assert lib.aero_mppi_step(ctypes.byref(aero.params_struct(params())),
                              ctypes.cast(arr, ctypes.c_void_p), 0, None, 0, None) == 2


def test_select_and_backward_validation_without_device():
    ws = FakeTensor((1 << 30,))
    ok = make_problem()
    S2, best = FakeTensor((2,)), FakeTensor((1,))
    expect_status(1, aero.select_best, params(), [ok], None, best, ws)
    expect_status(2, aero.select_best, params(), [make_problem(N=0)], S2, best, ws)
    expect_status(4, aero.select_best, params(), [ok], S2, best, FakeTensor((8,)))
    expect_status(3, aero.select_best, params(mass=0.0), [ok], S2, best, ws)
    g = FakeTensor((2, 10, 4))
    expect_status(1, aero.mppi_step_backward, params(), ok, None, None, FakeTensor((5,)), ws)
    expect_status(1, aero.mppi_step_backward, params(), ok, FakeTensor((1,)), g, None, ws)
    expect_status(4, aero.mppi_step_backward, params(), ok, None, g, FakeTensor((5,)),
                  FakeTensor((8,)))
    expect_status(1, aero.mppi_step_backward_indexed, params(), ok, None, g, FakeTensor((5,)), ws)


def test_position_count_limit():
    """Positions are addressed by 32-bit slots: M*N*K of a problem, and the sum over a
    call, must stay below 2^31 (AERO_ERR_SHAPE otherwise, before any workspace check)."""
    ws = FakeTensor((1 << 20,))
    at = make_problem(M=256, N=512, K=1 << 14)          # exactly 2^31 positions
    expect_status(2, aero.mppi_step, params(), [at], ws)
    expect_status(2, aero.select_best, params(), [at], FakeTensor((256,)), FakeTensor((1,)), ws)
    g = FakeTensor((256, 512, 4))
    expect_status(2, aero.mppi_step_backward, params(), at, None, g, FakeTensor((5,)), ws)
    below = make_problem(M=256, N=512, K=(1 << 14) - 1)  # allowed: fails only on the workspace
    expect_status(4, aero.mppi_step, params(), [below], ws)
    half = make_problem(M=128, N=512, K=1 << 14)         # 2^30 each, 2^31 together
    expect_status(4, aero.mppi_step, params(), [half], ws)
    expect_status(2, aero.mppi_step, params(), [half, half], ws)


def test_partition_and_guides_validation_without_device():
    t = FakeTensor((100,))
    out = [FakeTensor((1,)) for _ in range(6)]
    cloud = FakeTensor((10, 3))
    common = dict(p0=(0, 0, 0), d_tables=t, cloud=cloud, goal_dir=(1, 0, 0))
    names = ["fine_key", "fine_idx", "coarse_best", "anchor_cell", "anchor_fine", "anchors"]
    kw = dict(zip(names, out))
    expect_status(2, aero.partition_anchors, 0, 8, 4, 4, 2, 2, 30.0, 5.0, **common, **kw)
    expect_status(2, aero.partition_anchors, 32, 8, 4, 4, 33, 1, 30.0, 5.0, **common, **kw)
    expect_status(2, aero.partition_anchors, 32, 8, 4, 4, 4, 9, 30.0, 5.0, **common, **kw)
    expect_status(2, aero.partition_anchors, 1, 8, 2, 4, 1, 1, 30.0, 5.0, **common, **kw)
    expect_status(3, aero.partition_anchors, 32, 8, 4, 4, 4, 2, 0.0, 5.0, **common, **kw)
    expect_status(3, aero.partition_anchors, 32, 8, 4, 4, 4, 2, 30.0, float("nan"), **common, **kw)
    kw2 = dict(kw)
    kw2["anchors"] = None
    expect_status(1, aero.partition_anchors, 32, 8, 4, 4, 4, 2, 30.0, 5.0, **common, **kw2)
    c2 = dict(common)
    c2["d_tables"] = None
    expect_status(1, aero.partition_anchors, 32, 8, 4, 4, 4, 2, 30.0, 5.0, **c2, **kw)
    expect_status(2, aero.partition_anchors, 32, 8, 4, 4, 4, 2, 30.0, 5.0, **common, **kw,
                  n_points=-3)
    z = (0, 0, 0)
    expect_status(2, aero.build_guides, z, z, z, FakeTensor((1, 3)), 2.0, 0, FakeTensor((1,)))
    expect_status(3, aero.build_guides, z, z, z, FakeTensor((1, 3)), 0.0, 1, FakeTensor((1,)))
    expect_status(3, aero.build_guides, (np.nan, 0, 0), z, z, FakeTensor((1, 3)), 2.0, 1,
                  FakeTensor((1,)))
    expect_status(1, aero.build_guides, z, z, z, None, 2.0, 1, FakeTensor((1,)))


def test_front_end_validation_without_device():
    t = FakeTensor((100,))
    names = ["fine_key", "fine_idx", "coarse_best", "anchor_cell", "anchor_fine", "anchors",
             "coef"]

    def job(**over):
        a = dict(n_az_c=32, n_el_c=8, f_a=4, f_e=4, M_h=4, M_v=2, r_max=30.0, ell=5.0,
                 p0=(0, 0, 0), d_tables=t, cloud=FakeTensor((10, 3)), goal_dir=(1, 0, 0),
                 v0=(1, 0, 0), a0=(0, 0, 0), horizon_T=2.0)
        a.update({n: FakeTensor((1,)) for n in names})
        a.update(over)
        return aero.front_end_job(**a)

    n_ws = aero.front_end_workspace_size(2)
    assert n_ws > 0
    assert aero.front_end_workspace_size(0) == 0
    ws = FakeTensor((n_ws,))
    expect_status(2, aero.front_end, [], ws)
    expect_status(4, aero.front_end, [job(), job()], FakeTensor((n_ws - 1,)))
    # every job is checked before any launch: a bad second job fails the call
    expect_status(2, aero.front_end, [job(), job(M_h=33, M_v=1)], ws)
    expect_status(2, aero.front_end, [job(), job(n_points=-1)], ws)
    expect_status(3, aero.front_end, [job(), job(horizon_T=0.0)], ws)
    expect_status(3, aero.front_end, [job(), job(v0=(np.inf, 0, 0))], ws)
    expect_status(3, aero.front_end, [job(), job(r_max=float("nan"))], ws)
    expect_status(1, aero.front_end, [job(), job(coef=None)], ws)
    expect_status(1, aero.front_end, [job(), job(d_tables=None)], ws)
    expect_status(1, aero.front_end, [job(), job(cloud=None, n_points=5)], ws)


def test_loop_calls_validation_without_device():
    ring, st, off = FakeTensor((10, 3)), FakeTensor((2,)), FakeTensor((3,))
    poses, org, out = FakeTensor((2, 7)), FakeTensor((3,)), FakeTensor((10, 3))
    expect_status(1, aero.accumulate_cloud, ring, st, None, poses, org, out)
    expect_status(2, aero.accumulate_cloud, ring, st, FakeTensor((1,)), FakeTensor((0, 7)), org, out)
    expect_status(2, aero.accumulate_cloud, ring, FakeTensor((257,)), FakeTensor((258,)),
                  FakeTensor((257, 7)), org, out)
    expect_status(2, aero.accumulate_cloud, FakeTensor((0, 3)), st, off, poses, org, out)
    aero.accumulate_cloud(ring, st, off, poses, org, FakeTensor((0, 3)))  # nothing enqueued
    x, u, i = FakeTensor((10,)), FakeTensor((4, 6, 4)), FakeTensor((1,))
    expect_status(1, aero.advance_state, params(), x, u, None, x)
    expect_status(3, aero.advance_state, params(dt=-1.0), x, u, i, x)
    expect_status(2, aero.advance_state, params(), x, FakeTensor((0, 6, 4)), i, x)
    expect_status(2, aero.shift_controls, FakeTensor((0, 6, 4)), i, 1, u)
    expect_status(2, aero.shift_controls, u, i, -1, u)
    expect_status(2, aero.step_candidates, params(), FakeTensor((6, 4)), FakeTensor((6, 4)), 0.5, 0.5,
                  FakeTensor((0, 6, 4)))
    expect_status(3, aero.step_candidates, params(), FakeTensor((6, 4)), FakeTensor((6, 4)), -0.5,
                  0.5, FakeTensor((4, 6, 4)))


def test_binding_rejects_undersized_tensors():
    import torch
    with pytest.raises(ValueError):
        aero.shift_controls(torch.zeros((2, 5, 4)), torch.zeros(1, dtype=torch.int32), 1,
                            torch.zeros((3, 5, 3)))
    with pytest.raises(TypeError):
        aero.accumulate_cloud(torch.zeros((4, 3), dtype=torch.float64), torch.zeros(1, dtype=torch.int32),
                              torch.zeros(2, dtype=torch.int32), torch.zeros((1, 7)), torch.zeros(3),
                              torch.zeros((4, 3)))
    with pytest.raises(ValueError):
        aero.advance_state(params(), torch.zeros(10), torch.zeros((2, 5, 4)).transpose(0, 1),
                           torch.zeros(1, dtype=torch.int32), torch.zeros(10))


def test_binding_refuses_values_where_device_pointers_go():
    """A backward call reads the upstream gradient on the device: a Python number given
    in its place is refused on the host (it must never become an address), and so are
    host tensors for device arguments."""
    import torch
    ws = FakeTensor((1 << 30,))
    ok = make_problem()
    g, gw = FakeTensor((2, 10, 4)), FakeTensor((5,))
    for fn in (aero.mppi_step_backward, aero.mppi_step_backward_indexed):
        with pytest.raises(TypeError):
            fn(params(), ok, 1.0, g, gw, ws)
        with pytest.raises(ValueError):
            fn(params(), ok, torch.ones(1), g, gw, ws)     # host tensor
        with pytest.raises(TypeError):
            fn(params(), ok, torch.ones(1, dtype=torch.float64), g, gw, ws)
    with pytest.raises(TypeError):
        aero.shift_controls(FakeTensor((2, 5, 4)), 0.5, 1, FakeTensor((2, 5, 4)))
    with pytest.raises(ValueError):
        aero.advance_state(params(), torch.zeros(10), FakeTensor((2, 5, 4)),
                           FakeTensor((1,)), FakeTensor((10,)))


def test_select_best_noalloc_limits_without_device():
    """The entry point that allocates nothing checks its limits on the host, before any
    device work: at most AERO_NOALLOC_BATCH_MAX problems, and a Stage-II workspace that
    fits its AERO_NOALLOC_SCRATCH_BYTES array."""
    ok = make_problem()
    S2, best = FakeTensor((4096,)), FakeTensor((64,))
    fn = aero.select_best_noalloc
    expect_status(1, fn, params(), [ok], None, best)
    expect_status(1, fn, params(), [ok], S2, None)
    expect_status(2, fn, params(), [make_problem(N=0)], S2, best)
    expect_status(3, fn, params(mass=0.0), [ok], S2, best)
    expect_status(2, fn, params(), [ok] * 17, S2, best)             # beyond the batch limit
    big = make_problem(M=256, N=512, K=1)                            # one fits ...
    ws_one = aero.workspace_size(aero.CALL_SELECT_BEST, [big])
    assert 0 < ws_one <= 32 << 20
    expect_status(4, fn, params(), [big, big, big], S2, best)        # ... three do not
    assert aero.workspace_size(aero.CALL_SELECT_BEST, [big] * 3) > 32 << 20
    lib = aero.lib()
    assert lib.aero_select_best_noalloc(None, None, 1, None, None, None) == 1
