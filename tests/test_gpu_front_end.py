"""GPU: the batched front end (partition, anchors and guides of many problems in
three launches) against the single-problem calls and the oracle.

Bar: every output bit for bit equal to aero_partition_anchors followed by
aero_build_guides on the same problem; the partition outputs bit-exact against the
oracle as well, anchors and guide coefficients within 1e-6 relative of it.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2509_17340_amd as aero  # noqa: E402
from oracle import guides as OG  # noqa: E402
from oracle import partition as OP  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"

GRIDS = [dict(n_az_c=32, n_el_c=8, f_a=4, f_e=4, r_max=30.0, ell=5.0, M_h=4, M_v=2),
         dict(n_az_c=20, n_el_c=10, f_a=6, f_e=6, r_max=10.0, ell=5.0, M_h=5, M_v=3),
         dict(n_az_c=3, n_el_c=1, f_a=1, f_e=1, r_max=4.0, ell=2.0, M_h=1, M_v=1),
         dict(n_az_c=16, n_el_c=4, f_a=2, f_e=3, r_max=12.0, ell=3.0, M_h=16, M_v=4)]


def make_case(i, rng):
    """Problem i: a grid from GRIDS, a cloud of a few sizes (one empty, one ragged),
    a start state and, for every third problem, explicit end conditions."""
    g = dict(GRIDS[i % len(GRIDS)])
    sizes = [3000, 0, 77, 600, 1, 40000, 257]
    n = sizes[i % len(sizes)]
    cloud = (rng.normal(size=(n, 3)) * (2.0 + 3.0 * (i % 3))).astype(np.float32)
    goal = np.float32([0, 0, 0]) if i % 5 == 4 else rng.normal(size=3).astype(np.float32) * 20
    p0 = rng.normal(size=3).astype(np.float32)
    v0 = rng.normal(size=3).astype(np.float32) * 2
    a0 = rng.normal(size=3).astype(np.float32)
    T = float(np.float32(1.0 + 0.25 * (i % 4)))
    M = g["M_h"] * g["M_v"]
    ends = None
    if i % 3 == 2:
        ends = (rng.normal(size=(M, 3)).astype(np.float32),
                rng.normal(size=(M, 3)).astype(np.float32))
    return dict(g=g, cloud=cloud, goal=goal, p0=p0, v0=v0, a0=a0, T=T, M=M, ends=ends)


def buffers(c):
    g = c["g"]
    n_az, n_el = g["n_az_c"] * g["f_a"], g["n_el_c"] * g["f_e"]
    M = c["M"]
    return dict(fine_key=torch.full((n_az * n_el,), -1.0, dtype=torch.float64, device=DEV),
                fine_idx=torch.full((n_az * n_el,), -7, dtype=torch.int32, device=DEV),
                coarse_best=torch.full((g["n_az_c"] * g["n_el_c"],), -7, dtype=torch.int32,
                                       device=DEV),
                anchor_cell=torch.full((M,), -7, dtype=torch.int32, device=DEV),
                anchor_fine=torch.full((M,), -7, dtype=torch.int32, device=DEV),
                anchors=torch.full((M, 3), -7.0, dtype=torch.float32, device=DEV),
                coef=torch.full((M, 3, 6), -7.0, dtype=torch.float32, device=DEV))


def device_inputs(c):
    g = c["g"]
    tab = torch.from_numpy(aero.partition_tables(g["n_az_c"] * g["f_a"],
                                                 g["n_el_c"] * g["f_e"])).to(DEV)
    cl = torch.from_numpy(c["cloud"].reshape(-1, 3)).to(DEV)
    ends = None
    if c["ends"] is not None:
        ends = tuple(torch.from_numpy(e).to(DEV) for e in c["ends"])
    return tab, cl, ends


def single(c, tab, cl, ends):
    g = c["g"]
    out = buffers(c)
    coef = out.pop("coef")
    aero.partition_anchors(g["n_az_c"], g["n_el_c"], g["f_a"], g["f_e"], g["M_h"], g["M_v"],
                           g["r_max"], g["ell"], c["p0"], tab, cl, c["goal"], **out)
    ev, ea = ends if ends is not None else (None, None)
    aero.build_guides(c["p0"], c["v0"], c["a0"], out["anchors"], c["T"], c["M"], coef,
                      end_vel=ev, end_acc=ea)
    out["coef"] = coef
    return out


def job(c, tab, cl, ends, out):
    g = c["g"]
    ev, ea = ends if ends is not None else (None, None)
    return aero.front_end_job(g["n_az_c"], g["n_el_c"], g["f_a"], g["f_e"], g["M_h"], g["M_v"],
                              g["r_max"], g["ell"], c["p0"], tab, cl, c["goal"], c["v0"], c["a0"],
                              c["T"], end_vel=ev, end_acc=ea, **out)


def same_bits(a, b):
    a, b = a.detach().cpu().numpy(), b.detach().cpu().numpy()
    return a.shape == b.shape and a.tobytes() == b.tobytes()


@pytest.mark.parametrize("n", [1, 3, 13])
def test_front_end_batch_equals_single_calls(n):
    """n = 13 problems do not fit the launch argument, so the descriptors take the
    copy-kernel path; n <= 10 travel in the argument."""
    rng = np.random.default_rng(100 + n)
    cases = [make_case(i, rng) for i in range(n)]
    print(f"front end batch of {n}: clouds {[c['cloud'].shape[0] for c in cases]}", flush=True)
    ins = [device_inputs(c) for c in cases]
    ref = [single(c, *x) for c, x in zip(cases, ins)]
    outs = [buffers(c) for c in cases]
    ws = torch.empty(aero.front_end_workspace_size(n), dtype=torch.uint8, device=DEV)
    aero.front_end([job(c, *x, o) for c, x, o in zip(cases, ins, outs)], ws)
    torch.cuda.synchronize()
    for i, (r, o) in enumerate(zip(ref, outs)):
        for k in r:
            assert same_bits(r[k], o[k]), (i, k)
    # and against the oracle
    for c, o in zip(cases, outs):
        g = c["g"]
        op = OP.partition_anchors(c["cloud"], c["goal"], g["n_az_c"], g["n_el_c"], g["f_a"],
                                  g["f_e"], g["r_max"], g["ell"], g["M_h"], g["M_v"], p0=c["p0"])
        fk = o["fine_key"].cpu().numpy()
        assert np.array_equal(fk.view(np.uint64), op["fine_key"].view(np.uint64))
        for k in ("fine_idx", "coarse_best", "anchor_cell", "anchor_fine"):
            assert np.array_equal(o[k].cpu().numpy(), op[k]), k
        anchors = o["anchors"].cpu().numpy()
        np.testing.assert_allclose(anchors, op["anchors"], rtol=1e-6, atol=1e-6)
        ev, ea = c["ends"] if c["ends"] is not None else (None, None)
        og = OG.build_guides(c["p0"], c["v0"], c["a0"], anchors, c["T"], end_vel=ev, end_acc=ea)
        coef = o["coef"].cpu().numpy()
        assert np.all(np.abs(coef - og) <= 1e-6 * np.abs(og).max(-1, keepdims=True) + 1e-7)


def test_front_end_repeated_calls_reuse_workspace():
    """Two calls in a row on one workspace, the second with fewer problems, each equal
    to the single-problem path."""
    rng = np.random.default_rng(5)
    ws = torch.empty(aero.front_end_workspace_size(13), dtype=torch.uint8, device=DEV)
    for n in (13, 2):
        cases = [make_case(i + 1, rng) for i in range(n)]
        ins = [device_inputs(c) for c in cases]
        ref = [single(c, *x) for c, x in zip(cases, ins)]
        outs = [buffers(c) for c in cases]
        aero.front_end([job(c, *x, o) for c, x, o in zip(cases, ins, outs)], ws)
        torch.cuda.synchronize()
        for r, o in zip(ref, outs):
            for k in r:
                assert same_bits(r[k], o[k]), (n, k)
