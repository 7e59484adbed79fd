"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar:
  * partition keys / indices / coarse argmax / anchor cells: bit-exact
  * anchors, guide coefficients, clipped perturbations: <= 1e-6 relative
  * nearest distances: |d_gpu - d_oracle| <= 1e-5 m below d_max (where the
    collision penalty reads them); beyond d_max only on the same side
  * S1, S2: |dS| <= 1e-4 |S| elementwise; samples with some step whose oracle
    distance lies within 1e-5 m of d_max (the collision jump) are counted as
    straddles and accepted under either branch
  * u_nom: oracle weights fed the GPU's S1 (teacher forcing), |du| / |u| <= 1e-4
    per instance; end to end reported with kappa = max |dS| / lambda
  * best instance: identical unless the oracle's two lowest S2 are within 1e-6
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2509_17340_amd as aero  # noqa: E402
from fixtures import make_ensemble_problem, make_plain_problem  # noqa: E402
from oracle import guides as OG  # noqa: E402
from oracle import mppi as OM  # noqa: E402
from oracle import partition as OP  # noqa: E402
from oracle import philox as OPh  # noqa: E402
from oracle.cost import nearest  # noqa: E402
from paper_2509_17340_amd.planner import PlanStep  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def sync():
    torch.cuda.synchronize()


def np_(t):
    return t.detach().cpu().numpy()


# ----------------------------------------------------------------------------
# partition and anchors
# ----------------------------------------------------------------------------
def gpu_partition(cloud, part, M_h, M_v, goal, p0=(0.0, 0.0, 0.0)):
    n_az, n_el = part["n_az_c"] * part["f_a"], part["n_el_c"] * part["f_e"]
    tab = torch.from_numpy(aero.partition_tables(n_az, n_el)).to(DEV)
    c = torch.from_numpy(np.ascontiguousarray(cloud, np.float32).reshape(-1, 3)).to(DEV)
    M = M_h * M_v
    out = dict(fine_key=torch.full((n_az * n_el,), -1.0, dtype=torch.float64, device=DEV),
               fine_idx=torch.full((n_az * n_el,), -7, dtype=torch.int32, device=DEV),
               coarse_best=torch.full((part["n_az_c"] * part["n_el_c"],), -7, dtype=torch.int32,
                                      device=DEV),
               anchor_cell=torch.empty(M, dtype=torch.int32, device=DEV),
               anchor_fine=torch.empty(M, dtype=torch.int32, device=DEV),
               anchors=torch.empty((M, 3), dtype=torch.float32, device=DEV))
    aero.partition_anchors(part["n_az_c"], part["n_el_c"], part["f_a"], part["f_e"], M_h, M_v,
                           part["r_max"], part["ell"], p0, tab, c, goal, **out)
    sync()
    return {k: np_(v) for k, v in out.items()}


def check_partition(cloud, part, M_h, M_v, goal, p0=(0.0, 0.0, 0.0)):
    g = gpu_partition(cloud, part, M_h, M_v, goal, p0)
    o = OP.partition_anchors(cloud, goal, part["n_az_c"], part["n_el_c"], part["f_a"], part["f_e"],
                             part["r_max"], part["ell"], M_h, M_v, p0=p0)
    assert np.array_equal(g["fine_key"].view(np.uint64), o["fine_key"].view(np.uint64))
    assert np.array_equal(g["fine_idx"], o["fine_idx"])
    assert np.array_equal(g["coarse_best"], o["coarse_best"])
    assert np.array_equal(g["anchor_cell"], o["anchor_cell"])
    assert np.array_equal(g["anchor_fine"], o["anchor_fine"])
    np.testing.assert_allclose(g["anchors"], o["anchors"], rtol=1e-6, atol=1e-6)
    return g, o


def test_partition_ensemble_forest_bit_exact():
    prob = make_ensemble_problem()
    print(f"partition: forest cloud {prob['cloud'].shape}", flush=True)
    g, o = check_partition(prob["cloud"], prob["partition"], prob["M_h"], prob["M_v"],
                           prob["goal_dir"])
    assert (g["fine_idx"] >= 0).sum() > 500


@pytest.mark.parametrize("case", ["empty", "single", "tiny_ragged", "origin_and_far", "zero_goal",
                                  "paper_grid"])
def test_partition_edge_cases(case):
    rng = np.random.default_rng(7)
    part = dict(n_az_c=32, n_el_c=8, f_a=4, f_e=4, r_max=30.0, ell=5.0)
    Mh, Mv, goal = 4, 2, (18.0, 0.0, 0.0)
    if case == "empty":
        cloud = np.zeros((0, 3), np.float32)
    elif case == "single":
        cloud = np.float32([[3.0, -2.0, 0.5]])
    elif case == "tiny_ragged":
        cloud = (rng.normal(size=(77, 3)) * 5).astype(np.float32)
        cloud[5] = cloud[2]
    elif case == "origin_and_far":
        cloud = (rng.normal(size=(1000, 3)) * 20).astype(np.float32)
        cloud[:10] = 0.0
        cloud[10:20] *= 10.0
    elif case == "zero_goal":
        cloud = (rng.normal(size=(3000, 3)) * 8).astype(np.float32)
        goal = (0.0, 0.0, 0.0)
    else:  # the paper's 3 deg grid: 120 x 60 fine, 20 x 10 coarse, 200k points, r_max 10 m
        part = dict(n_az_c=20, n_el_c=10, f_a=6, f_e=6, r_max=10.0, ell=5.0)
        Mh, Mv = 5, 3
        cloud = (rng.normal(size=(200000, 3)) * 6).astype(np.float32)
        goal = (30.0, 4.0, 2.0)
    print(f"partition edge case {case}: {cloud.shape}", flush=True)
    check_partition(cloud, part, Mh, Mv, goal, p0=(0.25, -0.5, 1.0))


def test_guides_match_oracle():
    rng = np.random.default_rng(3)
    M = 13
    anchors = (rng.normal(size=(M, 3)) * 5).astype(np.float32)
    p0, v0, a0 = np.float32([0.5, -1, 2]), np.float32([3, 1, -0.5]), np.float32([0.2, 0, -1])
    coef = torch.empty((M, 3, 6), dtype=torch.float32, device=DEV)
    A = torch.from_numpy(anchors).to(DEV)
    aero.build_guides(p0, v0, a0, A, 2.0, M, coef)
    ev = torch.from_numpy((rng.normal(size=(M, 3))).astype(np.float32)).to(DEV)
    coef2 = torch.empty_like(coef)
    aero.build_guides(p0, v0, a0, A, 2.0, M, coef2, end_vel=ev, end_acc=ev)
    sync()
    o = OG.build_guides(p0, v0, a0, anchors, 2.0)
    o2 = OG.build_guides(p0, v0, a0, anchors, 2.0, end_vel=np_(ev), end_acc=np_(ev))
    scale = np.abs(o).max(-1, keepdims=True)
    assert np.all(np.abs(np_(coef) - o) <= 1e-6 * scale + 1e-7)
    assert np.all(np.abs(np_(coef2) - o2) <= 1e-6 * np.abs(o2).max(-1, keepdims=True) + 1e-7)


# ----------------------------------------------------------------------------
# Stage I
# ----------------------------------------------------------------------------
def run_stage1(prob):
    ps = PlanStep(prob, keep_debug=True)
    ps.front_end()
    sync()
    coef = np_(ps.coef)
    ps.stage1()
    sync()
    return ps, dict(coef=coef, deff=np_(ps.delta_eff), md2=np_(ps.min_dist2), S1=np_(ps.S1),
                    u_new=np_(ps.u_nom))


def straddles(d, d_max, tol=1e-5):
    return (np.abs(d - d_max) < tol).any(-1)


def compare_stage1(prob, g, samples=None, nearest_fn=nearest):
    """Oracle on the GPU's guide coefficients; optionally on a subset of samples."""
    M, K, N = prob["M"], prob["K"], prob["N"]
    prm = prob["params"]
    normals = OPh.normals(prm["seed"], prob["problem_id"], M, K, N, prm["iter_base"])
    coef = g["coef"].astype(np.float64)
    # clipped perturbations, all samples
    u, deff = OM.perturb(prob["u_nom"], normals, prm)
    gdeff = np.transpose(g["deff"], (0, 3, 1, 2))           # (M,K,N,4)
    np.testing.assert_allclose(gdeff, deff, rtol=1e-6, atol=1e-7)
    # costs and distances on (a subset of) samples
    sub = np.arange(K) if samples is None else np.asarray(samples)
    p2 = dict(prob)
    p2["K"] = len(sub)
    st = OM.mppi_step(p2, coef, normals=normals[:, sub], nearest_fn=nearest_fn)
    gd = np.sqrt(np.transpose(g["md2"], (0, 2, 1))[:, sub].astype(np.float64))
    d_max = float(np.float32(prm["d_max"]))
    # exact wherever the collision penalty depends on d (below d_max); beyond, the
    # reported value only has to stay on the zero-penalty side of d_max (+inf where
    # no cloud point lies within the cull step's reach of the position's block, as
    # for an empty cloud)
    near = np.isfinite(st["d"]) & (st["d"] < d_max)
    far = ~near
    assert not np.isnan(gd).any()
    assert np.abs(gd[near] - st["d"][near]).max(initial=0.0) <= 1e-5
    assert np.all(gd[far] >= d_max - 1e-5)
    strad = straddles(st["d"], float(np.float32(prm["d_max"])))
    S_o, S_g = st["S1"], g["S1"][:, sub]
    rel = np.abs(S_g - S_o) / np.abs(S_o)
    ok = (rel <= 1e-4) | strad
    assert ok.all(), f"S1 mismatch: max rel {rel[~strad].max()}"
    # teacher-forced update over all samples
    st_all_w = OM.mppi_weights(g["S1"], prm["lam"])
    u_tf = OM.mppi_update(prob["u_nom"], st_all_w, deff)
    num = np.linalg.norm((g["u_new"] - u_tf).reshape(M, -1), axis=1)
    den = np.linalg.norm(u_tf.reshape(M, -1), axis=1)
    assert (num / den).max() <= 1e-4, f"u_nom teacher-forced rel {num / den}"
    kappa = np.abs(S_g - S_o)[~strad].max(initial=0.0) / prm["lam"]
    return dict(straddles=int(strad.sum()), s1_rel=float(rel[~strad].max(initial=0.0)),
                u_tf_rel=float((num / den).max()), kappa=float(kappa))


# (variant, cull step on): the three first-pass variants over the culled pairs, and
# the split-FP16 pass over every (block, sub-tile) pair (brute force)
PASS_A_MODES = [(0, True), (1, True), (2, True), (2, False)]


def set_pass_a_mode(mode):
    aero.set_pass_a_variant(mode[0])
    aero.set_pass_a_cull(mode[1])


def reset_pass_a_mode():
    aero.set_pass_a_variant(-1)
    aero.set_pass_a_cull(True)


@pytest.fixture(params=PASS_A_MODES, ids=["valu", "f16s512", "f16s1024", "brute"])
def pass_a(request):
    """Run the test with the first distance pass forced to one variant (and the cull
    step on or off)."""
    set_pass_a_mode(request.param)
    yield request.param
    reset_pass_a_mode()


def test_stage1_plain_cylinders_full(pass_a):
    prob = make_plain_problem()
    print("stage1 plain K=256 N=20 P=5000", flush=True)
    ps, g = run_stage1(prob)
    rep = compare_stage1(prob, g)
    print(rep)
    # end to end: the oracle with its own costs
    prm = prob["params"]
    normals = OPh.normals(prm["seed"], 0, 1, 256, 20)
    st = OM.mppi_step(prob, g["coef"].astype(np.float64), normals=normals)
    e2e = np.linalg.norm(g["u_new"] - st["u_new"]) / np.linalg.norm(st["u_new"])
    print(f"end-to-end u_nom rel {e2e:.3e} kappa {rep['kappa']:.3e}")
    if rep["kappa"] <= 1e-3:
        assert e2e <= 1e-4


def test_stage1_ensemble_forest_sampled(pass_a):
    prob = make_ensemble_problem()
    print("stage1 ensemble M=8 K=1024 N=40 P=50000 (sampled)", flush=True)
    ps, g = run_stage1(prob)
    rng = np.random.default_rng(0)
    sub = np.sort(rng.choice(prob["K"], 24, replace=False))
    sub[0] = 0
    sub[-1] = prob["K"] - 1
    rep = compare_stage1(prob, g, samples=sub)
    print(rep)


@pytest.mark.parametrize("M,K,N,P", [(1, 1, 2, 1), (3, 257, 7, 1025), (2, 100, 13, 0),
                                     (5, 64, 3, 2048), (1, 513, 25, 77)])
def test_stage1_ragged_shapes(M, K, N, P, pass_a):
    rng = np.random.default_rng(M * 1000 + K)
    prob = dict(make_plain_problem())
    prob.update(M=M, K=K, N=N, M_h=M, M_v=1)
    prob["cloud"] = (rng.normal(size=(P, 3)) * 3 + np.float32([4, 0, 0])).astype(np.float32)
    prob["u_nom"] = (np.float32([9.81, 0, 0, 0]) + rng.normal(size=(M, N, 4)) * 0.3).astype(np.float32)
    prob["anchors"] = (rng.normal(size=(M, 3)) * 3).astype(np.float32)
    prob["problem_id"] = 3
    print(f"stage1 ragged M={M} K={K} N={N} P={P}", flush=True)
    ps, g = run_stage1(prob)
    compare_stage1(prob, g)


def test_stage1_cloud_beyond_64_super_tiles():
    """A 1.3M-point cloud has 80 boxes of 16 tiles, more than one wave round of the
    cull step's super-tile scan, in both cloud orders (16,384 positions: the positions
    and the cloud are spatially sorted).  Sampled S1 and distances against the
    oracle's k-d tree search."""
    from oracle.cost import nearest_kdtree
    rng = np.random.default_rng(77)
    M, K, N, P = 2, 1024, 8, 1_300_000
    prob = dict(make_plain_problem())
    prob.update(M=M, K=K, N=N, M_h=M, M_v=1)
    prob["cloud"] = (rng.normal(size=(P, 3)) * 4 + np.float32([4, 0, 0])).astype(np.float32)
    prob["u_nom"] = (np.float32([9.81, 0, 0, 0]) + rng.normal(size=(M, N, 4)) * 0.3).astype(np.float32)
    prob["anchors"] = (rng.normal(size=(M, 3)) * 3).astype(np.float32)
    print(f"stage1 M={M} K={K} N={N} P={P}", flush=True)
    ps, g = run_stage1(prob)
    sub = np.sort(rng.choice(K, 32, replace=False))
    print(compare_stage1(prob, g, samples=sub, nearest_fn=nearest_kdtree))


def test_stage1_iterations_teacher_forced():
    """Three MPPI iterations in one planning step: each iteration against the oracle
    started from the GPU's u_nom before it; the fused loop equals the single calls."""
    prob = dict(make_plain_problem())
    prm = dict(prob["params"], iter_base=2)
    prob.update(params=prm, n_iter=3)
    print("stage1 plain K=256 N=20, 3 iterations", flush=True)
    ps = PlanStep(prob, keep_debug=True)
    ps.front_end()
    sync()
    coef = np_(ps.coef)
    for i in range(3):
        u_before = np_(ps.u_nom)
        ps.stage1_iteration(i)
        sync()
        g = dict(coef=coef, deff=np_(ps.delta_eff), md2=np_(ps.min_dist2), S1=np_(ps.S1),
                 u_new=np_(ps.u_nom))
        pi = dict(prob, u_nom=u_before, params=dict(prm, iter_base=2 + i))
        print(i, compare_stage1(pi, g))
        assert not np.array_equal(g["u_new"], u_before)
    ps2 = PlanStep(prob)
    ps2.front_end()
    ps2.stage1()
    sync()
    assert np.array_equal(np_(ps2.u_nom), np_(ps.u_nom))


def test_stage1_zero_noise_returns_nominal():
    prob = dict(make_plain_problem())
    prm = dict(prob["params"])
    prm["sigma"] = np.zeros(4, np.float32)
    prob["params"] = prm
    ps, g = run_stage1(prob)
    assert np.all(g["S1"] == g["S1"][:, :1])
    assert np.array_equal(g["u_new"], prob["u_nom"])
    assert np.all(g["deff"] == 0.0)


@pytest.mark.parametrize("M,K,N,P", [(2, 64, 512, 3000), (256, 16, 8, 2000), (2, 5000, 4, 600),
                                     (1, 1 << 20, 2, 200)],
                         ids=["longest_horizon", "most_instances", "many_samples", "most_samples"])
def test_largest_horizon_and_instance_count(M, K, N, P):
    """The longest horizon (512), the most instances (256) and the most samples (2^20)
    the ABI accepts, and more samples than the update kernel's threads hold in
    registers (5000): Stage I
    (costs and distances against the oracle on a subset of samples, the update over
    all of them) and Stage II (S2 against the oracle)."""
    rng = np.random.default_rng(M + N)
    prob = dict(make_plain_problem())
    prob.update(M=M, K=K, N=N, M_h=M, M_v=1, problem_id=5)
    prob["cloud"] = (rng.normal(size=(P, 3)) * 3 + np.float32([4, 0, 0])).astype(np.float32)
    prob["u_nom"] = (np.float32([9.81, 0, 0, 0]) + rng.normal(size=(M, N, 4)) * 0.2).astype(np.float32)
    prob["anchors"] = (rng.normal(size=(M, 3)) * 3).astype(np.float32)
    print(f"largest shapes M={M} K={K} N={N} P={P}", flush=True)
    ps, g = run_stage1(prob)
    compare_stage1(prob, g, samples=[0, K // 2, K - 1])
    ps.stage2()
    sync()
    o = OM.select_best(prob, g["u_new"])
    S2 = np_(ps.S2)
    assert np.all(np.abs(S2 - o["S2"]) <= 1e-4 * np.abs(o["S2"]))


def test_stage1_deterministic_and_batched_equals_plain(pass_a):
    rng = np.random.default_rng(11)
    probs = []
    for b, (M, K, N, P) in enumerate([(2, 300, 9, 3000), (4, 128, 20, 1500), (1, 1000, 5, 0)]):
        p = dict(make_plain_problem())
        p.update(M=M, K=K, N=N, M_h=M, M_v=1, problem_id=b)
        p["cloud"] = (rng.normal(size=(P, 3)) * 4).astype(np.float32)
        p["u_nom"] = (np.float32([9.81, 0, 0, 0]) + rng.normal(size=(M, N, 4)) * 0.2).astype(np.float32)
        p["anchors"] = (rng.normal(size=(M, 3)) * 3).astype(np.float32)
        probs.append(p)
    steps = [PlanStep(p, keep_debug=True) for p in probs]
    for s in steps:
        s.front_end()
    # plain, twice
    outs = []
    for rep in range(2):
        for s in steps:
            s.reset()
            s.stage1()
        sync()
        outs.append([(np_(s.S1), np_(s.u_nom), np_(s.min_dist2)) for s in steps])
    for a, b in zip(outs[0], outs[1]):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    # batched: one call for all three problems
    for s in steps:
        s.reset()
    pr = [s.problem for s in steps]
    ws = torch.empty(aero.workspace_size(aero.CALL_MPPI_STEP, pr), dtype=torch.uint8, device=DEV)
    aero.mppi_step(probs[0]["params"], pr, ws)
    sync()
    for s, ref in zip(steps, outs[0]):
        assert np.array_equal(np_(s.S1), ref[0])
        assert np.array_equal(np_(s.u_nom), ref[1])
        assert np.array_equal(np_(s.min_dist2), ref[2])


def variant_outputs(prob, modes=tuple(PASS_A_MODES)):
    outs = []
    for m in modes:
        set_pass_a_mode(m)
        try:
            ps, g = run_stage1(prob)
        finally:
            reset_pass_a_mode()
        outs.append(g)
    return outs


def assert_same_costs(prob, outs, min_near=0):
    a = outs[0]
    d_max2 = np.float32(prob["params"]["d_max"]) ** 2
    for b in outs[1:]:
        assert np.array_equal(a["S1"], b["S1"])
        assert np.array_equal(a["u_new"], b["u_new"])
        near = (a["md2"] < d_max2) | (b["md2"] < d_max2)
        assert np.array_equal(a["md2"][near], b["md2"][near])
        assert np.all(b["md2"][~near] >= d_max2)
        assert near.sum() >= min_near


def test_pass_a_variants_give_identical_costs():
    """Every first-pass variant, with the cull step or over the whole cloud, yields
    bitwise-identical S1, u_nom and exact distances below d_max (they may differ only
    in first-pass values beyond d_max)."""
    prob = make_ensemble_problem()
    print("pass-A variants on the ensemble forest", flush=True)
    assert_same_costs(prob, variant_outputs(prob), min_near=1000)


def test_pass_a_far_points_and_wide_blocks():
    """Points far outside the half-precision range of the recentred form (200 m and
    1e18 away) and query blocks wider than its validity radius (d_max = 70 m):
    the same costs for every variant, and the oracle's."""
    rng = np.random.default_rng(17)
    prob = dict(make_plain_problem())
    prob.update(M=2, K=300, N=9, M_h=2, M_v=1)
    near = rng.normal(size=(1500, 3)) * 3 + np.float32([4, 0, 0])
    far = rng.normal(size=(40, 3)) * 5 + np.float32([200, -150, 30])
    huge = np.full((3, 3), 1e18)
    prob["cloud"] = np.concatenate([near, far, huge, near[:10] + 0.01]).astype(np.float32)
    prob["u_nom"] = (np.float32([9.81, 0, 0, 0]) + rng.normal(size=(2, 9, 4)) * 0.3).astype(np.float32)
    prob["anchors"] = (rng.normal(size=(2, 3)) * 3).astype(np.float32)
    for d_max in (1.0, 70.0):
        prm = dict(prob["params"], d_max=d_max)
        pr = dict(prob, params=prm)
        print(f"far points, d_max={d_max}", flush=True)
        outs = variant_outputs(pr)
        assert_same_costs(pr, outs, min_near=100)
        compare_stage1(pr, outs[2])


def test_pass_b_subtile_reach_on_ordered_cloud():
    """A cloud stored in spatial order (Morton order of 20,000 points, 20 tiles): its
    256-point sub-tiles are compact, so about half of the sub-tiles of a hit tile lie
    out of the query blocks' reach and pass B skips them (30 of 60 at d_max = 1 m,
    46 of 116 at 3 m, counted with an instrumented build).  Distances below d_max
    stay exact (oracle) and every variant gives the same costs."""
    rng = np.random.default_rng(23)
    base = make_plain_problem()
    prob = dict(base)
    prob.update(M=1, K=256, N=20)
    pts = np.concatenate([base["cloud"], base["cloud"] + rng.normal(size=base["cloud"].shape) * 0.3,
                          base["cloud"] + rng.normal(size=base["cloud"].shape) * 0.6,
                          base["cloud"] + rng.normal(size=base["cloud"].shape) * 0.9])
    g = np.floor((pts - pts.min(0)) / (pts.max(0) - pts.min(0)).max() * 1023.999).astype(np.int64)
    code = np.zeros(len(pts), np.int64)
    for b in range(10):
        for a in range(3):
            code |= ((g[:, a] >> b) & 1) << (3 * b + a)
    prob["cloud"] = pts[np.argsort(code, kind="stable")].astype(np.float32)
    for d_max in (1.0, 3.0):
        pr = dict(prob, params=dict(prob["params"], d_max=d_max))
        print(f"ordered cloud 20k, d_max={d_max}", flush=True)
        outs = variant_outputs(pr)
        assert_same_costs(pr, outs, min_near=50)
        compare_stage1(pr, outs[2])


def test_distance_stats_invariants():
    """The work counts of the distance passes after one Stage-I step on the forest:
    pass B's listed pairs are a subset of pass A's, the pairs it evaluates (groups
    within each query's cap) a subset of those; with the cull step off, pass A covers
    every (position, point) pair."""
    prob = make_ensemble_problem()
    ps = PlanStep(prob)
    ps.front_end()
    Q = ps.M * ps.N * ps.K
    try:
        for cull in (1, 0):
            aero.set_pass_a_cull(cull)
            ps.reset()
            ps.stage1()
            sync()
            st = aero.distance_stats([ps.problem], ps.ws)
            print(f"cull={cull}: {st}", flush=True)
            assert st["positions"] == Q
            assert st["pairs_a"] >= st["pairs_b"] >= st["pairs_b_eval"] > 0
            assert st["pairs_b_eval"] < st["pairs_b"]
            # pass A's evaluated pairs: within the listed ones; its matrix-core products
            # cover them (padding included)
            assert st["pairs_b_eval"] <= st["pairs_a_eval"] <= st["pairs_a"]
            assert st["pairs_a_products"] >= st["pairs_a_eval"]
            if not cull:
                assert st["pairs_a"] == Q * ps.n_points
                assert st["pairs_a_eval"] == st["pairs_a"]
    finally:
        aero.set_pass_a_cull(1)


def test_autotuner_settles_and_keeps_results():
    prob = make_plain_problem()
    aero.set_pass_a_variant(-1)
    ps = PlanStep(prob)
    ps.front_end()
    res = []
    for i in range(7):  # five timed configurations, then the choice
        ps.reset()
        ps.stage1()
        sync()
        res.append((np_(ps.S1), np_(ps.u_nom)))
    v = aero.pass_a_variant([ps.problem])
    g = aero.pass_a_grid([ps.problem])
    print(f"autotuned pass-A variant: {v}, {g} workgroups")
    assert v in (0, 1, 2)
    assert g in (1024, 4096)
    for r in res[1:]:
        assert np.array_equal(r[0], res[0][0]) and np.array_equal(r[1], res[0][1])


# ----------------------------------------------------------------------------
# Stage II
# ----------------------------------------------------------------------------
def test_stage2_select_matches_oracle():
    prob = make_ensemble_problem()
    ps = PlanStep(prob)
    ps.run()
    sync()
    u = np_(ps.u_nom)
    o = OM.select_best(prob, u)
    S2 = np_(ps.S2)
    assert np.all(np.abs(S2 - o["S2"]) <= 1e-4 * np.abs(o["S2"]))
    srt = np.sort(o["S2"])
    near_tie = (srt[1] - srt[0]) <= 1e-6 * abs(srt[0])
    if not near_tie:
        assert int(np_(ps.best)[0]) == o["best"]
    print(f"S2 {S2} best {int(np_(ps.best)[0])} oracle {o['best']}")


def test_stage2_batched_equals_plain():
    """Seven problems in one Stage-I and one Stage-II call (descriptors too large for
    a kernel argument, so they are uploaded by their own launches) give bitwise the
    S2 and selected instances of the plain per-problem calls (whose descriptors
    travel in the rollout launch's argument)."""
    from paper_2509_17340_amd.planner import BatchPlan
    rng = np.random.default_rng(29)
    probs = []
    for b in range(7):
        M, K, N, P = 1 + b % 3, 96 + 32 * b, 6 + b, 800 + 300 * b
        p = dict(make_plain_problem())
        p.update(M=M, K=K, N=N, M_h=M, M_v=1, problem_id=b)
        p["cloud"] = (rng.normal(size=(P, 3)) * 3 + np.float32([3, 0, 0])).astype(np.float32)
        p["u_nom"] = (np.float32([9.81, 0, 0, 0]) + rng.normal(size=(M, N, 4)) * 0.2).astype(np.float32)
        p["anchors"] = (rng.normal(size=(M, 3)) * 3).astype(np.float32)
        probs.append(p)
    print("stage2 batched: 7 problems", flush=True)
    bp = BatchPlan(probs)
    bp.reset()
    bp.run_plain()
    sync()
    plain_S2 = np.concatenate([np_(s.S2) for s in bp.steps])
    plain_best = np.array([int(np_(s.best)[0]) for s in bp.steps])
    bp.reset()
    bp.run_batched()
    sync()
    assert np.array_equal(np_(bp.S2), plain_S2)
    assert np.array_equal(np_(bp.best), plain_best)
    # and the first problem against the oracle
    o = OM.select_best(probs[0], np_(bp.steps[0].u_nom))
    S2 = plain_S2[:probs[0]["M"]]
    assert np.all(np.abs(S2 - o["S2"]) <= 1e-4 * np.abs(o["S2"]))


def test_two_problems_batched_equal_plain():
    """Two problems in one Stage-I and one Stage-II call: their descriptors still fit
    in the first kernel's argument (each kernel reads both problems' records from it)
    and the results equal the plain calls bit for bit."""
    from paper_2509_17340_amd.planner import BatchPlan
    rng = np.random.default_rng(31)
    probs = []
    for b, (M, K, N, P) in enumerate([(3, 200, 11, 2500), (2, 352, 7, 20000)]):
        p = dict(make_plain_problem())
        p.update(M=M, K=K, N=N, M_h=M, M_v=1, problem_id=b)
        p["cloud"] = (rng.normal(size=(P, 3)) * 3 + np.float32([3, 0, 0])).astype(np.float32)
        p["u_nom"] = (np.float32([9.81, 0, 0, 0]) + rng.normal(size=(M, N, 4)) * 0.2).astype(np.float32)
        p["anchors"] = (rng.normal(size=(M, 3)) * 3).astype(np.float32)
        probs.append(p)
    print("two problems batched", flush=True)
    bp = BatchPlan(probs)
    bp.reset()
    bp.run_plain()
    sync()
    plain = [(np_(s.S1), np_(s.u_nom), np_(s.S2), int(np_(s.best)[0])) for s in bp.steps]
    bp.reset()
    bp.run_batched()
    sync()
    for s, ref in zip(bp.steps, plain):
        assert np.array_equal(np_(s.S1), ref[0])
        assert np.array_equal(np_(s.u_nom), ref[1])
    assert np.array_equal(np_(bp.S2), np.concatenate([r[2] for r in plain]))
    assert np.array_equal(np_(bp.best), np.array([r[3] for r in plain]))


def test_stage2_rejects_instance_through_obstacle():
    rng = np.random.default_rng(0)
    th = rng.uniform(-np.pi, np.pi, 4000)
    z = rng.uniform(-2, 6, 4000)
    prob = dict(make_plain_problem())
    prob["cloud"] = np.stack([3.0 + 0.3 * np.cos(th), 0.3 * np.sin(th), z], 1).astype(np.float32)
    prob["x0"] = np.float32([0, 0, 0, 1, 0, 0, 0, 4.0, 0, 0])
    N = 40
    u = np.zeros((2, N, 4), np.float32)
    u[:, :, 0] = 9.81
    u[1, :10, 1] = -0.5
    prob.update(M=2, N=N, u_nom=u, M_h=2, M_v=1,
                anchors=np.float32([[5, 0, 0], [5, 1, 0]]))
    ps = PlanStep(prob)
    ps.stage2()
    sync()
    o = OM.select_best(prob, u)
    assert o["best"] == 1 and int(np_(ps.best)[0]) == 1
    assert np_(ps.S2)[0] >= 1e6


def test_stage2_skipped_tiles_keep_every_point_within_d_max():
    """Stage II skips, per wave of positions, the cloud tiles whose box lies beyond
    d_max of the wave's positions (the collision penalty is 0 from d_max on).  A cloud
    of far filler points, whose tiles are all skipped, with single points planted at
    0.3 to 1.02 d_max from chosen rollout positions at scattered indices: S2 matches
    the oracle, whose collision terms these points set."""
    from oracle.dynamics import rollout
    rng = np.random.default_rng(41)
    prob = dict(make_plain_problem())
    prm = prob["params"]
    M, N = 5, 30
    u = np.zeros((M, N, 4), np.float32)  # body rates that fan the instances out
    u[..., 0] = 10.5
    u[..., 1] = np.linspace(-1.0, 1.0, M, dtype=np.float32)[:, None]
    u[..., 2] = np.float32([0.3, -0.3, 0.0, 0.3, -0.3])[:, None]
    x0 = np.float32([0, 0, 0, 1, 0, 0, 0, 3.0, 0, 0])
    pos = rollout(x0, u, prm["dt"], prm["mass"], prm["gravity"])[:, 1:, :3]
    d_max = float(prm["d_max"])
    # filler: a shell 25-35 m out, beyond d_max of every position
    P = 14000
    v = rng.normal(size=(P, 3))
    filler = v / np.linalg.norm(v, axis=1, keepdims=True) * rng.uniform(25, 35, (P, 1))
    planted, k = [], 0
    for m in range(M):
        for t in (3, 11, 19, 27):
            f = (0.3, 0.6, 0.9, 0.99, 1.02)[k % 5]
            w = rng.normal(size=3)
            planted.append(pos[m, t] + f * d_max * w / np.linalg.norm(w))
            k += 1
    idx = np.sort(rng.choice(P, size=len(planted), replace=False))
    cloud = filler.copy()
    cloud[idx] = np.asarray(planted)
    prob.update(M=M, N=N, u_nom=u, x0=x0, M_h=M, M_v=1, cloud=cloud.astype(np.float32),
                anchors=pos[:, -1].astype(np.float32))
    print("stage2 planted points near d_max", flush=True)
    ps = PlanStep(prob)
    ps.stage2()
    sync()
    o = OM.select_best(prob, u)
    S2 = np_(ps.S2)
    assert (o["d"] < d_max).sum() >= 12  # the planted points reach the collision term
    assert np.all(np.abs(S2 - o["S2"]) <= 1e-4 * np.abs(o["S2"]))
    srt = np.sort(o["S2"])
    if (srt[1] - srt[0]) > 1e-6 * abs(srt[0]):
        assert int(np_(ps.best)[0]) == o["best"]


@pytest.mark.parametrize("P", [0, 1, 7, 1025])
def test_stage2_tiny_clouds(P):
    """Stage II against clouds of no point, one point, a partial point step and one
    point past a tile: S2 against the oracle (an empty cloud adds no collision term)."""
    rng = np.random.default_rng(P + 5)
    M, N = 3, 20
    prob = dict(make_plain_problem())
    u = np.zeros((M, N, 4), np.float32)
    u[..., 0] = 9.81
    u[..., 1:] = rng.normal(size=(M, 1, 3)).astype(np.float32) * 0.3
    x0 = np.float32([0, 0, 0, 1, 0, 0, 0, 2.0, 0, 0])
    # points near the rollouts' path (within d_max of some positions)
    cloud = (np.float32([1.5, 0.0, 0.0]) + rng.normal(size=(P, 3)) * 0.5).astype(np.float32)
    prob.update(M=M, N=N, u_nom=u, x0=x0, M_h=M, M_v=1, cloud=cloud.reshape(-1, 3),
                anchors=(rng.normal(size=(M, 3)) * 3).astype(np.float32))
    print(f"stage2 tiny cloud P={P}", flush=True)
    ps = PlanStep(prob)
    ps.stage2()
    sync()
    o = OM.select_best(prob, u)
    S2 = np_(ps.S2)
    assert np.all(np.abs(S2 - o["S2"]) <= 1e-4 * np.abs(o["S2"]))


@pytest.mark.parametrize("M,N", [(80, 64), (128, 100), (256, 80)],
                         ids=["2_per_lane", "4_per_lane", "8_per_lane"])
def test_stage2_many_positions_per_lane(M, N):
    """Stage II sets of more than 4096 positions hold 2, 4 or 8 positions per lane
    (5,120, 12,800 and 20,480 here), each wave's box over its lanes' positions: S2
    and the selected instance against the oracle (k-d tree search)."""
    from oracle.cost import nearest_kdtree
    rng = np.random.default_rng(M + N)
    prob = dict(make_plain_problem())
    u = np.zeros((M, N, 4), np.float32)
    u[..., 0] = 9.81 + rng.normal(size=(M, 1)).astype(np.float32) * 0.5
    u[..., 1:] = rng.normal(size=(M, 1, 3)).astype(np.float32) * 0.4
    prob.update(M=M, N=N, u_nom=u, M_h=M, M_v=1,
                anchors=(rng.normal(size=(M, 3)) * 3).astype(np.float32))
    print(f"stage2 M={M} N={N} ({M * N} positions) P={len(prob['cloud'])}", flush=True)
    ps = PlanStep(prob)
    ps.stage2()
    sync()
    o = OM.select_best(prob, u, nearest_fn=nearest_kdtree)
    S2 = np_(ps.S2)
    assert (o["d"] < float(prob["params"]["d_max"])).sum() > 0  # some collision terms
    assert np.all(np.abs(S2 - o["S2"]) <= 1e-4 * np.abs(o["S2"]))
    srt = np.sort(o["S2"])
    if (srt[1] - srt[0]) > 1e-6 * abs(srt[0]):
        assert int(np_(ps.best)[0]) == o["best"]


# ----------------------------------------------------------------------------
# the paper's operating point: 120 x 60 partition, 200k-point cloud, P_f collision set
# ----------------------------------------------------------------------------
def test_paper_point_filtered_collision_set():
    from fixtures import make_paper_point_problem
    prob = make_paper_point_problem()
    print("paper point: partition 120x60, 200k points, P_f", flush=True)
    ps = PlanStep(prob, keep_debug=True)
    ps.front_end()
    sync()
    part = prob["partition"]
    o = OP.partition_anchors(prob["cloud"], prob["goal_dir"], part["n_az_c"], part["n_el_c"],
                             part["f_a"], part["f_e"], part["r_max"], part["ell"],
                             prob["M_h"], prob["M_v"])
    assert np.array_equal(np_(ps.fine_idx), o["fine_idx"])
    assert np.array_equal(np_(ps.anchor_fine), o["anchor_fine"])
    pf = np_(ps.pf)
    has = o["fine_idx"] >= 0
    assert np.array_equal(pf[has], prob["cloud"][o["fine_idx"][has]])
    assert np.all(pf[~has] == np.float32(1e18))
    ps.stage1()
    sync()
    g = dict(coef=np_(ps.coef), deff=np_(ps.delta_eff), md2=np_(ps.min_dist2), S1=np_(ps.S1),
             u_new=np_(ps.u_nom))
    # the oracle scores against P_f itself (the closest point of every non-empty cone)
    p2 = dict(prob)
    p2["cloud"] = prob["cloud"][o["fine_idx"][has]]
    rep = compare_stage1(p2, g)
    print(rep)
    ps.stage2()
    sync()
    sel = OM.select_best(p2, g["u_new"])
    assert np.all(np.abs(np_(ps.S2) - sel["S2"]) <= 1e-4 * np.abs(sel["S2"]))


def test_batched_sorted_sets_with_indices_equal_plain():
    """Clouds large enough for the spatial sort (>= 16 tiles), nearest indices
    requested: one batched call equals the plain calls bit for bit (costs, controls,
    distances below and beyond d_max, indices)."""
    rng = np.random.default_rng(23)
    probs = []
    for b, (M, K, N, P) in enumerate([(3, 700, 12, 20000), (2, 1500, 9, 41000), (2, 300, 7, 0)]):
        p = dict(make_plain_problem())
        p.update(M=M, K=K, N=N, M_h=M, M_v=1, problem_id=b)
        th = rng.uniform(-np.pi, np.pi, P)
        r = rng.uniform(0.5, 6.0, P)
        p["cloud"] = np.stack([2 + r * np.cos(th), r * np.sin(th), rng.uniform(-2, 3, P)], 1).astype(np.float32)
        p["u_nom"] = (np.float32([9.81, 0, 0, 0]) + rng.normal(size=(M, N, 4)) * 0.2).astype(np.float32)
        p["anchors"] = (rng.normal(size=(M, 3)) * 3).astype(np.float32)
        probs.append(p)
    print("batched sorted sets", flush=True)
    steps = [PlanStep(p, keep_debug=True) for p in probs]
    idx = [torch.full((p["M"], p["N"], p["K"]), -7, dtype=torch.int32, device=DEV) for p in probs]
    for s, i in zip(steps, idx):
        s.front_end()
        s.problem.nearest_idx = i
    ws = torch.empty(aero.workspace_size(aero.CALL_MPPI_STEP, [s.problem for s in steps]),
                     dtype=torch.uint8, device=DEV)
    ref = []
    for s, i in zip(steps, idx):
        s.reset()
        aero.mppi_step(s.params, [s.problem], ws)
        sync()
        ref.append((np_(s.S1), np_(s.u_nom), np_(s.min_dist2), np_(i)))
    for s in steps:
        s.reset()
    aero.mppi_step(probs[0]["params"], [s.problem for s in steps], ws)
    sync()
    for s, i, r in zip(steps, idx, ref):
        for got, exp in zip((np_(s.S1), np_(s.u_nom), np_(s.min_dist2), np_(i)), r):
            assert np.array_equal(got, exp)
    assert np.all(ref[2][3] == -1)                       # no cloud: no index
    assert (ref[0][3] >= 0).any() and (ref[1][3] >= 0).any()
