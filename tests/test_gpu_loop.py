"""Closed-loop helpers on the GPU against the oracle: warm-start shift, the
adjoint refinement of the selected sequence (gradient, candidates, Stage-II
choice) and one full loop step."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fixtures import make_loop_step  # noqa: E402
from oracle import adjoint as OA  # noqa: E402
from oracle import loop as OL  # noqa: E402
from oracle import mppi as OM  # noqa: E402
from oracle.cost import nearest_kdtree  # noqa: E402
from paper_2509_17340_amd.planner import LoopRunner  # noqa: E402

pytestmark = pytest.mark.gpu


def small_loop_problem(step):
    prob = dict(make_loop_step(step))
    rng = np.random.default_rng(step)
    keep = np.sort(rng.choice(len(prob["cloud"]), 40000, replace=False))
    prob["cloud"] = prob["cloud"][keep]
    prob.update(M=4, K=256, N=20, M_h=2, M_v=2)
    prob["u_nom"] = prob["u_nom"][:4, :20].copy()
    return prob


def np_(t):
    return t.detach().cpu().numpy()


def test_loop_refinement_and_warm_start():
    prob = small_loop_problem(10)
    lr = LoopRunner(prob)
    ps = lr.ps
    print("loop step pieces: M=4 K=256 N=20 P=40000", flush=True)
    ps.run()
    torch.cuda.synchronize()
    u_nom, best = np_(ps.u_nom), int(np_(ps.best)[0])
    lr._shift(ps.u_nom, ps.best, 0, lr.u_sel)
    torch.cuda.synchronize()
    assert np.array_equal(np_(lr.u_sel)[0], u_nom[best])
    # refinement gradient of S2 (one noise-free rollout, weights (0,0,0,1,1))
    lr._bwd(lr.refine_params, lr.ref_problem, None, lr.grad, lr.grad_w, lr.ws_b)
    torch.cuda.synchronize()
    ref = dict(prob)
    ref.update(M=1, K=1, params=lr.refine_params, u_nom=np_(lr.u_sel))
    coef = np_(ps.coef)[:1].astype(np.float64)
    act = OA.active_set(ref, coef, nearest_fn=nearest_kdtree)
    og, _, _ = OA.grad(ref, coef, act)
    g = np_(lr.grad).astype(np.float64)
    rel = np.linalg.norm(g - og) / max(np.linalg.norm(og), 1e-30)
    print(f"refinement gradient rel err {rel:.2e}")
    assert rel <= 1e-4
    # candidates and their Stage-II choice
    lr._cand(ps.params, lr.u_sel[0], lr.grad[0], lr.s0, lr.beta, lr.cands)
    torch.cuda.synchronize()
    oc = OL.step_candidates(np_(lr.u_sel)[0], np_(lr.grad)[0], lr.s0, lr.beta, lr.n_cand,
                            prob["params"]["u_min"], prob["params"]["u_max"])
    np.testing.assert_allclose(np_(lr.cands), oc, rtol=1e-6, atol=1e-6)
    from paper_2509_17340_amd import select_best
    select_best(ps.params, [lr.cand_problem], lr.cS2, lr.cbest, lr.ws_c)
    torch.cuda.synchronize()
    cand = dict(prob)
    cand["M"] = lr.n_cand
    sel = OM.select_best(cand, np_(lr.cands), nearest_fn=nearest_kdtree)
    assert np.all(np.abs(np_(lr.cS2) - sel["S2"]) <= 1e-4 * np.abs(sel["S2"]))
    cb = int(np_(lr.cbest)[0])
    srt = np.sort(sel["S2"])
    if srt[1] - srt[0] > 1e-6 * abs(srt[0]):
        assert cb == sel["best"]
    assert sel["S2"][cb] <= sel["S2"][0] * (1 + 1e-6)       # never worse than no step
    lr._shift(lr.cands, lr.cbest, 1, ps.u_nom)
    torch.cuda.synchronize()
    ws = OL.shift_controls(np_(lr.cands), cb, 1, 4)
    assert np.array_equal(np_(ps.u_nom), ws.astype(np.float32))


def test_loop_steps_run_and_warm_start():
    prob = small_loop_problem(0)
    lr = LoopRunner(prob)
    for s in (0, 5):
        lr.load(small_loop_problem(s))
        lr.step()
        torch.cuda.synchronize()
        u = np_(lr.ps.u_nom)
        assert np.all(np.isfinite(u))
        assert np.all(u == u[:1])          # every instance warm-started from one plan


def test_true_closed_loop_cycles():
    """Frames recorded at the simulated pose, accumulated on the device, planned on
    and the first control applied through the model: each cycle's cloud and state
    against the oracle."""
    from fixtures import forest_scene, make_plain_problem, record_frame
    from oracle import frames as FR
    from paper_2509_17340_amd.planner import ClosedLoop

    rng = np.random.Generator(np.random.PCG64(8))
    cyl, boxes = forest_scene(rng, half=20.0)
    el = np.linspace(-15.0, 15.0, 16)

    def record(x):
        return record_frame(rng, cyl, boxes, x, 360, el, 25.0, 0.02)

    prob = dict(make_plain_problem())
    prob.pop("anchors")
    prob.update(M=4, M_h=2, M_v=2, K=256, N=20,
                x0=np.float32([0, 0, 1.5, 1, 0, 0, 0, 0, 0, 0]),
                p_goal=np.float32([18.0, 0.0, 1.5]))
    prob["u_nom"] = np.broadcast_to(prob["u_nom"][:1], (4, 20, 4)).copy()
    cl = ClosedLoop(prob, record, n_frames=3, frame_capacity=6000)
    prm = prob["params"]
    x_start = cl.x_world.copy()
    for c in range(5):
        x_prev = cl.x_world.copy()
        print(f"closed loop cycle {c}", flush=True)
        x_new = cl.cycle()
        torch.cuda.synchronize()
        F = len(cl.held)
        off = np_(cl.offsets)[:F + 1]
        n = int(off[-1])
        assert F == min(c + 1, 3) and n == cl.lr.ps.n_points > 1000
        exp = FR.to_local(np_(cl.ring), np_(cl.start)[:F], off, np_(cl.poses)[:F], x_prev[:3])
        got = np_(cl.lr.ps.cloud)[:n].astype(np.float64)
        sp = np.spacing(np.abs(exp).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(got - exp) <= sp)
        xs = FR.advance_state(x_prev, np_(cl.lr.cands), int(np_(cl.lr.cbest)[0]), prm["dt"],
                              prm["mass"], prm["gravity"])
        assert np.all(np.abs(x_new - xs) <= 2 * np.spacing(np.abs(xs).astype(np.float32)) + 1e-12)
    assert np.all(np.isfinite(cl.x_world)) and not np.array_equal(cl.x_world, x_start)
