"""A captured planning step replays bitwise identically to the eager step,
with eager work and synchronisations between the replays."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fixtures import make_batched_problems, make_ensemble_problem  # noqa: E402
from paper_2509_17340_amd.planner import BatchPlan, GraphStep, PlanStep  # noqa: E402

pytestmark = pytest.mark.gpu


def snapshot(ps):
    return [ps.u_nom.cpu().numpy().copy(), ps.S1.cpu().numpy().copy(),
            ps.S2.cpu().numpy().copy(), ps.best.cpu().numpy().copy(),
            ps.anchors.cpu().numpy().copy(), ps.coef.cpu().numpy().copy()]


def test_graph_replay_matches_eager():
    prob = make_ensemble_problem()
    ps = PlanStep(prob)
    ps.reset()
    ps.run()
    torch.cuda.synchronize()
    ref = snapshot(ps)
    g = GraphStep(ps)
    other = PlanStep(prob)          # unrelated eager work between replays
    for rep in range(3):
        print(f"graph replay {rep}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        got = snapshot(ps)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        other.reset()
        other.run()
        torch.cuda.synchronize()


def batch_snapshot(bp):
    out = [bp.S2.cpu().numpy().copy(), bp.best.cpu().numpy().copy()]
    for s in bp.steps:
        out += [s.u_nom.cpu().numpy().copy(), s.S1.cpu().numpy().copy(),
                s.anchors.cpu().numpy().copy(), s.coef.cpu().numpy().copy()]
    return out


def test_batched_graph_replay_matches_eager():
    """Eight uneven problems (10k-200k points, mixed M, K, N) in one batched step:
    captured once, replayed three times with eager work between, each replay bit for
    bit the eager batched step (descriptors of more than 2 KB, so the copy launches
    are part of the graph)."""
    probs = make_batched_problems()[:8]
    bp = BatchPlan(probs)
    for _ in range(3):                       # the autotuner settles outside the capture
        bp.reset()
        bp.run_batched()
    torch.cuda.synchronize()
    ref = batch_snapshot(bp)
    g = bp.graph()
    other = PlanStep(make_ensemble_problem())
    for rep in range(3):
        print(f"batched graph replay {rep}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        got = batch_snapshot(bp)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        other.reset()
        other.run()
        torch.cuda.synchronize()
