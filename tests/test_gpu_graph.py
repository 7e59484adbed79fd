"""A captured planning step replays bitwise identically to the eager step,
with eager work and synchronisations between the replays."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from fixtures import make_ensemble_problem  # noqa: E402
from paper_2509_17340_amd.planner import GraphStep, PlanStep  # noqa: E402

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
