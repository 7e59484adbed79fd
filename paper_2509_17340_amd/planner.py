"""One planning step on the device: partition -> guides -> Stage I -> Stage II.

`PlanStep` owns the device buffers of one problem and enqueues the four C-ABI
calls on the current stream; it does no arithmetic of its own.
"""
import numpy as np
import torch

from . import (CALL_MPPI_STEP, CALL_SELECT_BEST, Problem, accumulate_cloud, advance_state,
               build_guides, filtered_cloud, front_end, front_end_job, front_end_workspace_size,
               mppi_step, partition_tables, select_best, workspace_size)


class PlanStep:
    """Device state of one planning problem given as a fixture dict.

    The dict carries cloud, x0, p_goal, v_goal, q_goal, M, K, N, M_h, M_v,
    partition (n_az_c, n_el_c, f_a, f_e, r_max, ell), params, u_nom, problem_id
    and, optionally, `anchors` (then the partition is skipped and the given
    anchors are used, as for a single straight-line guide) and `collision`
    ("raw": the whole cloud, default; "filtered": P_f, the closest point of every
    fine cone) and `n_iter` (MPPI iterations per planning step, default 1;
    iteration i draws its noise at counter word iter_base + i).
    """

    def __init__(self, prob, device="cuda", keep_debug=False):
        self.prob = prob
        dev = torch.device(device)
        self.dev = dev
        self.M, self.K, self.N = prob["M"], prob["K"], prob["N"]
        M, K, N = self.M, self.K, self.N
        self.cloud = torch.from_numpy(np.ascontiguousarray(prob["cloud"], np.float32)).to(dev)
        self.n_points = int(self.cloud.shape[0])
        part = prob["partition"]
        self.part = part
        self.n_az = part["n_az_c"] * part["f_a"]
        self.n_el = part["n_el_c"] * part["f_e"]
        self.fixed_anchors = prob.get("anchors")
        if self.fixed_anchors is None:
            self.tables = torch.from_numpy(partition_tables(self.n_az, self.n_el)).to(dev)
            nf = self.n_az * self.n_el
            nc = part["n_az_c"] * part["n_el_c"]
            self.fine_key = torch.empty(nf, dtype=torch.float64, device=dev)
            self.fine_idx = torch.empty(nf, dtype=torch.int32, device=dev)
            self.coarse_best = torch.empty(nc, dtype=torch.int32, device=dev)
            self.anchor_cell = torch.empty(M, dtype=torch.int32, device=dev)
            self.anchor_fine = torch.empty(M, dtype=torch.int32, device=dev)
            self.anchors = torch.empty((M, 3), dtype=torch.float32, device=dev)
        else:
            self.anchors = torch.from_numpy(np.ascontiguousarray(self.fixed_anchors, np.float32)).to(dev)
        self.collision = prob.get("collision", "raw")
        self.pf = None
        mppi_cloud = self.cloud
        if self.collision == "filtered":
            assert self.fixed_anchors is None, "P_f needs the partition"
            self.pf = torch.empty((self.n_az * self.n_el, 3), dtype=torch.float32, device=dev)
            mppi_cloud = self.pf
        self.coef = torch.empty((M, 3, 6), dtype=torch.float32, device=dev)
        self.u_init = torch.from_numpy(np.ascontiguousarray(prob["u_nom"], np.float32)).to(dev)
        self.u_nom = self.u_init.clone()
        self.S1 = torch.empty((M, K), dtype=torch.float64, device=dev)
        self.S2 = torch.empty(M, dtype=torch.float64, device=dev)
        self.best = torch.empty(1, dtype=torch.int32, device=dev)
        self.delta_eff = self.min_dist2 = None
        if keep_debug:
            self.delta_eff = torch.empty((M, N, 4, K), dtype=torch.float32, device=dev)
            self.min_dist2 = torch.empty((M, N, K), dtype=torch.float32, device=dev)
        self.problem = Problem(mppi_cloud, M, K, N, prob["x0"], prob["p_goal"], self.u_nom,
                               coef=self.coef, v_goal=prob["v_goal"], q_goal=prob["q_goal"],
                               S1=self.S1, delta_eff=self.delta_eff, min_dist2=self.min_dist2,
                               problem_id=prob.get("problem_id", 0))
        ws = max(workspace_size(CALL_MPPI_STEP, [self.problem]),
                 workspace_size(CALL_SELECT_BEST, [self.problem]))
        self.ws = torch.empty(ws, dtype=torch.uint8, device=dev)
        self.fe_ws = torch.empty(front_end_workspace_size(1), dtype=torch.uint8, device=dev)
        self.params = prob["params"]
        self.n_iter = int(prob.get("n_iter", 1))
        if self.n_iter < 1:
            raise ValueError("n_iter must be at least 1")
        base = int(self.params.get("iter_base", 0))
        self.iter_params = [dict(self.params, iter_base=base + i) for i in range(self.n_iter)]
        x0 = np.asarray(prob["x0"], np.float32)
        self.p0, self.v0 = x0[0:3].copy(), x0[7:10].copy()
        self.a0 = np.zeros(3, np.float32)
        self.T = float(np.float32(N * np.float32(self.params["dt"])))

    def reset(self):
        self.u_nom.copy_(self.u_init)

    def set_points(self, n_points):
        """Use the first n_points rows of the cloud buffer (raw collision mode)."""
        if not 0 <= n_points <= self.cloud.shape[0]:
            raise ValueError("n_points exceeds the cloud buffer")
        self.n_points = int(n_points)
        if self.collision == "raw":
            self.problem.n_points = self.n_points

    def set_state(self, x0, p_goal):
        """New start state (drone-centred frame: p = 0) and goal for the next step."""
        x0 = np.asarray(x0, np.float32)
        p_goal = np.asarray(p_goal, np.float32)
        self.prob = dict(self.prob, x0=x0, p_goal=p_goal,
                         goal_dir=(p_goal - x0[:3]).astype(np.float32))
        self.p0, self.v0 = x0[0:3].copy(), x0[7:10].copy()
        self.problem.x0, self.problem.p_goal = x0, p_goal

    def front_end_job(self):
        """This problem's partition + guides job (None with fixed anchors)."""
        if self.fixed_anchors is not None:
            return None
        p = self.part
        return front_end_job(p["n_az_c"], p["n_el_c"], p["f_a"], p["f_e"], self.prob["M_h"],
                             self.prob["M_v"], p["r_max"], p["ell"], self.p0, self.tables,
                             self.cloud, self.prob["goal_dir"], self.v0, self.a0, self.T,
                             self.fine_key, self.fine_idx, self.coarse_best, self.anchor_cell,
                             self.anchor_fine, self.anchors, self.coef, n_points=self.n_points)

    def front_end_rest(self):
        """What follows the partition + guides job: P_f, or the guides of fixed anchors."""
        if self.fixed_anchors is not None:
            build_guides(self.p0, self.v0, self.a0, self.anchors, self.T, self.M, self.coef)
        elif self.pf is not None:
            filtered_cloud(self.cloud, self.fine_idx, self.pf)

    def front_end(self):
        job = self.front_end_job()
        if job is not None:
            front_end([job], self.fe_ws)
        self.front_end_rest()

    def stage1(self):
        for prm in self.iter_params:
            mppi_step(prm, [self.problem], self.ws)

    def stage1_iteration(self, i):
        """Only iteration i of Stage I (u_nom is read and updated in place)."""
        mppi_step(self.iter_params[i], [self.problem], self.ws)

    def stage2(self):
        select_best(self.params, [self.problem], self.S2, self.best, self.ws)

    def run(self):
        """One full planning step (all enqueued on the current stream)."""
        self.front_end()
        self.stage1()
        self.stage2()


class BatchPlan:
    """Many independent planning problems: per-problem calls or one batched call.

    Both modes run one batched partition + guides call; Stage I and Stage II are
    either 2 x n_problems plain calls or 2 batched calls.
    """

    def __init__(self, probs, device="cuda"):
        self.steps = [PlanStep(p, device=device) for p in probs]
        self.problems = [s.problem for s in self.steps]
        self.params = probs[0]["params"]
        dev = torch.device(device)
        ws = max(workspace_size(CALL_MPPI_STEP, self.problems),
                 workspace_size(CALL_SELECT_BEST, self.problems))
        self.ws = torch.empty(ws, dtype=torch.uint8, device=dev)
        self.S2 = torch.empty(sum(s.M for s in self.steps), dtype=torch.float64, device=dev)
        self.best = torch.empty(len(self.steps), dtype=torch.int32, device=dev)
        self.fe_ws = torch.empty(max(front_end_workspace_size(len(self.steps)), 1),
                                 dtype=torch.uint8, device=dev)
        self.rollout_steps = sum(s.M * s.K * s.N + s.M * s.N for s in self.steps)
        self.pairs = sum(s.M * s.K * s.N * int(s.cloud.shape[0]) for s in self.steps)

    def reset(self):
        for s in self.steps:
            s.reset()

    def front_end(self):
        """Partition and guides of every problem in one batched call, then P_f and the
        guides of problems with fixed anchors."""
        jobs = [j for j in (s.front_end_job() for s in self.steps) if j is not None]
        if jobs:
            front_end(jobs, self.fe_ws)
        for s in self.steps:
            s.front_end_rest()

    def run_plain(self):
        self.front_end()
        for s in self.steps:
            s.stage1()
        for s in self.steps:
            s.stage2()

    def run_batched(self):
        self.front_end()
        mppi_step(self.params, self.problems, self.ws)
        select_best(self.params, self.problems, self.S2, self.best, self.ws)

    def graph(self, warmup=7):
        """The batched step captured as one HIP graph (see GraphStep)."""
        return GraphStep(self, warmup=warmup, run=self.run_batched)


class GraphStep:
    """A PlanStep (or a BatchPlan, with run=its run_batched) captured once into a HIP
    graph (torch.cuda.CUDAGraph) and replayed: reset of u_nom followed by the step's
    library calls.  The warm-up runs settle the autotuner's per-shape choice (its
    timing trials synchronize, so they must not fall inside the capture).  Valid while
    the step's buffers and host inputs stay unchanged."""

    def __init__(self, step, warmup=7, run=None):
        self.step = step
        run = run or step.run
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                step.reset()
                run()
                # the tuner reads its trials' events without waiting: let each call
                # finish, so that the shape is settled before the capture
                torch.cuda.synchronize()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            step.reset()
            run()
        torch.cuda.synchronize()

    def replay(self):
        self.graph.replay()


class LoopRunner:
    """Closed loop over replayed poses: each step runs a full planning step, refines
    the selected sequence once by a gradient step on its Stage-II cost (the adjoint
    of a single noise-free rollout with weights (0, 0, 0, w_goal, w_col), step
    length picked among `n_cand` candidates by Stage II), and warm-starts every
    instance from the refined sequence advanced by one step."""

    def __init__(self, prob, n_cand=4, s0=0.5, beta=0.5, device="cuda"):
        from . import (CALL_BACKWARD, mppi_step_backward, shift_controls, step_candidates)
        self._bwd, self._shift, self._cand = mppi_step_backward, shift_controls, step_candidates
        self.ps = PlanStep(prob, device=device)
        ps = self.ps
        dev = ps.dev
        N = ps.N
        self.s0, self.beta, self.n_cand = s0, beta, n_cand
        self.u_sel = torch.empty((1, N, 4), dtype=torch.float32, device=dev)
        self.grad = torch.empty((1, N, 4), dtype=torch.float32, device=dev)
        self.grad_w = torch.empty(5, dtype=torch.float32, device=dev)
        self.cands = torch.empty((n_cand, N, 4), dtype=torch.float32, device=dev)
        self.cS2 = torch.empty(n_cand, dtype=torch.float64, device=dev)
        self.cbest = torch.empty(1, dtype=torch.int32, device=dev)
        prm = dict(ps.params)
        prm["sigma"] = np.zeros(4, np.float32)
        w = np.asarray(prm["w"], np.float32)
        prm["w"] = np.float32([0.0, 0.0, 0.0, w[3], w[4]])
        self.refine_params = prm
        self.ref_problem = Problem(ps.cloud, 1, 1, N, prob["x0"], prob["p_goal"], self.u_sel,
                                   coef=ps.coef, v_goal=prob["v_goal"], q_goal=prob["q_goal"])
        self.cand_problem = Problem(ps.cloud, n_cand, 1, N, prob["x0"], prob["p_goal"], self.cands,
                                    coef=ps.coef, v_goal=prob["v_goal"], q_goal=prob["q_goal"])
        self.ws_b = torch.empty(workspace_size(CALL_BACKWARD, [self.ref_problem]),
                                dtype=torch.uint8, device=dev)
        self.ws_c = torch.empty(workspace_size(CALL_SELECT_BEST, [self.cand_problem]),
                                dtype=torch.uint8, device=dev)

    def load(self, prob):
        """Next replayed pose: new cloud (same size) and goal; outside the timed step."""
        ps = self.ps
        ps.cloud.copy_(torch.from_numpy(np.ascontiguousarray(prob["cloud"], np.float32)))
        self.set_state(prob["x0"], prob["p_goal"])

    def load_device(self, cloud, prob):
        """Next replayed pose from a cloud already in device memory (same size), copied
        into the planner's cloud buffer on the current stream, and the pose's goal."""
        self.ps.cloud.copy_(cloud)
        self.set_state(prob["x0"], prob["p_goal"])

    def set_points(self, n_points):
        self.ps.set_points(n_points)
        self.ref_problem.n_points = self.cand_problem.n_points = self.ps.n_points

    def set_state(self, x0, p_goal):
        self.ps.set_state(x0, p_goal)
        for p in (self.ref_problem, self.cand_problem):
            p.x0, p.p_goal = self.ps.problem.x0, self.ps.problem.p_goal

    def step(self):
        self.plan()
        self.refine()

    def plan(self):
        """The planning step (partition, guides, Stage I, Stage II)."""
        self.ps.run()

    def refine(self):
        """One gradient step on the selected sequence's Stage-II cost, then the warm
        start of every instance from the refined sequence advanced by one step."""
        ps = self.ps
        self._shift(ps.u_nom, ps.best, 0, self.u_sel)
        self._bwd(self.refine_params, self.ref_problem, None, self.grad, self.grad_w, self.ws_b)
        self._cand(ps.params, self.u_sel[0], self.grad[0], self.s0, self.beta, self.cands)
        select_best(ps.params, [self.cand_problem], self.cS2, self.cbest, self.ws_c)
        self._shift(self.cands, self.cbest, 1, ps.u_nom)


class ClosedLoop:
    """A true closed loop on the device.

    Every cycle records one LiDAR frame at the vehicle's pose (`record(x)` returns
    sensor-frame points and the pose row (p, q)), stores it in the next slot of a
    device ring holding the last `n_frames` frames, accumulates the ring into the
    drone-centred cloud, runs a `LoopRunner` step (plan, refine, warm start) and
    advances the vehicle one control period under the first control of the refined
    plan.  `prob` gives M, K, N, partition, params and the goal in world
    coordinates (`p_goal`), and the initial world state `x0`.
    """

    def __init__(self, prob, record, n_frames=10, frame_capacity=100000, device="cuda"):
        dev = torch.device(device)
        self.F, self.cap, self.record = int(n_frames), int(frame_capacity), record
        self.goal_world = np.asarray(prob["p_goal"], np.float32)
        self.x_world = np.asarray(prob["x0"], np.float32).copy()
        rows = self.F * self.cap
        tmpl = dict(prob, cloud=np.zeros((rows, 3), np.float32))
        self.lr = LoopRunner(tmpl, device=device)
        self.ring = torch.zeros((rows, 3), dtype=torch.float32, device=dev)
        self.start = torch.zeros(self.F, dtype=torch.int32, device=dev)
        self.offsets = torch.zeros(self.F + 1, dtype=torch.int32, device=dev)
        self.poses = torch.zeros((self.F, 7), dtype=torch.float32, device=dev)
        self.state = torch.from_numpy(self.x_world.copy()).to(dev)
        self.held = []          # (slot, count, pose) of the frames in the ring, oldest first
        self.cycles = 0

    def _upload_frame(self, pts, pose):
        pts = np.ascontiguousarray(pts, np.float32).reshape(-1, 3)
        if len(pts) > self.cap:
            raise ValueError("frame larger than the ring slot")
        slot = self.cycles % self.F
        if len(pts):
            self.ring[slot * self.cap:slot * self.cap + len(pts)].copy_(torch.from_numpy(pts))
        self.held = [h for h in self.held if h[0] != slot] + [(slot, len(pts), np.float32(pose))]

    def cycle(self):
        ps = self.lr.ps
        pts, pose = self.record(self.x_world)
        self._upload_frame(pts, pose)
        F = len(self.held)
        counts = np.array([h[1] for h in self.held], np.int32)
        start = np.array([h[0] * self.cap for h in self.held], np.int32)
        off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        self.start[:F].copy_(torch.from_numpy(start))
        self.offsets[:F + 1].copy_(torch.from_numpy(off))
        self.poses[:F].copy_(torch.from_numpy(np.stack([h[2] for h in self.held])))
        n = int(off[-1])
        accumulate_cloud(self.ring, self.start[:F], self.offsets[:F + 1], self.poses[:F],
                         self.state, ps.cloud, n_points=n)
        self.lr.set_points(n)
        x_local = self.x_world.copy()
        x_local[0:3] = 0.0
        self.lr.set_state(x_local, self.goal_world - self.x_world[0:3])
        self.lr.step()
        # the refined plan's first control, applied through the same model and RK4 step
        advance_state(ps.params, self.state, self.lr.cands, self.lr.cbest, self.state)
        self.x_world = self.state.cpu().numpy()
        self.cycles += 1
        return self.x_world
