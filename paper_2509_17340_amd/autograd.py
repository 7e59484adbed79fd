"""torch.autograd.Function over the Stage-I cost of one planning problem.

    L = StageOneCost.apply(u_nom, w, step)    # L = sum_{m,k} S1[m,k]

forward runs aero_mppi_step on a copy of u_nom (the input is not modified),
storing the nearest cloud point of every rollout position, and returns the summed
cost; backward runs aero_mppi_step_backward_indexed from those indices (no distance
pass) and returns dL/du_nom and dL/dw.  The term weights w and the upstream
gradient stay in device memory (the library reads them there), so neither
direction synchronises with the host and both can be captured into a graph.  Both
directions are single library calls; this module only moves pointers.
One context serves one forward/backward pair at a time (the indices are its own).
"""
import torch

from . import (CALL_BACKWARD, CALL_MPPI_STEP, Problem, mppi_step, mppi_step_backward_indexed,
               workspace_size)


class StageOneContext:
    """Device inputs of one problem that the cost depends on besides u_nom, w."""

    def __init__(self, cloud, coef, M, K, N, x0, p_goal, params, v_goal=(0, 0, 0),
                 q_goal=(1, 0, 0, 0), problem_id=0):
        self.cloud, self.coef = cloud, coef
        self.M, self.K, self.N = M, K, N
        self.x0, self.p_goal, self.v_goal, self.q_goal = x0, p_goal, v_goal, q_goal
        self.params = dict(params)
        self.problem_id = problem_id
        dev = cloud.device
        self.S1 = torch.empty((M, K), dtype=torch.float64, device=dev)
        self.nearest_idx = torch.empty((M, N, K), dtype=torch.int32, device=dev)
        p = self._problem(torch.empty((M, N, 4), dtype=torch.float32, device=dev), None,
                          with_idx=True)
        ws = max(workspace_size(CALL_MPPI_STEP, [p]), workspace_size(CALL_BACKWARD, [p]))
        self.ws = torch.empty(ws, dtype=torch.uint8, device=dev)

    def _problem(self, u, w, with_idx=False):
        return Problem(self.cloud, self.M, self.K, self.N, self.x0, self.p_goal, u, coef=self.coef,
                       v_goal=self.v_goal, q_goal=self.q_goal, S1=self.S1,
                       nearest_idx=self.nearest_idx if with_idx else None,
                       problem_id=self.problem_id, w=w)


class StageOneCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u_nom, w, sc):
        u = u_nom.detach().to(torch.float32).contiguous().clone()
        wd = w.detach().to(torch.float32).contiguous()
        mppi_step(sc.params, [sc._problem(u, wd, with_idx=True)], sc.ws)
        ctx.save_for_backward(u_nom.detach().to(torch.float32).contiguous(), wd)
        ctx.w_dtype = w.dtype
        ctx.sc = sc
        return sc.S1.sum()

    @staticmethod
    def backward(ctx, gL):
        u_nom, wd = ctx.saved_tensors
        sc = ctx.sc
        gu = torch.empty_like(u_nom)
        gw = torch.empty(5, dtype=torch.float32, device=u_nom.device)
        g = gL.detach().to(torch.float32).reshape(1).contiguous()
        mppi_step_backward_indexed(sc.params, sc._problem(u_nom, wd, with_idx=True), g, gu, gw,
                                   sc.ws)
        return gu, gw.to(ctx.w_dtype), None
