"""One trajectory-optimizer iteration of the whole-body hot path.

cuRoboV2's iteration (Sec. 3, the six-step loop) evaluates kinematics and
inverse dynamics on every seed x timestep state, evaluates costs, runs the
backward pass through all of them and updates the decision variables.  This
module runs the whole-body part of that loop on a batch of B states:

    FK -> sphere centres -> self-collision (max penetration, argmax, count)
    RNEA -> torques
    cost head: torque cost (sum w.tau, or c ||tau||^2) + hinge(max_pen + margin)
    backward: hinge -> two sphere gradients -> FK adjoint; tau-bar -> RNEA VJP
    optional gradient step on (q, qd, qdd)

``PlainIteration`` issues one launch per operation through the C ABI (the
"plain launch" form); ``FusedIteration`` runs the same iteration as one
kernel (``wb_wholebody_step``).  Every buffer is allocated once, so ``run``
can be captured into a HIP graph with ``torch.cuda.graph``.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import wb


class PlainIteration:
    def __init__(self, robot: wb.Robot, B: int, w: Optional[torch.Tensor] = None,
                 torque_weight: float = 1e-3, margin: float = 0.01, hinge_weight: float = 1.0,
                 lr: float = 0.0, recompute_fk_in_backward: bool = False):
        self.robot, self.B = robot, B
        self.w, self.tw, self.margin, self.hw, self.lr = w, torque_weight, margin, hinge_weight, lr
        self.recompute = recompute_fk_in_backward
        n, L, S = robot.n_dof, robot.n_links, robot.n_spheres
        e = lambda *shape, dt=torch.float32: torch.empty(shape, dtype=dt, device=robot.device)
        self.pose, self.spheres = e(L, 12, B), e(S, 3, B)
        self.max_pen, self.argmax, self.n_coll = e(B), e(B, dt=torch.int32), e(B, dt=torch.int32)
        self.tau, self.cache = e(n, B), e(L, 18, B)
        self.cost, self.g_tau, self.g_mp = e(B), e(n, B), e(B)
        self.g_spheres = e(S, 3, B)
        self.g_q_fk, self.g_q, self.g_qd, self.g_qdd = e(n, B), e(n, B), e(n, B), e(n, B)
        self.workspace = robot.workspace(B)

    def run(self, q: torch.Tensor, qd: torch.Tensor, qdd: torch.Tensor, step: bool = True) -> None:
        r = self.robot
        wb.wb_fk(r, q, self.pose, self.spheres)
        wb.wb_self_collision(r, self.spheres, self.max_pen, self.argmax, self.n_coll)
        wb.wb_rnea(r, q, qd, qdd, self.tau, self.cache)
        wb.wb_cost_head(self.tau, self.w, self.tw, self.max_pen, self.margin, self.hw, self.cost,
                        self.g_tau, self.g_mp)
        wb.wb_self_collision_backward(r, self.spheres, self.argmax, self.max_pen, self.margin, self.g_mp,
                                      self.g_spheres)
        wb.wb_fk_backward(r, q, g_spheres=self.g_spheres, link_pose=None if self.recompute else self.pose,
                          g_q=self.g_q_fk, workspace=self.workspace)
        wb.wb_rnea_backward(r, q, qd, qdd, self.cache, self.g_tau, self.g_q, self.g_qd, self.g_qdd,
                            self.workspace)
        if step and self.lr != 0.0:
            wb.wb_sgd_step(self.lr, q, qd, qdd, self.g_q, self.g_qd, self.g_qdd, g_q2=self.g_q_fk)


class PlanIteration:
    """Several robots, each with its own batch, in one persistent launch."""

    def __init__(self, robots, Bs, tunes=None, torque_weight: float = 1e-3, margin: float = 0.01,
                 hinge_weight: float = 1.0, lr: float = 0.0, outputs: bool = True, ws=None):
        self.plan = wb.Plan(robots, Bs, tunes)
        self.tw, self.margin, self.hw, self.lr = torque_weight, margin, hinge_weight, lr
        self.bufs = []
        for i, (r, B) in enumerate(zip(robots, Bs)):
            e = lambda *shape, dt=torch.float32: torch.empty(shape, dtype=dt, device=r.device)
            d = {"cost": e(B), "max_pen": e(B), "argmax": e(B, dt=torch.int32), "n_coll": e(B, dt=torch.int32)}
            if outputs:
                d.update(tau=e(r.n_dof, B), g_q=e(r.n_dof, B), g_qd=e(r.n_dof, B), g_qdd=e(r.n_dof, B))
            if ws is not None and ws[i] is not None:
                d["w"] = ws[i]
            self.bufs.append(d)

    def run(self, states, step: bool = True) -> None:
        ios = [dict(q=q, qd=qd, qdd=qdd, **b) for (q, qd, qdd), b in zip(states, self.bufs)]
        self.plan.run(ios, self.tw, self.margin, self.hw, self.lr if step else 0.0)


class FusedIteration:
    """The iteration as a single launch; same costs, gradients and step."""

    def __init__(self, robot: wb.Robot, B: int, w: Optional[torch.Tensor] = None,
                 torque_weight: float = 1e-3, margin: float = 0.01, hinge_weight: float = 1.0,
                 lr: float = 0.0, outputs: bool = True):
        if not robot.fused_supported:
            raise ValueError("robot not supported by the fused iteration (needs <= 64 links, no mimic joints)")
        self.robot, self.B = robot, B
        self.w, self.tw, self.margin, self.hw, self.lr = w, torque_weight, margin, hinge_weight, lr
        n = robot.n_dof
        e = lambda *shape, dt=torch.float32: torch.empty(shape, dtype=dt, device=robot.device)
        self.cost, self.max_pen = e(B), e(B)
        self.argmax, self.n_coll = e(B, dt=torch.int32), e(B, dt=torch.int32)
        self.tau = e(n, B) if outputs else None
        self.g_q = e(n, B) if outputs else None
        self.g_qd = e(n, B) if outputs else None
        self.g_qdd = e(n, B) if outputs else None

    def run(self, q: torch.Tensor, qd: torch.Tensor, qdd: torch.Tensor, step: bool = True) -> None:
        wb.wb_wholebody_step(self.robot, q, qd, qdd, self.w, self.tw, self.margin, self.hw,
                             self.lr if step else 0.0, self.tau, self.cost, self.max_pen, self.argmax,
                             self.n_coll, self.g_q, self.g_qd, self.g_qdd)
