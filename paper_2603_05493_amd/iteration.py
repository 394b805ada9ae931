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
            raise ValueError("robot not supported by the fused iteration (needs <= 64 links and its sweep "
                             "tables within the LDS budget)")
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


class OptimizerGraph:
    """``iters`` fused iterations with the gradient step, captured in one HIP
    graph (the paper captures the optimizer's inner loop as a CUDA graph,
    Sec. 7.2).  At every ``every``-th iteration i, ``hist`` records the state
    x_i = (q, qd, qdd) before its step (device-to-device copies), and the
    kernel writes the gradient of the cost at x_i, the cost, the maximum
    penetration and the argmax pair straight into its slot, so a run can be checked afterwards
    without host round trips.  Snapshot iterations run the kernel with its
    per-joint outputs enabled; the others write only the state and the
    per-state scalars.

    q, qd, qdd: [n][B] device tensors, updated in place by every iteration.
    """

    def __init__(self, robot: wb.Robot, q: torch.Tensor, qd: torch.Tensor, qdd: torch.Tensor,
                 iters: int = 100, every: int = 10, w: Optional[torch.Tensor] = None,
                 torque_weight: float = 1e-3, margin: float = 0.01, hinge_weight: float = 1.0,
                 lr: float = 1e-3):
        if iters < 1 or every < 1:
            raise ValueError("iters and every must be >= 1")
        B = q.shape[-1]
        kw = dict(w=w, torque_weight=torque_weight, margin=margin, hinge_weight=hinge_weight, lr=lr)
        self.q, self.qd, self.qdd = q, qd, qdd
        self.lean = FusedIteration(robot, B, outputs=False, **kw)
        self.full = FusedIteration(robot, B, outputs=True, **kw)
        self.iters, self.every = iters, every
        ns = (iters + every - 1) // every
        n = robot.n_dof
        e = lambda *shape: torch.empty(shape, dtype=torch.float32, device=q.device)
        self.hist = {k: e(ns, n, B) for k in ("q", "qd", "qdd", "g_q", "g_qd", "g_qdd")}
        self.hist["cost"], self.hist["max_pen"] = e(ns, B), e(ns, B)
        self.hist["argmax"] = torch.empty((ns, B), dtype=torch.int32, device=q.device)
        self.graph = None

    def _body(self) -> None:
        h = self.hist
        for i in range(self.iters):
            k, r = divmod(i, self.every)
            if r:
                self.lean.run(self.q, self.qd, self.qdd, step=True)
                continue
            for name, x in (("q", self.q), ("qd", self.qd), ("qdd", self.qdd)):
                h[name][k].copy_(x)
            it = self.full
            wb.wb_wholebody_step(it.robot, self.q, self.qd, self.qdd, it.w, it.tw, it.margin, it.hw, it.lr, it.tau,
                                 h["cost"][k], h["max_pen"][k], h["argmax"][k], it.n_coll, h["g_q"][k], h["g_qd"][k],
                                 h["g_qdd"][k])

    def run_eager(self) -> None:
        """The same iterations and snapshots, issued launch by launch."""
        self._body()

    def capture(self) -> None:
        # run each kernel once (no step) before capture, on a side stream
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.lean.run(self.q, self.qd, self.qdd, step=False)
            self.full.run(self.q, self.qd, self.qdd, step=False)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._body()

    def replay(self) -> None:
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()


class BsplineIteration:
    """The optimizer iteration over B-spline control points (Sec. 3 step 1
    and Sec. 4 in front of the whole-body terms): sample the splines into
    states (wb_bspline_eval), run the fused whole-body iteration on those
    states without its own step, then pull the state gradients back onto the
    control points and step them (wb_bspline_backward).

    U [d][T][K] control points (updated in place when stepping, by the
    plain or the row-normalized rule); theta0, dtheta0, ddtheta0 [d][T] the
    initial state of each trajectory; the samples are the states
    b = traj * H + t of the fused iteration.  Three forms: two_launch
    (wb_bspline_eval writes the samples, the fused iteration reads them,
    wb_bspline_backward reduces their gradients and steps), fused_sampling
    (the fused kernel forms the samples itself, wb_bspline_backward
    follows) and one_launch (wb_wholebody_step_bspline does all of it,
    reducing the control-point gradient inside the kernel; per-sample
    outputs only with sample_outputs).
    """

    def __init__(self, robot: wb.Robot, U: torch.Tensor, theta0: torch.Tensor,
                 dtheta0: Optional[torch.Tensor] = None, ddtheta0: Optional[torch.Tensor] = None,
                 dt: float = 0.05, n_interp: int = 4, reading: int = wb.GHOST_EXACT,
                 w: Optional[torch.Tensor] = None, torque_weight: float = 1e-3, margin: float = 0.01,
                 hinge_weight: float = 1.0, lr: float = 0.0, step_rule: int = wb.STEP_PLAIN,
                 form: Optional[str] = None, sample_outputs: bool = True):
        d, T, K = U.shape
        if form is None:   # the fastest form the robot and the sampling allow
            form = "fused_sampling" if n_interp == 4 and not robot.has_mimic else "two_launch"
        if form not in ("two_launch", "fused_sampling", "one_launch"):
            raise ValueError(f"unknown form {form!r}")
        if form != "two_launch" and n_interp != 4:
            raise ValueError("the fused forms take four samples per knot interval")
        if d != robot.n_dof:
            raise ValueError(f"U has {d} joints, the robot {robot.n_dof}")
        self.U, self.theta0, self.dtheta0, self.ddtheta0 = U, theta0, dtheta0, ddtheta0
        self.dt, self.n_interp, self.reading, self.lr, self.step_rule = dt, n_interp, reading, lr, step_rule
        self.K, self.T = K, T
        self.H = wb.bspline_horizon(K, n_interp)
        B = T * self.H
        e = lambda *shape: torch.empty(shape, dtype=torch.float32, device=U.device)
        self.q, self.qd, self.qdd = e(d, B), e(d, B), e(d, B)
        self.fused = FusedIteration(robot, B, w=w, torque_weight=torque_weight, margin=margin,
                                    hinge_weight=hinge_weight, lr=0.0,
                                    outputs=form != "one_launch" or sample_outputs)
        self.g_U = e(d, T, K)
        self.form = form

    def run(self, step: bool = True) -> None:
        f = self.fused
        if self.form == "one_launch":   # samples, iteration, control-point gradient and step in one kernel
            wb.wb_wholebody_step_bspline(f.robot, self.U, self.theta0, self.dt, self.dtheta0, self.ddtheta0,
                                         self.reading, f.w, f.tw, f.margin, f.hw, g_U=self.g_U,
                                         lr=self.lr if step else 0.0, step_rule=self.step_rule, tau=f.tau,
                                         cost=f.cost, max_pen=f.max_pen, argmax=f.argmax, n_coll=f.n_coll, g_q=f.g_q,
                                         g_qd=f.g_qd, g_qdd=f.g_qdd)
            return
        if self.form == "fused_sampling":   # the samples are formed inside the fused kernel
            wb.wb_wholebody_step_bspline(f.robot, self.U, self.theta0, self.dt, self.dtheta0, self.ddtheta0,
                                         self.reading, f.w, f.tw, f.margin, f.hw, tau=f.tau, cost=f.cost,
                                         max_pen=f.max_pen, argmax=f.argmax, n_coll=f.n_coll, g_q=f.g_q,
                                         g_qd=f.g_qd, g_qdd=f.g_qdd)
        else:
            wb.wb_bspline_eval(self.U, self.theta0, self.dt, self.n_interp, self.dtheta0, self.ddtheta0,
                               q=self.q, qd=self.qd, qdd=self.qdd, reading=self.reading)
            f.run(self.q, self.qd, self.qdd, step=False)
        wb.wb_bspline_backward(self.K, self.T, self.dt, self.n_interp, g_q=f.g_q, g_qd=f.g_qd, g_qdd=f.g_qdd,
                               g_U=self.g_U, lr=self.lr if step else 0.0, U=self.U, step_rule=self.step_rule)
