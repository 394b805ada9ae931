"""The control-point step of the optimizer load, on the oracle (no GPU): the
gradient reaching the control points carries the samples' dt^-1 and dt^-2
scaling, so the plain step U -= lr g at a rate that moves joint angles
visibly (1e-3) throws the trajectories far off and the cost grows by orders
of magnitude, while the row-normalized step at lr = 1e-2 (each joint's row
of control points moves by 0.01 rad RMS per step) lowers the cost at every
one of five steps.  Setup: the benchmark's B-spline load in small -- the
48-DoF humanoid, 4 trajectories of 9 control points U[-1.5, 1.5], initial
states at rest, dt = 0.05 s, four samples per knot interval, cost
1e-3 |tau|^2 + hinge(max_pen + 0.01)."""
import numpy as np

from oracle import bspline as bs
from paper_2603_05493_amd import synth
from tests import parity as P

DT, K, T = 0.05, 9, 4


def _problem():
    rb = synth.humanoid48(seed=0)
    rng = np.random.default_rng(3)
    U = rng.uniform(-1.5, 1.5, (T, rb.n_dof, K))
    th0 = rng.uniform(-1.5, 1.5, (T, rb.n_dof))
    return rb, U, th0


def _cost_grad(O, rb, U, th0):
    z = np.zeros_like(th0)
    Th = bs.evaluate(U, th0, z, z, DT, 4)
    H, d = Th.shape[1], rb.n_dof
    q, qd, qdd = (Th[..., r].reshape(T * H, d) for r in range(3))
    ref = P.oracle_iteration(O, rb, q, qd, qdd, None, 1e-3, 0.01, 1.0)
    g = np.stack([ref["g_q"], ref["g_qd"], ref["g_qdd"]], -1).reshape(T, H, d, 3)
    return float(ref["cost"].sum()), bs.backward(g, K, DT, 4)


def test_plain_step_at_a_useful_rate_blows_up(oracle):
    rb, U, th0 = _problem()
    c0, g = _cost_grad(oracle, rb, U, th0)
    c1, _ = _cost_grad(oracle, rb, U - 1e-3 * g, th0)
    assert np.abs(g).max() > 1e5                    # the dt^-2 scale reaches the control points
    assert c1 > 1e6 * c0


def test_row_normalized_step_lowers_the_cost(oracle):
    rb, U, th0 = _problem()
    costs = []
    for _ in range(5):
        c, g = _cost_grad(oracle, rb, U, th0)
        costs.append(c)
        U = bs.row_rms_step(U, g, 1e-2)
    assert all(b < a for a, b in zip(costs, costs[1:])), costs
    assert costs[-1] < 0.85 * costs[0]
