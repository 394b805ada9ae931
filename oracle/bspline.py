"""FP64 oracle of the B-spline trajectory front end (cuRoboV2 Sec. 4).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the benchmark's
CPU-baseline leg, never by the HIP library or its binding; it shares no code
with the HIP path.

What it computes, in the paper's notation (Sec. 4, Eqs. 10-17):
  * each joint trajectory is a uniform cubic B-spline over control points
    u_0 .. u_{K-1}; the segment that starts at knot k uses the window
    U_k = [u_{k-1}, u_k, u_{k+1}, u_{k+2}];
  * at interpolation parameter alpha in [0, 1) the state
    Theta = [theta, theta_dot, theta_ddot, theta_dddot] is B(alpha) U_k with
    B(alpha) = T P(alpha) C (Eq. 10): P holds the cubic monomials and their
    alpha-derivatives, C the cubic B-spline coefficients, T = diag(1, dt^-1,
    dt^-2, dt^-3) the time scaling;
  * the control-point gradient is the transpose, B(alpha)^T g per sample,
    summed over every sample whose window contains the control point
    (Eqs. 13-14);
  * boundaries (Sec. 4 "Boundary conditions"): three ghost knots u_{-3},
    u_{-2}, u_{-1} anchored to the initial state, and the final control point
    repeated so that it appears four times (a static goal).

Readings where the paper is silent or inconsistent:
  * sampling: every segment of the extended knot vector
    [u_{-3}, u_{-2}, u_{-1}, u_0 .. u_{K-1}, u_{K-1}, u_{K-1}, u_{K-1}]
    is sampled at alpha = i / n_interp, i = 0 .. n_interp-1, giving
    H = (K + 3) n_interp timesteps per trajectory (the paper fixes uniform
    sampling and n_interp = 4, not the count);
  * ghost knots: with the printed C, the printed Eqs. 15-17 place the first
    sample at the state reached after one knot interval of constant
    acceleration from Theta_0, not at Theta_0.  reading="exact" (default)
    solves theta(0) = theta_0, theta_dot(0) = theta_dot_0,
    theta_ddot(0) = theta_ddot_0 for the three ghost knots instead;
    reading="printed" uses Eqs. 15-17 as printed.  The ghost knots depend only
    on Theta_0, which is not an optimization variable, so no gradient flows
    to them;
  * copies of the repeated final control point are the same variable: their
    gradients add into u_{K-1}.

Arrays are trajectory-major: U [T, d, K], initial state [T, d] each, states
[T, H, d], so state b = traj * H + t in the batch order of the hot path.
"""
from __future__ import annotations

import numpy as np

# Cubic B-spline coefficient matrix (Sec. 4), rows multiply the window
# [u_{k-1}, u_k, u_{k+1}, u_{k+2}].
C_CUBIC = np.array([[-1.0, 3.0, -3.0, 1.0],
                    [3.0, -6.0, 3.0, 0.0],
                    [-3.0, 0.0, 3.0, 0.0],
                    [1.0, 4.0, 1.0, 0.0]]) / 6.0


def monomials(alpha: float) -> np.ndarray:
    """P(alpha): cubic monomials and their successive alpha-derivatives."""
    a = float(alpha)
    return np.array([[a ** 3, a ** 2, a, 1.0],
                     [3 * a ** 2, 2 * a, 1.0, 0.0],
                     [6 * a, 2.0, 0.0, 0.0],
                     [6.0, 0.0, 0.0, 0.0]])


def time_scaling(dt: float) -> np.ndarray:
    """T = diag(1, dt^-1, dt^-2, dt^-3)."""
    return np.diag([1.0, 1.0 / dt, 1.0 / dt ** 2, 1.0 / dt ** 3])


def basis(alpha: float, dt: float) -> np.ndarray:
    """B(alpha) = T P(alpha) C, the 4x4 map from a window to Theta."""
    return time_scaling(dt) @ monomials(alpha) @ C_CUBIC


def ghost_knots(theta0, dtheta0, ddtheta0, dt: float, reading: str = "exact"):
    """Ghost knots (u_{-3}, u_{-2}, u_{-1}) anchoring the spline to Theta_0."""
    th, v, a = np.asarray(theta0, float), np.asarray(dtheta0, float) * dt, np.asarray(ddtheta0, float) * dt * dt
    if reading == "printed":
        return (-a / 6.0 + th, a / 3.0 + th + v, 11.0 * a / 6.0 + th + 2.0 * v)
    if reading != "exact":
        raise ValueError(reading)
    # theta(0) = (u-3 + 4 u-2 + u-1)/6, theta_dot(0) dt = (u-1 - u-3)/2,
    # theta_ddot(0) dt^2 = u-3 - 2 u-2 + u-1, solved for the three knots
    return (th - v + a / 3.0, th - a / 6.0, th + v + a / 3.0)


def extended_knots(U: np.ndarray, theta0, dtheta0, ddtheta0, dt: float, reading: str = "exact") -> np.ndarray:
    """[u_{-3}, u_{-2}, u_{-1}, u_0 .. u_{K-1}, u_{K-1} x3] per trajectory and joint: [T, d, K + 6]."""
    g3, g2, g1 = ghost_knots(theta0, dtheta0, ddtheta0, dt, reading)
    last = U[..., -1:]
    return np.concatenate([g3[..., None], g2[..., None], g1[..., None], U, last, last, last], axis=-1)


def horizon(K: int, n_interp: int) -> int:
    return (K + 3) * n_interp


def evaluate(U, theta0, dtheta0, ddtheta0, dt: float, n_interp: int = 4, reading: str = "exact"):
    """Theta at every sample: [T, H, d, 4] (position, velocity, acceleration, jerk)."""
    U = np.asarray(U, float)
    T, d, K = U.shape
    E = extended_knots(U, theta0, dtheta0, ddtheta0, dt, reading)
    H = horizon(K, n_interp)
    out = np.empty((T, H, d, 4))
    for seg in range(K + 3):
        window = E[..., seg:seg + 4]                      # [T, d, 4] = U_k for k = seg - 2
        for i in range(n_interp):
            out[:, seg * n_interp + i] = window @ basis(i / n_interp, dt).T
    return out


def backward(g, K: int, dt: float, n_interp: int = 4):
    """Control-point gradient from upstream gradients g [T, H, d, m] on the
    first m state components (m <= 4): [T, d, K]."""
    g = np.asarray(g, float)
    T, H, d, m = g.shape
    assert H == horizon(K, n_interp)
    gE = np.zeros((T, d, K + 6))
    for seg in range(K + 3):
        for i in range(n_interp):
            Bm = basis(i / n_interp, dt)[:m]               # rows of the components with gradients
            gE[..., seg:seg + 4] += g[:, seg * n_interp + i] @ Bm
    gU = gE[..., 3:3 + K].copy()
    gU[..., -1] += gE[..., 3 + K:].sum(-1)                 # copies of the final control point
    return gU


def row_rms_step(U, gU, lr: float):
    """The row-normalized control-point step: every (trajectory, joint) row
    of K control points moves by lr * g / rms(g), rms over the row; an
    all-zero row stays.  Dividing each row by its own positive scale is a
    positive diagonal preconditioner, so the step is a descent direction
    whatever the rows' scales (the acceleration samples reach the gradient
    scaled by dt^-2)."""
    U = np.asarray(U, float)
    g = np.asarray(gU, float)
    rms = np.sqrt((g * g).mean(-1, keepdims=True))
    return U - lr * np.where(rms > 0, g / np.where(rms > 0, rms, 1.0), 0.0)
