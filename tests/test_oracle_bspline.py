"""Pins of the B-spline oracle (cuRoboV2 Sec. 4, Eqs. 10-17) against what the
mathematics fixes: polynomial reproduction of the uniform cubic B-spline,
C2 continuity at the knots, time derivatives, the anchoring of the ghost
knots (both readings), the static goal, local support, and the control-point
gradient as the exact transpose of the evaluation."""
import numpy as np
import pytest

from oracle import bspline as bs

DT = 0.05


def _rand(T=3, d=4, K=9, seed=0):
    rng = np.random.default_rng(seed)
    U = rng.uniform(-1.5, 1.5, (T, d, K))
    th0 = rng.uniform(-1.5, 1.5, (T, d))
    v0 = rng.normal(size=(T, d))
    a0 = rng.normal(size=(T, d))
    return U, th0, v0, a0


def test_horizon_of_the_optimizer_load():
    # 12 segments of 4 samples: 48 timesteps per seed from 9 control points
    assert bs.horizon(9, 4) == 48
    U, th0, v0, a0 = _rand(K=9)
    assert bs.evaluate(U, th0, v0, a0, DT, 4).shape == (3, 48, 4, 4)


def test_constant_control_points_are_a_rest_state():
    U = np.full((2, 3, 6), 0.7)
    z = np.zeros((2, 3))
    Th = bs.evaluate(U, z + 0.7, z, z, DT, 4)
    np.testing.assert_allclose(Th[..., 0], 0.7, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Th[..., 1:], 0.0, atol=1e-12)


@pytest.mark.parametrize("n_interp", [1, 2, 4, 5])
def test_quadratic_reproduction_and_exact_ghosts(n_interp):
    """The uniform cubic B-spline over u_k = f(k) - f''/6 reproduces a
    quadratic f exactly (Marsden's identity); with the exact ghost knots
    computed from f's state at the first sample, every sample of every
    segment not touched by the final repeats lies on f."""
    c0, c1, c2 = 0.3, -0.8, 0.45
    f = lambda x: c2 * x * x + c1 * x + c0
    K = 8
    k = np.arange(K, dtype=float)
    U = (f(k) - c2 / 3.0)[None, None, :]                   # f'' / 6 = c2 / 3
    x0 = -2.0                                              # the first sample sits at knot index -2
    th0 = np.array([[f(x0)]])
    v0 = np.array([[(2 * c2 * x0 + c1) / DT]])
    a0 = np.array([[2 * c2 / DT ** 2]])
    Th = bs.evaluate(U, th0, v0, a0, DT, n_interp)
    for seg in range(K):                                   # windows free of the repeated final knot
        for i in range(n_interp):
            x = seg - 2 + i / n_interp
            t = Th[0, seg * n_interp + i, 0]
            np.testing.assert_allclose(t[0], f(x), rtol=0, atol=1e-12)
            np.testing.assert_allclose(t[1], (2 * c2 * x + c1) / DT, rtol=1e-12, atol=1e-10)
            np.testing.assert_allclose(t[2], 2 * c2 / DT ** 2, rtol=1e-12)
            np.testing.assert_allclose(t[3], 0.0, atol=1e-6)


def test_exact_ghosts_start_at_the_initial_state():
    U, th0, v0, a0 = _rand()
    Th = bs.evaluate(U, th0, v0, a0, DT, 4, reading="exact")
    np.testing.assert_allclose(Th[:, 0, :, 0], th0, atol=1e-12)
    np.testing.assert_allclose(Th[:, 0, :, 1], v0, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(Th[:, 0, :, 2], a0, rtol=1e-10, atol=1e-10)


def test_printed_ghosts_start_one_interval_of_constant_acceleration_later():
    """The ghost knots as printed place the first sample at Theta_0 carried
    forward by dt with zero jerk -- the reason the exact reading is the
    default."""
    U, th0, v0, a0 = _rand()
    Th = bs.evaluate(U, th0, v0, a0, DT, 4, reading="printed")
    np.testing.assert_allclose(Th[:, 0, :, 0], th0 + v0 * DT + 0.5 * a0 * DT ** 2, atol=1e-12)
    np.testing.assert_allclose(Th[:, 0, :, 1], v0 + a0 * DT, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(Th[:, 0, :, 2], a0, rtol=1e-10, atol=1e-10)
    assert np.abs(Th[:, 0, :, 0] - th0).max() > 1e-3


def test_c2_continuity_at_the_knots():
    U, th0, v0, a0 = _rand(seed=1)
    E = bs.extended_knots(U, th0, v0, a0, DT)
    for seg in range(U.shape[-1] + 2):
        end = E[..., seg:seg + 4] @ bs.basis(1.0, DT).T
        start = E[..., seg + 1:seg + 5] @ bs.basis(0.0, DT).T
        np.testing.assert_allclose(end[..., :3], start[..., :3], rtol=1e-11, atol=1e-9)


def test_derivative_rows_are_time_derivatives():
    """Row r of B(alpha) is d/dt of row r-1 (t = alpha dt), by central
    differences in alpha."""
    h = 1e-6
    for alpha in (0.1, 0.37, 0.9):
        Bp, Bm, B0 = bs.basis(alpha + h, DT), bs.basis(alpha - h, DT), bs.basis(alpha, DT)
        fd = (Bp[:3] - Bm[:3]) / (2 * h * DT)
        np.testing.assert_allclose(fd, B0[1:], rtol=1e-6, atol=1e-4)


def test_static_goal():
    U, th0, v0, a0 = _rand(seed=2)
    n = 4
    Th = bs.evaluate(U, th0, v0, a0, DT, n)
    last = Th[:, -n:]                                      # the all-repeat segment
    np.testing.assert_allclose(last[..., 0], np.broadcast_to(U[:, None, :, -1], last[..., 0].shape), atol=1e-12)
    np.testing.assert_allclose(last[..., 1:], 0.0, atol=1e-9)
    # and it is reached smoothly: the end of the previous segment is that rest state
    E = bs.extended_knots(U, th0, v0, a0, DT)
    K = U.shape[-1]
    end = E[..., K + 1:K + 5] @ bs.basis(1.0, DT).T
    np.testing.assert_allclose(end[..., 0], U[..., -1], atol=1e-12)
    np.testing.assert_allclose(end[..., 1:3], 0.0, atol=1e-9)


def test_backward_local_support():
    """A gradient on one sample of segment s reaches exactly the control
    points of its window (extended indices s .. s+3) that are variables."""
    K, n, d = 9, 4, 1
    for seg in range(K + 3):
        g = np.zeros((1, bs.horizon(K, n), d, 3))
        g[0, seg * n + 1, 0] = [1.0, 0.5, 0.25]
        gU = bs.backward(g, K, DT, n)[0, 0]
        ext = [e - 3 for e in range(seg, seg + 4)]           # control point indices of the window
        expect = sorted({min(max(k, -99), K - 1) for k in ext if k >= 0})
        nz = sorted(np.nonzero(np.abs(gU) > 0)[0].tolist())
        assert nz == expect, (seg, nz, expect)


def test_backward_is_the_transpose_of_evaluation():
    """<g, J dU> = <J^T g, dU>: evaluation is affine in U for a fixed
    initial state, so J dU = eval(U + dU) - eval(U)."""
    U, th0, v0, a0 = _rand(T=2, d=3, K=7, seed=3)
    rng = np.random.default_rng(4)
    dU = rng.normal(size=U.shape)
    H = bs.horizon(7, 4)
    g = rng.normal(size=(2, H, 3, 4))
    JdU = bs.evaluate(U + dU, th0, v0, a0, DT) - bs.evaluate(U, th0, v0, a0, DT)
    lhs = np.sum(g * JdU)
    rhs = np.sum(bs.backward(g, 7, DT) * dU)
    assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(lhs))


def test_backward_matches_central_fd():
    U, th0, v0, a0 = _rand(T=1, d=2, K=6, seed=5)
    rng = np.random.default_rng(6)
    w = rng.normal(size=(1, bs.horizon(6, 4), 2, 3))
    loss = lambda X: np.sum(w * bs.evaluate(X, th0, v0, a0, DT)[..., :3])
    gU = bs.backward(w, 6, DT)
    h = 1e-6
    for idx in [(0, 0, 0), (0, 1, 2), (0, 0, 5), (0, 1, 3)]:
        Up, Um = U.copy(), U.copy()
        Up[idx] += h
        Um[idx] -= h
        fd = (loss(Up) - loss(Um)) / (2 * h)
        np.testing.assert_allclose(gU[idx], fd, rtol=1e-6, atol=1e-3)


def test_control_point_gradient_scales_as_dt_powers():
    """With the sample gradients held fixed, the part of the control-point
    gradient that comes through the velocity samples scales as 1/dt and the
    part through the acceleration samples as 1/dt^2 (the time scaling of
    Eqs. 11-12), exactly."""
    T, d, K = 2, 3, 9
    H = bs.horizon(K, 4)
    g = np.random.default_rng(4).normal(size=(T, H, d, 3))
    only = lambda c: np.where(np.arange(3) == c, g, 0.0)
    for c, power in ((0, 0), (1, 1), (2, 2)):
        a = bs.backward(only(c), K, DT, 4)
        b = bs.backward(only(c), K, DT / 2, 4)
        np.testing.assert_allclose(b, a * 2.0 ** power, rtol=1e-12, atol=1e-12)


def test_row_rms_step_moves_every_row_by_lr():
    U, _, _, _ = _rand(T=3, d=4, K=9, seed=5)
    g = np.random.default_rng(6).normal(size=U.shape) * np.array([1e-3, 1.0, 1e3, 1e6])[None, :, None]
    g[1, 2] = 0.0                                   # an all-zero row does not move
    U1 = bs.row_rms_step(U, g, 0.01)
    dU = U - U1
    rms = np.sqrt((dU * dU).mean(-1))
    expect = np.full(rms.shape, 0.01)
    expect[1, 2] = 0.0
    np.testing.assert_allclose(rms, expect, rtol=1e-12, atol=1e-15)
    assert np.all(np.sign(dU) == np.sign(g))        # along the gradient, row by row
