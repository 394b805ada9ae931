"""Kinetic and potential energy of a robot from forward kinematics only.

Used to pin the oracle's inverse dynamics against the physics definitions
(Lagrangian mechanics) rather than against its own recursion: link
velocities come from central finite differences of the oracle's FK, and the
energies are the textbook sums over rigid bodies.
"""
import numpy as np


def _vee(W):
    return np.array([W[2, 1] - W[1, 2], W[0, 2] - W[2, 0], W[1, 0] - W[0, 1]]) * 0.5


def com_world(O, rb, q):
    R, p, _ = O.fk(rb, q[None])
    return np.einsum("lij,lj->li", R[0], rb.com) + p[0], R[0]


def potential(O, rb, q):
    """PE = -sum_k m_k g . c_k (g is the gravity vector)."""
    c, _ = com_world(O, rb, q)
    return -float(np.sum(rb.mass * (c @ rb.gravity)))


def kinetic(O, rb, q, qd, h=1e-6):
    """KE = 1/2 sum_k (m_k |dc_k/dt|^2 + w_k^T R_k Ic_k R_k^T w_k), velocities by FD of FK."""
    cp, Rp = com_world(O, rb, q + h * qd)
    cm, Rm = com_world(O, rb, q - h * qd)
    c0, R0 = com_world(O, rb, q)
    vc = (cp - cm) / (2 * h)
    ke = 0.0
    for k in range(rb.parent.shape[0]):
        Rdot = (Rp[k] - Rm[k]) / (2 * h)
        w = _vee(Rdot @ R0[k].T)
        Iw = R0[k] @ rb.inertia[k] @ R0[k].T
        ke += 0.5 * (rb.mass[k] * vc[k] @ vc[k] + w @ Iw @ w)
    return ke


def mass_matrix(O, rb, q):
    """M = d^2 KE / d qd^2 by polarization (exact: KE is quadratic in qd)."""
    n = q.shape[0]
    E = np.eye(n)
    ke1 = [kinetic(O, rb, q, E[i]) for i in range(n)]
    M = np.zeros((n, n))
    for i in range(n):
        M[i, i] = 2.0 * ke1[i]
        for j in range(i + 1, n):
            M[i, j] = M[j, i] = kinetic(O, rb, q, E[i] + E[j]) - ke1[i] - ke1[j]
    return M
