"""Pins for the oracle's forward kinematics and its adjoint.

The paper prints no numeric FK example, so the oracle is pinned to closed
forms (planar two-link arm), to a composition built from scipy's rotation
routine, to rotation-group invariants, and to central finite differences.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2603_05493_amd import synth


def _robots():
    return [synth.serial_chain(7, 5, seed=3, random_fixed_rotation=True),
            synth.random_tree(12, 3, seed=4, random_fixed_rotation=True),
            synth.humanoid48(seed=1)]


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_rotations_orthonormal(oracle, idx):
    rb = _robots()[idx]
    st = synth.states(rb, 8, seed=idx)
    R, _, _ = oracle.fk(rb, st.q)
    RtR = np.einsum("blji,bljk->blik", R, R)
    # inputs are float32-rounded (axes and fixed rotations unit/orthonormal to ~1e-7)
    assert np.abs(RtR - np.eye(3)).max() < 2e-6
    assert np.abs(np.linalg.det(R) - 1.0).max() < 2e-6


def test_planar_2r_closed_form(oracle):
    rb = synth.planar_2r(l1=0.5, l2=0.4)
    rng = np.random.default_rng(0)
    q = rng.uniform(-np.pi, np.pi, size=(16, 2))
    R, p, c = oracle.fk(rb, q)
    q1, q2 = q[:, 0], q[:, 1]
    l1, l2 = rb.fixed_p[2, 0], rb.sphere_pos[1, 0]   # 0.5 and 0.4 as float32 values
    elbow = np.stack([l1 * np.cos(q1), l1 * np.sin(q1), 0 * q1], 1)
    tip = elbow + np.stack([l2 * np.cos(q1 + q2), l2 * np.sin(q1 + q2), 0 * q1], 1)
    np.testing.assert_allclose(p[:, 2], elbow, atol=1e-12)
    np.testing.assert_allclose(c[:, 1], tip, atol=1e-12)
    np.testing.assert_allclose(c[:, 0], elbow, atol=1e-12)
    # orientation of link 2 is a z-rotation by q1 + q2
    for b in range(16):
        np.testing.assert_allclose(R[b, 2], Rotation.from_euler("z", q1[b] + q2[b]).as_matrix(),
                                   atol=1e-12)


def test_chain_matches_scipy_composition(oracle):
    """Compose the chain with scipy's axis-angle rotations and numpy products."""
    rb = synth.serial_chain(7, 5, seed=5, random_fixed_rotation=True)
    st = synth.states(rb, 6, seed=2)
    R, p, c = oracle.fk(rb, st.q)
    for b in range(6):
        Rw, pw = np.eye(3), np.zeros(3)
        for k in range(1, rb.n_links):
            Rj = Rotation.from_rotvec(rb.axis[k] / np.linalg.norm(rb.axis[k]) *
                                      st.q[b, rb.joint_index[k]]).as_matrix()
            pw = Rw @ rb.fixed_p[k] + pw
            Rw = Rw @ rb.fixed_R[k] @ Rj
            np.testing.assert_allclose(R[b, k], Rw, atol=1e-6)
            np.testing.assert_allclose(p[b, k], pw, atol=1e-6)
        s = np.where(rb.sphere_link == rb.n_links - 1)[0][0]
        np.testing.assert_allclose(c[b, s], Rw @ rb.sphere_pos[s] + pw, atol=1e-6)


def test_single_joint_is_rodrigues(oracle):
    rb = synth.serial_chain(1, 1, seed=9, random_fixed_rotation=True)
    q = np.linspace(-3, 3, 13)[:, None]
    R, _, _ = oracle.fk(rb, q)
    ax = rb.axis[1] / np.linalg.norm(rb.axis[1])
    for b in range(13):
        ref = rb.fixed_R[1] @ Rotation.from_rotvec(ax * q[b, 0]).as_matrix()
        np.testing.assert_allclose(R[b, 1], ref, atol=2e-7)


def _fd_fk_backward(oracle, rb, q, gc, gR, gp, h=1e-6):
    n = q.shape[1]
    out = np.zeros_like(q)
    for j in range(n):
        e = np.zeros(n)
        e[j] = h
        Rp, pp, cp = oracle.fk(rb, q + e)
        Rm, pm, cm = oracle.fk(rb, q - e)
        out[:, j] = (np.sum(gc * (cp - cm), axis=(1, 2)) + np.sum(gR * (Rp - Rm), axis=(1, 2, 3)) +
                     np.sum(gp * (pp - pm), axis=(1, 2))) / (2 * h)
    return out


@pytest.mark.parametrize("idx", [0, 1, 2])
def test_fk_backward_matches_fd(oracle, idx):
    rb = _robots()[idx]
    B = 4
    st = synth.states(rb, B, seed=11)
    rng = np.random.default_rng(7)
    gc = rng.normal(size=(B, rb.n_spheres, 3))
    gR = rng.normal(size=(B, rb.n_links, 3, 3))
    gp = rng.normal(size=(B, rb.n_links, 3))
    ana = oracle.fk_backward(rb, st.q, g_spheres=gc, g_R=gR, g_p=gp)
    fd = _fd_fk_backward(oracle, rb, st.q, gc, gR, gp)
    np.testing.assert_allclose(ana, fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max())
    # each gradient source alone
    ana_c = oracle.fk_backward(rb, st.q, g_spheres=gc)
    fd_c = _fd_fk_backward(oracle, rb, st.q, gc, 0 * gR, 0 * gp)
    np.testing.assert_allclose(ana_c, fd_c, rtol=1e-6, atol=1e-6 * np.abs(fd_c).max())


def test_mimic_joint_fk_equals_expanded(oracle):
    """A link driven as m*q_j + o equals an independent joint set to that angle."""
    rb = synth.serial_chain(4, 2, seed=2)
    mim = synth.serial_chain(4, 2, seed=2)
    mim.joint_index = np.array([-1, 0, 1, 1, 2], dtype=np.int32)
    mim.joint_mult = np.array([1.0, 1.0, 1.0, -0.5, 2.0])
    mim.joint_offset = np.array([0.0, 0.0, 0.0, 0.25, 0.0])
    st = synth.states(mim, 5, seed=3)
    qx = np.stack([st.q[:, 0], st.q[:, 1], -0.5 * st.q[:, 1] + 0.25, 2.0 * st.q[:, 2]], 1)
    _, _, c_m = oracle.fk(mim, st.q)
    _, _, c_x = oracle.fk(rb, qx)
    np.testing.assert_allclose(c_m, c_x, atol=1e-12)
