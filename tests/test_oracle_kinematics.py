"""Pins of the kinematics oracle (tool poses, centre of mass, Alg. 2's
Jacobian, the CoM Jacobian and the tool/CoM gradient) against what the
mathematics fixes: central finite differences of the oracle's forward
kinematics, the closed form of the planar two-link arm, the static gravity
torque of the RNEA oracle, and Alg. 2's sparsity."""
import numpy as np
import pytest

from oracle import kinematics as K
from paper_2603_05493_amd import synth


def _tools(rb, links, seed):
    rng = np.random.default_rng(seed)
    Rs = []
    for _ in links:
        a = rng.normal(size=3)
        a /= np.linalg.norm(a)
        th = rng.uniform(-np.pi, np.pi)
        A = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
        Rs.append(np.eye(3) + np.sin(th) * A + (1 - np.cos(th)) * A @ A)
    return list(links), np.array(Rs), rng.uniform(-0.1, 0.1, (len(links), 3))


def _mimic_tree():
    rb = synth.random_tree(9, 2, seed=4)
    rb.joint_index = rb.joint_index.copy()
    rb.joint_mult = rb.joint_mult.copy()
    rb.joint_offset = rb.joint_offset.copy()
    # links 5 and 8 follow joints 1 and 2 with a gain and an offset
    rb.joint_index[5], rb.joint_mult[5], rb.joint_offset[5] = rb.joint_index[2], -0.7, 0.2
    rb.joint_index[8], rb.joint_mult[8], rb.joint_offset[8] = rb.joint_index[3], 1.5, 0.0
    used = sorted(set(int(j) for j in rb.joint_index if j >= 0))
    remap = {j: i for i, j in enumerate(used)}
    rb.joint_index = np.array([remap[int(j)] if j >= 0 else -1 for j in rb.joint_index], dtype=np.int32)
    return rb


def _exact(rb):
    """The robot with its FP32-rounded fixed rotations replaced by the nearest
    rotations and its axes by unit vectors, in FP64: the Jacobian's
    [s x (x - o); s] is the derivative of FK only for orthonormal frames, and
    FP32 rounding leaves an O(1e-7) difference that would mask errors."""
    U, _, Vt = np.linalg.svd(np.asarray(rb.fixed_R, float))
    rb.fixed_R = U @ Vt
    ax = np.asarray(rb.axis, float)
    rb.axis = ax / np.linalg.norm(ax, axis=1, keepdims=True)
    return rb


ROBOTS = [("chain7", lambda: _exact(synth.serial_chain(7, 2, seed=0))),
          ("tree12", lambda: _exact(synth.random_tree(12, 2, seed=1))),
          ("humanoid48", lambda: _exact(synth.humanoid48(seed=0))),
          ("mimic_tree", lambda: _exact(_mimic_tree()))]


def _tool_links(rb):
    L = rb.n_links
    return [L - 1, L // 2, 1, 0, L - 1]      # the same link twice, the base, a first-level link


def _vee(W):
    return np.stack([W[..., 2, 1] - W[..., 1, 2], W[..., 0, 2] - W[..., 2, 0], W[..., 1, 0] - W[..., 0, 1]], -1) / 2


@pytest.mark.parametrize("label,factory", ROBOTS)
def test_jacobian_matches_central_differences(oracle, label, factory):
    """Column j is d(x)/dq_j for the tool point and vee(dR/dq_j R^T) for the
    tool orientation, differenced through the oracle's forward kinematics."""
    rb = factory()
    links, tR, tp = _tools(rb, _tool_links(rb), seed=3)
    st = synth.states(rb, 3, seed=7)
    J = K.jacobian(rb, st.q, links, tR, tp)
    h = 1e-6
    for j in range(rb.n_dof):
        dq = np.zeros(rb.n_dof)
        dq[j] = h
        Rp, xp = K.tool_poses(rb, st.q + dq, links, tR, tp)
        Rm, xm = K.tool_poses(rb, st.q - dq, links, tR, tp)
        R0, _ = K.tool_poses(rb, st.q, links, tR, tp)
        lin = (xp - xm) / (2 * h)
        ang = _vee((Rp - Rm) / (2 * h) @ np.swapaxes(R0, -1, -2))
        np.testing.assert_allclose(J[..., :3, j], lin, atol=1e-9)
        np.testing.assert_allclose(J[..., 3:, j], ang, atol=1e-9)


def test_jacobian_sparsity_follows_the_chain():
    """Alg. 2's filters: a column is exactly zero unless the joint drives a
    link on the tool link's chain; for a humanoid hand that is the torso and
    that arm only."""
    rb = synth.humanoid48(seed=0)
    L = rb.n_links
    links, tR, tp = _tools(rb, list(range(L)), seed=5)
    st = synth.states(rb, 2, seed=8)
    J = K.jacobian(rb, st.q, links, tR, tp)
    aff = K.affects(rb, links)
    nz = np.abs(J).max(axis=(0, 2)) > 0                   # [T, n]
    np.testing.assert_array_equal(nz, aff.T)
    for e in range(L):
        chain = K.link_chain(rb, e)
        expect = sorted(int(rb.joint_index[k]) for k in chain if k > 0 and rb.joint_index[k] >= 0)
        assert sorted(np.nonzero(aff[:, e])[0].tolist()) == expect
    per_tool = aff.sum(0)
    assert per_tool[0] == 0                                   # nothing moves the base
    assert per_tool[1:].min() > 0 and per_tool.max() < rb.n_dof   # no link lies below every joint


def test_planar_2r_tool_point_closed_form():
    """A tool a distance d further along the second link of the planar arm:
    x = l1 c1 + (l2 + d) c12, y = l1 s1 + (l2 + d) s12, its Jacobian the
    textbook one, and the angular rows the z axis for both joints."""
    rb = synth.planar_2r(l1=0.5, l2=0.4)
    l1 = float(rb.fixed_p[2, 0])
    d = 0.55
    rng = np.random.default_rng(0)
    q = rng.uniform(-np.pi, np.pi, (16, 2))
    R, x = K.tool_poses(rb, q, [2], np.eye(3)[None], np.array([[d, 0, 0]]))
    J = K.jacobian(rb, q, [2], np.eye(3)[None], np.array([[d, 0, 0]]))[:, 0]
    c1, s1 = np.cos(q[:, 0]), np.sin(q[:, 0])
    c12, s12 = np.cos(q.sum(1)), np.sin(q.sum(1))
    np.testing.assert_allclose(x[:, 0, 0], l1 * c1 + d * c12, atol=1e-12)
    np.testing.assert_allclose(x[:, 0, 1], l1 * s1 + d * s12, atol=1e-12)
    np.testing.assert_allclose(R[:, 0, :2, :2], np.stack([np.stack([c12, -s12], -1), np.stack([s12, c12], -1)], -2),
                               atol=1e-12)
    np.testing.assert_allclose(J[:, 0, 0], -l1 * s1 - d * s12, atol=1e-12)
    np.testing.assert_allclose(J[:, 0, 1], -d * s12, atol=1e-12)
    np.testing.assert_allclose(J[:, 1, 0], l1 * c1 + d * c12, atol=1e-12)
    np.testing.assert_allclose(J[:, 1, 1], d * c12, atol=1e-12)
    np.testing.assert_allclose(J[:, 2], 0.0, atol=1e-15)
    np.testing.assert_allclose(J[:, 5], 1.0, atol=1e-15)
    np.testing.assert_allclose(J[:, 3:5], 0.0, atol=1e-15)


def test_planar_2r_centre_of_mass_closed_form():
    rb = synth.planar_2r(l1=0.5, l2=0.4, m1=1.0, m2=0.7)
    l1 = float(rb.fixed_p[2, 0])
    a1, a2 = float(rb.com[1, 0]), float(rb.com[2, 0])
    m1, m2 = float(rb.mass[1]), float(rb.mass[2])
    rng = np.random.default_rng(1)
    q = rng.uniform(-np.pi, np.pi, (16, 2))
    c1, s1 = np.cos(q[:, 0]), np.sin(q[:, 0])
    c12, s12 = np.cos(q.sum(1)), np.sin(q.sum(1))
    x = (m1 * a1 * c1 + m2 * (l1 * c1 + a2 * c12)) / (m1 + m2)
    y = (m1 * a1 * s1 + m2 * (l1 * s1 + a2 * s12)) / (m1 + m2)
    com = K.center_of_mass(rb, q)
    np.testing.assert_allclose(com[:, 0], x, atol=1e-12)
    np.testing.assert_allclose(com[:, 1], y, atol=1e-12)
    np.testing.assert_allclose(com[:, 2], 0.0, atol=1e-15)


@pytest.mark.parametrize("label,factory", [ROBOTS[0], ("planar2r", lambda: synth.planar_2r()),
                                           ("chain3", lambda: _exact(synth.serial_chain(3, 1, seed=5)))])
def test_com_matches_static_gravity_torque(oracle, label, factory):
    """At rest, the torque at a joint holding its subtree against gravity is
    s . ((C - M o) x (-g)) with M and C the subtree's mass and first moment;
    for a first-level joint whose subtree is everything but the base, C is
    M_total com - m_0 c_0.  The torque comes from the RNEA oracle, a separate
    computation."""
    rb = factory()
    children = [k for k in range(1, rb.n_links) if rb.parent[k] == 0]
    assert len(children) == 1
    k1 = children[0]
    st = synth.states(rb, 4, seed=9)
    z = np.zeros_like(st.q)
    tau = oracle.rnea(rb, st.q, z, z)
    R, p, _ = oracle.fk(rb, st.q)
    m = np.asarray(rb.mass, float)
    M = m.sum()
    com = K.center_of_mass(rb, st.q)
    c0 = R[:, 0] @ np.asarray(rb.com[0], float) + p[:, 0]
    C = M * com - m[0] * c0
    s = np.einsum("bij,j->bi", R[:, k1], np.asarray(rb.axis[k1], float))
    g = np.asarray(rb.gravity, float)
    expect = np.einsum("bi,bi->b", s, np.cross(C - (M - m[0]) * p[:, k1], -g))
    np.testing.assert_allclose(tau[:, int(rb.joint_index[k1])], expect, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("label,factory", ROBOTS)
def test_com_jacobian_matches_central_differences(oracle, label, factory):
    rb = factory()
    st = synth.states(rb, 3, seed=10)
    Jc = K.com_jacobian(rb, st.q)
    h = 1e-6
    for j in range(rb.n_dof):
        dq = np.zeros(rb.n_dof)
        dq[j] = h
        fd = (K.center_of_mass(rb, st.q + dq) - K.center_of_mass(rb, st.q - dq)) / (2 * h)
        np.testing.assert_allclose(Jc[:, :, j], fd, atol=1e-9)


@pytest.mark.parametrize("label,factory", ROBOTS)
def test_backward_matches_central_differences(oracle, label, factory):
    rb = factory()
    links, tR, tp = _tools(rb, _tool_links(rb), seed=11)
    st = synth.states(rb, 2, seed=12)
    rng = np.random.default_rng(13)
    T = len(links)
    gR, gp, gc = rng.normal(size=(2, T, 3, 3)), rng.normal(size=(2, T, 3)), rng.normal(size=(2, 3))

    def loss(q):
        R, x = K.tool_poses(rb, q, links, tR, tp)
        return (np.sum(gR * R, axis=(1, 2, 3)) + np.sum(gp * x, axis=(1, 2))
                + np.sum(gc * K.center_of_mass(rb, q), 1))

    g = K.backward(rb, st.q, links, tR, tp, gR, gp, gc)
    h = 1e-6
    for j in range(rb.n_dof):
        dq = np.zeros(rb.n_dof)
        dq[j] = h
        np.testing.assert_allclose(g[:, j], (loss(st.q + dq) - loss(st.q - dq)) / (2 * h), rtol=1e-8, atol=1e-8)
    # each source alone
    g_only = K.backward(rb, st.q, links, tR, tp, g_com=gc)
    np.testing.assert_allclose(g_only, np.einsum("bij,bi->bj", K.com_jacobian(rb, st.q), gc), atol=1e-14)


def test_mimic_column_sums_the_driven_links():
    """A mimic joint's column is the multiplier-weighted sum of the columns the
    driven links would have as independent joints."""
    mim = _mimic_tree()
    indep = synth.random_tree(9, 2, seed=4)
    st = synth.states(mim, 3, seed=14)
    # the independent tree's angles that reproduce the mimic tree's links
    ang = np.zeros((3, indep.n_dof))
    for k in range(1, mim.n_links):
        if mim.joint_index[k] >= 0:
            ang[:, indep.joint_index[k]] = (mim.joint_mult[k] * st.q[:, mim.joint_index[k]]
                                            + mim.joint_offset[k])
    links, tR, tp = _tools(mim, [mim.n_links - 1, 6, 8], seed=15)
    Jm = K.jacobian(mim, st.q, links, tR, tp)
    Ji = K.jacobian(indep, ang, links, tR, tp)
    expect = np.zeros_like(Jm)
    for k in range(1, mim.n_links):
        if mim.joint_index[k] >= 0:
            expect[..., mim.joint_index[k]] += mim.joint_mult[k] * Ji[..., indep.joint_index[k]]
    np.testing.assert_allclose(Jm, expect, atol=1e-12)


def test_massless_robot_has_no_centre_of_mass():
    rb = synth.serial_chain(3, 1, seed=0)
    rb.mass = np.zeros_like(rb.mass)
    with pytest.raises(ValueError):
        K.center_of_mass(rb, np.zeros((1, 3)))
