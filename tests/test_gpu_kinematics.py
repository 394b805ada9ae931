"""GPU parity of the kinematics-outputs kernel (wb_kinematics,
wb_kinematics_backward): link poses, sphere centres, tool poses, centre of
mass, Alg. 2's tool Jacobians, the CoM Jacobian and the tool/CoM gradient,
against the FP64 oracle on the same FP32 robot tables.

The Jacobians are state-major on the device ([B, T, 6, n], [B, 3, n]).

Tolerances (FP32 against FP64), per state: positions and the centre of
mass scaled by the robot extent (1e-4); rotations, Jacobians and gradients
1e-4 normwise (floors 1e-3 and 1e-6).  Columns that Alg. 2's filters drop
must be exactly zero."""
import numpy as np
import pytest
import torch

from oracle import kinematics as K
from paper_2603_05493_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu


def _mimic_tree():
    rb = synth.random_tree(9, 2, seed=4)
    rb.joint_index = rb.joint_index.copy()
    rb.joint_mult = rb.joint_mult.copy()
    rb.joint_offset = rb.joint_offset.copy()
    rb.joint_index[5], rb.joint_mult[5], rb.joint_offset[5] = rb.joint_index[2], -0.7, 0.2
    rb.joint_index[8], rb.joint_mult[8], rb.joint_offset[8] = rb.joint_index[3], 1.5, 0.0
    used = sorted(set(int(j) for j in rb.joint_index if j >= 0))
    remap = {j: i for i, j in enumerate(used)}
    rb.joint_index = np.array([remap[int(j)] if j >= 0 else -1 for j in rb.joint_index], dtype=np.int32)
    rb.joint_mult, rb.joint_offset = synth._f32(rb.joint_mult), synth._f32(rb.joint_offset)
    return rb


def _mimic3_tree():
    """One joint drives three links (a longer connectedLinks list)."""
    rb = _mimic_tree()
    rb.joint_index = rb.joint_index.copy()
    rb.joint_mult = rb.joint_mult.copy()
    rb.joint_index[8], rb.joint_mult[8] = rb.joint_index[2], np.float32(0.5)
    used = sorted(set(int(j) for j in rb.joint_index if j >= 0))
    remap = {j: i for i, j in enumerate(used)}
    rb.joint_index = np.array([remap[int(j)] if j >= 0 else -1 for j in rb.joint_index], dtype=np.int32)
    return rb


def _tools(rb, links, seed):
    rng = np.random.default_rng(seed)
    Rs = []
    for _ in links:
        a = rng.normal(size=3)
        a /= np.linalg.norm(a)
        th = rng.uniform(-np.pi, np.pi)
        A = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
        Rs.append(np.eye(3) + np.sin(th) * A + (1 - np.cos(th)) * A @ A)
    return list(links), synth._f32(np.array(Rs)), synth._f32(rng.uniform(-0.1, 0.1, (len(links), 3)))


ROBOTS = [("chain7", lambda: synth.serial_chain(7, 5, seed=0), 1000),
          ("tree12", lambda: synth.random_tree(12, 6, seed=1), 777),
          ("tree23", lambda: synth.random_tree(23, 6, seed=2), 513),
          ("humanoid48", lambda: synth.humanoid48(seed=0), 1500),
          ("mimic_tree", _mimic_tree, 300),
          ("mimic3_tree", _mimic3_tree, 300),
          ("planar2r", lambda: synth.planar_2r(), 33)]


def _setup(rb, B, seed):
    from paper_2603_05493_amd import wb
    r = wb.Robot(rb).to_device("cuda:0")
    L = rb.n_links
    links, tR, tp = _tools(rb, [L - 1, L // 2, 0, 1, L - 1], seed)
    tR[4], tp[4] = tR[0], tp[0]                  # the last tool repeats the first
    r.set_tool_frames(links, tR, tp)
    st = synth.states(rb, B, seed=seed + 1)
    return r, st, links, tR, tp


def _host_sm(t):              # state-major device array -> float64 numpy, same axes
    return t.detach().cpu().numpy().astype(np.float64)


def _pose_host(t):            # [T, 12, B] -> R [B, T, 3, 3], p [B, T, 3]
    a = P.host(t)
    return a[:, :, :9].reshape(a.shape[0], a.shape[1], 3, 3), a[:, :, 9:]


@pytest.mark.parametrize("label,factory,B", ROBOTS)
def test_kinematics_outputs_match_oracle(oracle, label, factory, B):
    from paper_2603_05493_amd import wb
    rb = factory()
    r, st, links, tR, tp = _setup(rb, B, seed=20)
    out = wb.wb_kinematics(r, P.dev(st.q), link_pose=True, spheres=True, tool_pose=True, com=True,
                           jacobian=True, com_jacobian=True)
    torch.cuda.synchronize()
    R_ref, p_ref, c_ref = oracle.fk(rb, st.q)
    ext = P.extent(c_ref) if rb.n_spheres else np.linalg.norm(p_ref, axis=-1).max(-1)
    Rt_ref, xt_ref = K.tool_poses(rb, st.q, links, tR, tp)
    J_ref = K.jacobian(rb, st.q, links, tR, tp)
    Jc_ref = K.com_jacobian(rb, st.q)
    com_ref = K.center_of_mass(rb, st.q)
    lp = P.host(out["link_pose"])                                 # [B, L, 12]
    Rt, xt = _pose_host(out["tool_pose"])
    J = _host_sm(out["jacobian"])                                 # [B, T, 6, n]
    errs = dict(
        link_R=P.normwise(lp[:, :, :9], R_ref.reshape(B, -1, 9), floor=1.0).max(),
        link_p=P.scaled(lp[:, :, 9:], p_ref, ext).max(),
        spheres=P.scaled(P.host(out["spheres"]), c_ref, ext).max() if rb.n_spheres else 0.0,
        tool_R=P.normwise(Rt, Rt_ref, floor=1.0).max(),
        tool_x=P.scaled(xt, xt_ref, ext).max(),
        com=P.scaled(P.host(out["com"]), com_ref, ext).max(),
        jac=max(P.normwise(J[:, t], J_ref[:, t], floor=1e-3).max() for t in range(len(links))),
        com_jac=P.normwise(_host_sm(out["com_jacobian"]), Jc_ref, floor=1e-3).max())
    print(label, " ".join(f"{k}={v:.3g}" for k, v in errs.items()), flush=True)
    assert all(v < P.TOL for v in errs.values())
    # Alg. 2's filters: columns of joints off the chain are exactly zero
    aff = K.affects(rb, links)                                    # [n, T]
    for t in range(len(links)):
        off = ~aff[:, t]
        assert np.all(J[:, t][:, :, off] == 0.0)
    # the base tool has an all-zero Jacobian; the repeated tool repeats its rows
    assert np.all(J[:, 2] == 0.0)
    np.testing.assert_array_equal(J[:, 0], J[:, 4])


@pytest.mark.parametrize("label,factory,B", ROBOTS)
def test_kinematics_backward_matches_oracle(oracle, label, factory, B):
    from paper_2603_05493_amd import wb
    rb = factory()
    r, st, links, tR, tp = _setup(rb, B, seed=30)
    rng = np.random.default_rng(31)
    T = len(links)
    gR, gp, gc = rng.normal(size=(B, T, 3, 3)), rng.normal(size=(B, T, 3)), rng.normal(size=(B, 3))
    g_tool = synth._f32(np.concatenate([gR.reshape(B, T, 9), gp], -1))
    gc = synth._f32(gc)
    q = P.dev(st.q)
    g_q = torch.full((rb.n_dof, B), float("nan"), device="cuda")
    wb.wb_kinematics_backward(r, q, g_tool_pose=P.dev(g_tool), g_com=P.dev(gc), g_q=g_q)
    g_tool_only = wb.wb_kinematics_backward(r, q, g_tool_pose=P.dev(g_tool))
    g_com_only = wb.wb_kinematics_backward(r, q, g_com=P.dev(gc))
    torch.cuda.synchronize()
    g64 = g_tool.astype(np.float64)
    ref = K.backward(rb, st.q, links, tR, tp, g64[..., :9].reshape(B, T, 3, 3), g64[..., 9:], gc)
    ref_t = K.backward(rb, st.q, links, tR, tp, g64[..., :9].reshape(B, T, 3, 3), g64[..., 9:])
    ref_c = K.backward(rb, st.q, links, tR, tp, g_com=gc)
    e = [P.normwise(P.host(x), y, floor=1e-6).max() for x, y in ((g_q, ref), (g_tool_only, ref_t),
                                                                 (g_com_only, ref_c))]
    print(label, "backward", [f"{v:.3g}" for v in e], flush=True)
    assert max(e) < P.TOL


@pytest.mark.parametrize("B", [1, 63, 64, 65, 4097])
def test_kinematics_ragged_batches(oracle, B):
    from paper_2603_05493_amd import wb
    rb = synth.random_tree(12, 6, seed=1)
    r, st, links, tR, tp = _setup(rb, B, seed=40)
    out = wb.wb_kinematics(r, P.dev(st.q), tool_pose=True, com=True, jacobian=True)
    torch.cuda.synchronize()
    J_ref = K.jacobian(rb, st.q, links, tR, tp)
    J = _host_sm(out["jacobian"])
    assert max(P.normwise(J[:, t], J_ref[:, t], floor=1e-3).max() for t in range(len(links))) < P.TOL
    _, xt = _pose_host(out["tool_pose"])
    _, xt_ref = K.tool_poses(rb, st.q, links, tR, tp)
    assert np.abs(xt - xt_ref).max() < 1e-4 * (1.0 + np.abs(xt_ref).max())


def test_kinematics_empty_batch_and_no_tools():
    from paper_2603_05493_amd import wb
    rb = synth.serial_chain(7, 5, seed=0)
    r = wb.Robot(rb).to_device("cuda:0")
    out = wb.wb_kinematics(r, torch.empty((7, 0), device="cuda"))
    assert out["com"].shape == (3, 0)
    q = P.dev(synth.states(rb, 50, seed=1).q)
    out = wb.wb_kinematics(r, q, tool_pose=True, jacobian=True, com=False)   # no tools: nothing to write
    assert out["jacobian"].shape == (50, 0, 6, 7)
    g = wb.wb_kinematics_backward(r, q)                                      # no loss terms: zero gradient
    torch.cuda.synchronize()
    assert torch.equal(g, torch.zeros_like(g))


def test_kinematics_sees_payload_and_new_tools(oracle):
    """A payload changes the centre of mass; re-set tools replace the old ones."""
    import copy
    from paper_2603_05493_amd import wb
    rb = synth.humanoid48(seed=0)
    r, st, links, tR, tp = _setup(rb, 256, seed=50)
    q = P.dev(st.q)
    heavy = copy.deepcopy(rb)
    heavy.mass = rb.mass.copy()
    heavy.mass[30] = np.float32(rb.mass[30] + 3.0)
    r.set_link_inertia(30, float(heavy.mass[30]), rb.com[30], [rb.inertia[30][0, 0], rb.inertia[30][1, 1],
                                                             rb.inertia[30][2, 2], rb.inertia[30][0, 1],
                                                             rb.inertia[30][0, 2], rb.inertia[30][1, 2]])
    links2, tR2, tp2 = _tools(rb, [5, 17], seed=51)
    r.set_tool_frames(links2, tR2, tp2)
    out = wb.wb_kinematics(r, q, com=True, tool_pose=True, jacobian=True, com_jacobian=True)
    torch.cuda.synchronize()
    ext = P.extent(oracle.fk(rb, st.q)[2])
    assert P.scaled(P.host(out["com"]), K.center_of_mass(heavy, st.q), ext).max() < P.TOL
    assert P.scaled(P.host(out["com"]), K.center_of_mass(rb, st.q), ext).max() > 100 * P.TOL
    assert P.normwise(_host_sm(out["com_jacobian"]), K.com_jacobian(heavy, st.q), floor=1e-3).max() < P.TOL
    J = _host_sm(out["jacobian"])
    J_ref = K.jacobian(rb, st.q, links2, tR2, tp2)
    assert J.shape[1] == 2
    assert max(P.normwise(J[:, t], J_ref[:, t], floor=1e-3).max() for t in range(2)) < P.TOL


def test_kinematics_optimizer_size_sampled(oracle):
    """The humanoid at 24,576 states (the optimizer batch), sampled states
    against the oracle."""
    from paper_2603_05493_amd import wb
    rb = synth.humanoid48(seed=0)
    B = 24576
    r, st, links, tR, tp = _setup(rb, B, seed=60)
    out = wb.wb_kinematics(r, P.dev(st.q), tool_pose=True, com=True, jacobian=True, com_jacobian=True)
    torch.cuda.synchronize()
    idx = np.random.default_rng(61).choice(B, 300, replace=False)
    q = st.q[idx]
    J = _host_sm(out["jacobian"])[idx]
    J_ref = K.jacobian(rb, q, links, tR, tp)
    assert max(P.normwise(J[:, t], J_ref[:, t], floor=1e-3).max() for t in range(len(links))) < P.TOL
    assert P.normwise(_host_sm(out["com_jacobian"])[idx], K.com_jacobian(rb, q), floor=1e-3).max() < P.TOL


def test_kinematics_rejects_bad_arguments():
    from paper_2603_05493_amd import _abi, wb
    rb = synth.serial_chain(5, 2, seed=0)
    r = wb.Robot(rb).to_device("cuda:0")
    bad = [([9], None, None), ([1] * 33, None, None), ([1], np.full((1, 3, 3), 2.0), None),
           ([1], None, np.array([[0.0, np.nan, 0.0]]))]
    for links, R, p in bad:
        with pytest.raises(_abi.WbError):
            r.set_tool_frames(links, R, p)
    q = torch.zeros((5, 8), device="cuda")
    assert wb.wb_kinematics(r, q, tool_pose=False, com=False, jacobian=False) == {}   # nothing requested
    light = synth.serial_chain(5, 2, seed=0)
    light.mass = np.zeros_like(light.mass)
    r0 = wb.Robot(light).to_device("cuda:0")
    with pytest.raises(_abi.WbError):
        wb.wb_kinematics(r0, q, com=True, jacobian=False, tool_pose=False)
    big = synth.random_tree(70, 1, seed=3)
    rbig = wb.Robot(big).to_device("cuda:0")
    assert not rbig.kinematics_supported
    with pytest.raises(_abi.WbError):
        wb.wb_kinematics(rbig, torch.zeros((big.n_dof, 4), device="cuda"))
