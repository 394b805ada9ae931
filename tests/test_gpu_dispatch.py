"""GPU: the per-operation calls' two forms of forward kinematics and its
adjoint -- one lane per state, and one group of lanes per state (pointer
jumping, world-frame wrenches summed over subtrees) taken for batches below
the robot's dispatch threshold -- each against the FP64 oracle on the same
robots, forced with wb_robot_set_dispatch: DFS and breadth-first link
numbering, random fixed rotations, mimic joints, the 588-sphere humanoid."""
import numpy as np
import pytest
import torch

from paper_2603_05493_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu


def _mimic_robot():
    rb = synth.random_tree(9, 3, seed=31, random_fixed_rotation=True)
    rb.joint_index = np.array([-1, 0, 1, 1, 2, 3, 4, 5, 5, 6], dtype=np.int32)
    rb.joint_mult = synth._f32([1.0, 1.0, 1.0, -0.5, 1.0, 2.0, 1.0, 1.0, 0.75, 1.0])
    rb.joint_offset = synth._f32([0.0, 0.0, 0.1, 0.25, 0.0, 0.0, -0.2, 0.0, 0.0, 0.0])
    return rb


CASES = [("chain7", lambda: synth.serial_chain(7, 5, seed=0), 500),
         ("tree20_bfs_rotated", lambda: synth.random_tree(20, 3, seed=33, random_fixed_rotation=True,
                                                          dfs_order=False), 333),
         ("humanoid48", lambda: synth.humanoid48(seed=0), 700),
         ("humanoid48_paper_scale", synth.humanoid48_paper_scale, 300),
         ("mimic_tree9", _mimic_robot, 400)]


@pytest.mark.parametrize("form", ["lane", "group"])
@pytest.mark.parametrize("label,factory,B", CASES)
def test_fk_forms_against_oracle(oracle, label, factory, B, form):
    from paper_2603_05493_amd import wb
    rb = factory()
    r = wb.Robot(rb).to_device("cuda:0")
    f = (1 << 40) if form == "group" else 0
    r.set_dispatch(-1, f, f)
    st = synth.states(rb, B, seed=3, q_range=1.5)
    q = P.dev(st.q)
    pose, sph = wb.wb_fk(r, q)
    _, sph2 = wb.wb_fk(r, q, want_pose=False)
    rng = np.random.default_rng(4)
    gc = rng.normal(size=(B, rb.n_spheres, 3))
    gR = rng.normal(size=(B, rb.n_links, 3, 3))
    gp = rng.normal(size=(B, rb.n_links, 3))
    gpose = np.concatenate([gR.reshape(B, -1, 9), gp], 2)
    g_s = wb.wb_fk_backward(r, q, g_spheres=P.dev(gc), link_pose=pose)
    g_p = wb.wb_fk_backward(r, q, g_link_pose=P.dev(gpose), link_pose=None)
    torch.cuda.synchronize()
    R, p, c = oracle.fk(rb, st.q)
    ext = P.extent(c)
    pose_h = P.host(pose)
    e_R = P.normwise(pose_h[:, :, :9], R.reshape(B, -1, 9), floor=1.0).max()
    e_p = P.scaled(pose_h[:, :, 9:], p, ext).max()
    e_c = max(P.scaled(P.host(sph), c, ext).max(), P.scaled(P.host(sph2), c, ext).max())
    ref_s = oracle.fk_backward(rb, st.q, g_spheres=gc)
    ref_p = oracle.fk_backward(rb, st.q, g_R=gR, g_p=gp)
    e_gs = P.normwise(P.host(g_s), ref_s, floor=1e-6).max()
    e_gp = P.normwise(P.host(g_p), ref_p, floor=1e-6).max()
    print(label, form, f"e_R={e_R:.3g} e_p={e_p:.3g} e_c={e_c:.3g} e_g_spheres={e_gs:.3g} e_g_pose={e_gp:.3g}",
          flush=True)
    assert max(e_R, e_p, e_c, e_gs, e_gp) < P.TOL
