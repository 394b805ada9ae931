"""GPU parity of wb_self_collision's two forms -- one state per wavefront,
and one state per workgroup with its link blocks dealt over four
wavefronts and a second reduce through LDS (the paper's two-stage
map-reduce for large pair sets) -- against the FP64 oracle and against each
other, including the paper-scale humanoid (588 spheres, 162,432 checked
pairs, up to 12 spheres per link) at the paper's kinematics batch of 1000
states and at one GPU's 3072-state share.

max_pen is compared scaled by the robot's extent; argmax exactly wherever
the oracle's maximum beats the runner-up by DELTA; counts within the DELTA
band.  The two forms evaluate every pair with the same arithmetic and both
sweep every pair that can matter, so their three outputs agree bit for bit."""
import numpy as np
import pytest
import torch

from paper_2603_05493_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu


def _robot(rb):
    from paper_2603_05493_amd import wb
    return wb.Robot(rb).to_device("cuda:0")


def _small_radius_humanoid():
    rb = synth.humanoid48(seed=4)
    rb.sphere_r = synth._f32(rb.sphere_r * 0.3)
    return rb


def _sweep(r, sph, split):
    from paper_2603_05493_amd import wb
    r.set_sweep_split(1 << 40 if split else 0)
    out = wb.wb_self_collision(r, sph)
    r.set_sweep_split(-1)
    return out


def _oracle_check(O, rb, c, mp, am, nc, label):
    pens = O.self_collision_pens(rb, c)
    ext = P.extent(c)
    mp_ref = pens.max(1) if pens.shape[1] else np.full(len(c), -np.inf)
    e_mp = P.scaled(mp[:, None], mp_ref[:, None], ext).max()
    amb = P.unambiguous(pens)
    lo, hi = P.count_band(pens)
    am_ref = np.argmax(pens, 1)
    print(label, f"e_mp={e_mp:.3g} banded={int((~amb).sum())} of {len(c)}", flush=True)
    assert e_mp < P.TOL
    np.testing.assert_array_equal(am[amb], am_ref[amb])
    assert np.all((nc >= lo) & (nc <= hi))


CASES = [("chain7", lambda: synth.serial_chain(7, 5, seed=0), 777, np.pi),
         ("humanoid48", lambda: synth.humanoid48(seed=0), 1000, 1.5),
         ("humanoid48_small_r", _small_radius_humanoid, 700, 1.5),
         ("tree48", lambda: synth.random_tree(48, 6, seed=3), 300, np.pi),
         ("humanoid48_paper_scale", synth.humanoid48_paper_scale, 300, 1.5)]


@pytest.mark.parametrize("label,factory,B,qr", CASES)
def test_both_forms_agree_and_match_oracle(oracle, label, factory, B, qr):
    from paper_2603_05493_amd import wb
    rb = factory()
    r = _robot(rb)
    st = synth.states(rb, B, seed=23, q_range=qr)
    _, sph = wb.wb_fk(r, P.dev(st.q), want_pose=False)
    a = _sweep(r, sph, split=False)
    b = _sweep(r, sph, split=True)
    torch.cuda.synchronize()
    for x, y, nm in zip(a, b, ("max_pen", "argmax", "n_coll")):
        assert torch.equal(x, y), f"{label}: {nm} differs between the two forms"
    _, _, c = oracle.fk(rb, st.q)
    mp, am, nc = (t.cpu().numpy() for t in b)
    _oracle_check(oracle, rb, c, mp.astype(np.float64), am, nc, label)


def test_exact_tie_and_no_pairs_in_the_split_form(oracle):
    from paper_2603_05493_amd import wb
    L = 4
    z = np.zeros((L, 3))
    fp = np.array([[0, 0, 0], [0.125, 0, 0], [-0.125, 0, 0], [0, 0, 0.0625]])
    axis = np.tile([0.0, 0.0, 1.0], (L, 1))
    inertia = np.tile(np.eye(3) * 1e-3, (L, 1, 1))
    rb = synth._finish("tie", 0, [-1, 0, 0, 0], axis, np.tile(np.eye(3), (L, 1, 1)), fp,
                       np.ones(L), z, inertia, [1, 2, 3], np.zeros((3, 3)), np.full(3, 0.0875))
    r = _robot(rb)
    q = torch.zeros((3, 130), device="cuda")
    _, sph = wb.wb_fk(r, q)
    mp, am, nc = _sweep(r, sph, split=True)
    torch.cuda.synchronize()
    assert np.all(am.cpu().numpy() == 1) and np.all(nc.cpu().numpy() == 2)   # pairs (1,3) and (2,3) tie
    rb2 = synth.serial_chain(1, 3, seed=0)
    r2 = _robot(rb2)
    _, sph2 = wb.wb_fk(r2, torch.zeros((1, 70), device="cuda"))
    mp2, am2, nc2 = _sweep(r2, sph2, split=True)
    torch.cuda.synchronize()
    assert torch.isneginf(mp2).all() and (am2 == -1).all() and (nc2 == 0).all()


@pytest.mark.parametrize("B", [1000, 3072])
def test_paper_scale_humanoid_at_the_papers_batches(oracle, B):
    """The 162k-pair humanoid at batch 1000 (the paper's kinematics and
    self-collision benchmark) and 3072, in the form the library picks for
    that batch, on 256 sampled states; every state's result is also
    compared with the other form bit for bit."""
    from paper_2603_05493_amd import wb
    rb = synth.humanoid48_paper_scale()
    r = _robot(rb)
    assert r.n_pairs == 162432 and r.max_spheres_per_link == 12
    st = synth.states(rb, B, seed=29, q_range=1.5)
    _, sph = wb.wb_fk(r, P.dev(st.q), want_pose=False)
    mp, am, nc = wb.wb_self_collision(r, sph)
    other = _sweep(r, sph, split=False)
    torch.cuda.synchronize()
    for x, y in zip((mp, am, nc), other):
        assert torch.equal(x, y)
    sample = np.sort(np.random.default_rng(31).choice(B, 256, replace=False))
    _, _, c = oracle.fk(rb, st.q[sample])
    h = lambda t: t.cpu().numpy()[sample]
    _oracle_check(oracle, rb, c, h(mp).astype(np.float64), h(am), h(nc), f"paper-scale humanoid B={B}")


def test_paper_scale_forward_backward(oracle):
    """FK -> self-collision -> hinge adjoint -> FK adjoint on the 162k-pair
    humanoid (the plain per-operation launches; the fused iteration takes up
    to 8 spheres per link), against the oracle's gradient for the GPU's
    argmax choice on every state."""
    from paper_2603_05493_amd import wb
    rb = synth.humanoid48_paper_scale()
    r = _robot(rb)
    B = 256
    st = synth.states(rb, B, seed=37, q_range=1.5)
    q = P.dev(st.q)
    pose, sph = wb.wb_fk(r, q)
    mp, am, nc = wb.wb_self_collision(r, sph)
    g_cost = torch.ones(B, device="cuda")
    g_sph = wb.wb_self_collision_backward(r, sph, am, mp, 0.01, g_cost)
    g_q = wb.wb_fk_backward(r, q, g_spheres=g_sph, link_pose=pose)
    torch.cuda.synchronize()
    _, _, c = oracle.fk(rb, st.q)
    mp_ref, am_ref, _ = oracle.self_collision(rb, c)
    ref = dict(c=c, max_pen=mp_ref, argmax=am_ref, g_q_rnea=np.zeros((B, rb.n_dof)))
    got = P.host(g_q)
    g_ref, tied, kink, alt = P.reference_gq(oracle, rb, st.q, ref, got, am.cpu().numpy(), 0.01)
    # This is the hinge's FK gradient alone, with no torque term to share the
    # scale: for the joints above both spheres of the pair the exact value is
    # 0 (the two forces are equal, opposite and collinear) and FP32 leaves
    # noise of order eps |c| |g| there, so its scale is floored at 1 % of the
    # robot's extent times the hinge weight, as for the plain form's FK-adjoint
    # stage check; the states the floor decides are counted.
    e_plain = P.normwise(got, g_ref, floor=1e-6)
    e = P.normwise(got, g_ref, floor=P.fk_grad_floor(dict(c=c)))
    print("paper-scale humanoid hinge gradient: max err", float(e.max()), "(without the floor",
          float(e_plain.max()), ") floor decided", int(((e_plain > P.TOL) & (e <= P.TOL)).sum()), "of", B,
          "tied", int(tied.sum()), "kink", int(kink.sum()), flush=True)
    assert np.all(e <= P.TOL)
