"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded
inputs (see tests/parity.py for the tolerance rules).  Sizes span several
workgroup tiles and a ragged tail; the full-size optimizer workload is
checked on sampled states."""
import numpy as np
import pytest
import torch

from paper_2603_05493_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu


def _wb():
    from paper_2603_05493_amd import wb
    return wb


_robots_cache = {}


def _dev_robot(rb):
    key = id(rb)
    if key not in _robots_cache:
        _robots_cache[key] = (rb, _wb().Robot(rb).to_device("cuda:0"))
    return _robots_cache[key][1]


def _log(name, **kv):
    print(name, " ".join(f"{k}={v:.3g}" if isinstance(v, float) else f"{k}={v}" for k, v in kv.items()),
          flush=True)


def _check_forward(O, rb, st, label):
    wb = _wb()
    r = _dev_robot(rb)
    q, qd, qdd = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
    pose, sph = wb.wb_fk(r, q)
    mp, am, nc = wb.wb_self_collision(r, sph)
    tau, cache = wb.wb_rnea(r, q, qd, qdd)
    torch.cuda.synchronize()
    R, p, c = O.fk(rb, st.q)
    ext = P.extent(c)
    pose_h = P.host(pose)                       # [B, L, 12]
    e_R = P.normwise(pose_h[:, :, :9], R.reshape(st.B, -1, 9), floor=1.0).max()
    e_p = P.scaled(pose_h[:, :, 9:], p, ext).max()
    e_c = P.scaled(P.host(sph), c, ext).max()
    tau_ref = O.rnea(rb, st.q, st.qd, st.qdd)
    e_t = P.normwise(P.host(tau), tau_ref, floor=1e-3).max()
    mp_ref, am_ref, nc_ref = O.self_collision(rb, c)
    _log(label, e_R=e_R, e_p=e_p, e_c=e_c, e_tau=e_t)
    assert e_R < P.TOL and e_p < P.TOL and e_c < P.TOL and e_t < P.TOL
    if r.n_pairs:
        pens = O.self_collision_pens(rb, c)
        e_mp = P.scaled(P.host(mp), mp_ref, ext).max()
        ok = P.unambiguous(pens)
        am_h = am.cpu().numpy()
        lo, hi = P.count_band(pens)
        nc_h = nc.cpu().numpy()
        _log(label + " selfcoll", e_mp=e_mp, banded=int((~ok).sum()), B=st.B)
        assert e_mp < P.TOL
        np.testing.assert_array_equal(am_h[ok], am_ref[ok])
        assert np.all((nc_h >= lo) & (nc_h <= hi))
        # stage-isolated: the GPU's own sphere centres through the FP64 sweep
        mp_s, am_s, nc_s = O.self_collision(rb, P.host(sph))
        pens_s = O.self_collision_pens(rb, P.host(sph))
        ok_s = P.unambiguous(pens_s, 1e-6)
        np.testing.assert_array_equal(am_h[ok_s], am_s[ok_s])
        assert np.abs(P.host(mp) - mp_s).max() < 1e-6
    else:
        assert np.all(np.isneginf(P.host(mp))) and np.all(am.cpu().numpy() == -1)
        assert np.all(nc.cpu().numpy() == 0)


@pytest.mark.parametrize("label,factory,B,qr", [
    ("chain7_B32", lambda: synth.serial_chain(7, 5, seed=0), 32, np.pi),
    ("chain7_B4096", lambda: synth.serial_chain(7, 5, seed=0), 4096, np.pi),
    ("humanoid48_B2048", lambda: synth.humanoid48(seed=0), 2048, 1.5),
    ("tree7_B8192", lambda: synth.random_tree(7, 6, seed=0), 8192, np.pi),
    ("tree12_B4096", lambda: synth.random_tree(12, 6, seed=1), 4096, np.pi),
    ("tree23_B2048", lambda: synth.random_tree(23, 6, seed=2), 2048, np.pi),
    ("tree48_B1024", lambda: synth.random_tree(48, 6, seed=3), 1024, np.pi),
])
def test_forward_parity(oracle, label, factory, B, qr):
    rb = factory()
    st = synth.states(rb, B, seed=11, q_range=qr)
    _check_forward(oracle, rb, st, label)


@pytest.mark.parametrize("B", [1, 17, 63, 65, 1000])
def test_forward_ragged_batches(oracle, B):
    rb = synth.humanoid48(seed=1)
    _check_forward(oracle, rb, synth.states(rb, B, seed=B, q_range=1.5), f"humanoid_ragged_B{B}")


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
def test_forward_spheres_per_link(oracle, k):
    rb = synth.random_tree(10, k, seed=20 + k, random_fixed_rotation=True)
    _check_forward(oracle, rb, synth.states(rb, 300, seed=k), f"tree10_k{k}")


def _mimic_robot():
    rb = synth.random_tree(9, 3, seed=31, random_fixed_rotation=True)
    rb.joint_index = np.array([-1, 0, 1, 1, 2, 3, 4, 5, 5, 6], dtype=np.int32)
    rb.joint_mult = np.array([1.0, 1.0, 1.0, -0.5, 1.0, 2.0, 1.0, 1.0, 0.75, 1.0])
    rb.joint_offset = np.array([0.0, 0.0, 0.1, 0.25, 0.0, 0.0, -0.2, 0.0, 0.0, 0.0])
    return rb


def test_forward_mimic_joints(oracle):
    rb = _mimic_robot()
    _check_forward(oracle, rb, synth.states(rb, 500, seed=3), "mimic_tree9")


def test_forward_explicit_allow_and_no_pairs(oracle):
    rb = synth.random_tree(11, 2, seed=40)
    L = rb.n_links
    a = np.triu((np.random.default_rng(1).uniform(size=(L, L)) < 0.4).astype(np.uint8), 1)
    rb.allow = a + a.T
    _check_forward(oracle, rb, synth.states(rb, 200, seed=2), "allow_tree11")
    rb2 = synth.serial_chain(1, 3, seed=0)
    _check_forward(oracle, rb2, synth.states(rb2, 70, seed=2), "no_pairs_chain1")


def test_batch_zero_is_noop():
    wb = _wb()
    rb = synth.serial_chain(7, 5, seed=0)
    r = _dev_robot(rb)
    q = torch.empty((7, 0), device="cuda")
    pose, sph = wb.wb_fk(r, q)
    assert pose.shape == (8, 12, 0)
    wb.wb_self_collision(r, sph)


def _check_iteration(O, rb, st, label, w=None, torque_weight=1e-3, margin=0.01, sample=None):
    from paper_2603_05493_amd.iteration import PlainIteration
    r = _dev_robot(rb)
    wt = P.dev(w) if w is not None else None
    it = PlainIteration(r, st.B, w=wt, torque_weight=torque_weight, margin=margin, hinge_weight=1.0)
    q, qd, qdd = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
    it.run(q, qd, qdd, step=False)
    torch.cuda.synchronize()
    idx = np.arange(st.B) if sample is None else sample
    sub = lambda a: a[idx]
    ref = P.oracle_iteration(O, rb, sub(st.q), sub(st.qd), sub(st.qdd), None if w is None else sub(w),
                             torque_weight, margin, 1.0)
    pens = O.self_collision_pens(rb, ref["c"])
    g = lambda t: sub(P.host(t))
    cscale = P.cost_scale(ref, w, torque_weight, margin)
    e_cost = (np.abs(g(it.cost) - ref["cost"]) / cscale).max()
    am = sub(it.argmax.cpu().numpy())
    gq = P.check_grad_q(O, rb, sub(st.q), ref, g(it.g_q) + g(it.g_q_fk), am, margin, pens=pens)
    # the FK-through-hinge part on its own, against the same reference choice; for
    # joints above both spheres of the pair the exact value is 0 and FP32 leaves
    # rounding noise of order eps |c| |g|, so its scale is floored (fk_grad_floor)
    g_ref, _, _, _ = P.reference_gq(O, rb, sub(st.q), ref, g(it.g_q) + g(it.g_q_fk), am, margin, pens=pens)
    fk_ref = g_ref - ref["g_q_rnea"]
    e_fk_plain = P.normwise(g(it.g_q_fk), fk_ref, floor=1e-6)
    e_fk = P.normwise(g(it.g_q_fk), fk_ref, floor=P.fk_grad_floor(ref))
    floored = int(((e_fk_plain > P.TOL) & (e_fk <= P.TOL)).sum())
    e_gqd = P.normwise(g(it.g_qd), ref["g_qd"], floor=1e-6).max()
    e_gqdd = P.normwise(g(it.g_qdd), ref["g_qdd"], floor=1e-6).max()
    _log(label + " fwd+bwd", e_cost=e_cost, e_gq_fk=float(e_fk.max()), fk_floor_decided=floored, e_gqd=e_gqd,
         e_gqdd=e_gqdd, **gq)
    for e in (e_cost, float(e_fk.max()), e_gqd, e_gqdd):
        assert e < P.TOL
    ok = P.unambiguous(pens) & (np.abs(ref["max_pen"] + margin) >= P.DELTA)
    return it, ref, ok


def test_chain7_fwdbwd_weighted(oracle):
    rb = synth.serial_chain(7, 5, seed=0)
    st = synth.states(rb, 4096, seed=12)
    w = synth.weights((4096, 7), seed=13)
    _check_iteration(oracle, rb, st, "chain7_B4096", w=w)


def test_chain7_fwdbwd_against_fd_of_oracle(oracle):
    """GPU gradient of sum(w.tau) + hinge against central FD (h=1e-6) of the FP64 oracle."""
    rb = synth.serial_chain(7, 5, seed=0)
    st = synth.states(rb, 64, seed=14)
    w = synth.weights((64, 7), seed=15)
    it, ref, ok = _check_iteration(oracle, rb, st, "chain7_B64_fd", w=w)
    h = 1e-6

    def cost(q, qd, qdd):
        return P.oracle_iteration(oracle, rb, q, qd, qdd, w)["cost"]

    gq = P.host(it.g_q) + P.host(it.g_q_fk)
    for j in range(7):
        e = np.zeros_like(st.q)
        e[:, j] = h
        fd = (cost(st.q + e, st.qd, st.qdd) - cost(st.q - e, st.qd, st.qdd)) / (2 * h)
        sel = ok & (np.abs(fd) > 1e-3)
        assert np.all(np.abs(gq[sel, j] - fd[sel]) <= 1e-4 * np.maximum(np.abs(gq[sel]).max(1), 1e-3))


def test_humanoid_fwdbwd(oracle):
    rb = synth.humanoid48(seed=0)
    st = synth.states(rb, 2048, seed=16, q_range=1.5)
    _check_iteration(oracle, rb, st, "humanoid48_B2048")


@pytest.mark.parametrize("i", [0, 1, 2, 3])
def test_uneven_trees_fwdbwd(oracle, i):
    n, B = synth.UNEVEN_TREES[i]
    rb = synth.random_tree(n, 6, seed=i)
    st = synth.states(rb, B, seed=17 + i)
    _check_iteration(oracle, rb, st, f"tree{n}_B{B}")


def test_mimic_fwdbwd(oracle):
    rb = _mimic_robot()
    st = synth.states(rb, 700, seed=18)
    w = synth.weights((700, rb.n_dof), seed=19)
    _check_iteration(oracle, rb, st, "mimic_tree9", w=w)


def test_optimizer_size_sampled(oracle):
    """The full optimizer-shaped batch (48-DoF, 24576 states) in the launch
    configuration the benchmark times, checked on 768 sampled states."""
    rb = synth.humanoid48(seed=0)
    B = 24576
    st = synth.states(rb, B, seed=21, q_range=1.5)
    sample = np.sort(np.random.default_rng(0).choice(B, 768, replace=False))
    _check_iteration(oracle, rb, st, "humanoid48_B24576_sampled", sample=sample)


def test_fk_backward_dense_and_pose_grads(oracle):
    wb = _wb()
    rb = synth.random_tree(15, 4, seed=50, random_fixed_rotation=True)
    r = _dev_robot(rb)
    B = 777
    st = synth.states(rb, B, seed=51)
    rng = np.random.default_rng(52)
    gc = rng.normal(size=(B, rb.n_spheres, 3))
    gR = rng.normal(size=(B, rb.n_links, 3, 3))
    gp = rng.normal(size=(B, rb.n_links, 3))
    gpose = np.concatenate([gR.reshape(B, -1, 9), gp], 2)
    q = P.dev(st.q)
    pose, _ = wb.wb_fk(r, q)
    ref = oracle.fk_backward(rb, st.q, g_spheres=gc, g_R=gR, g_p=gp)
    for lp in (pose, None):   # cached transforms, then recomputed in the backward
        g = wb.wb_fk_backward(r, q, g_spheres=P.dev(gc), g_link_pose=P.dev(gpose), link_pose=lp)
        torch.cuda.synchronize()
        e = P.normwise(P.host(g), ref, floor=1e-6).max()
        _log("fk_backward_dense", recompute=lp is None, e=e)
        assert e < P.TOL


def test_autograd_wrappers_match_abi(oracle):
    wb = _wb()
    rb = synth.random_tree(12, 3, seed=60)
    r = _dev_robot(rb)
    B = 256
    st = synth.states(rb, B, seed=61)
    q = P.dev(st.q).requires_grad_(True)
    qd = P.dev(st.qd).requires_grad_(True)
    qdd = P.dev(st.qdd).requires_grad_(True)
    sph = wb.forward_kinematics(r, q)
    mp, am, nc = wb.self_collision(r, sph)
    tau = wb.inverse_dynamics(r, q, qd, qdd)
    w = P.dev(synth.weights((B, rb.n_dof), seed=62))
    loss = (w * tau).sum() + mp.sum()
    loss.backward()
    R, p, c = oracle.fk(rb, st.q)
    mpr, amr, _ = oracle.self_collision(rb, c)
    gc = oracle.self_collision_backward(rb, c, amr, mpr, 1e30, np.ones(B))
    g_rnea = oracle.rnea_vjp(rb, st.q, st.qd, st.qdd, synth.weights((B, rb.n_dof), seed=62))[0]
    # every state: the oracle's gradient for the pair the GPU chose where the maximum is tied
    info = P.check_grad_q(oracle, rb, st.q, dict(c=c, max_pen=mpr, argmax=amr, g_q_rnea=g_rnea),
                          P.host(q.grad), am.cpu().numpy(), margin=1e30)
    _log("autograd", **info)


def test_bitwise_deterministic():
    from paper_2603_05493_amd.iteration import PlainIteration
    rb = synth.humanoid48(seed=0)
    r = _dev_robot(rb)
    st = synth.states(rb, 3000, seed=70, q_range=1.5)
    outs = []
    for _ in range(2):
        it = PlainIteration(r, st.B)
        it.run(P.dev(st.q), P.dev(st.qd), P.dev(st.qdd), step=False)
        torch.cuda.synchronize()
        outs.append([t.clone() for t in (it.max_pen, it.argmax, it.n_coll, it.tau, it.g_q, it.g_q_fk,
                                         it.g_qd, it.g_qdd)])
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def _small_radius_humanoid():
    rb = synth.humanoid48(seed=4)
    rb.sphere_r = synth._f32(rb.sphere_r * 0.3)
    return rb


def test_forward_no_collision_regime(oracle):
    """Mostly negative maxima: the broad phase's threshold comes from the seed."""
    rb = _small_radius_humanoid()
    _check_forward(oracle, rb, synth.states(rb, 1500, seed=7, q_range=1.5), "humanoid_small_r")


def _tie_robot():
    """Root with three children; spheres at the child origins make the pairs
    (1,3) and (2,3) exact mirror images, so their penetrations tie in FP32."""
    L = 4
    z = np.zeros((L, 3))
    fp = np.array([[0, 0, 0], [0.125, 0, 0], [-0.125, 0, 0], [0, 0, 0.0625]])
    axis = np.tile([0.0, 0.0, 1.0], (L, 1))
    inertia = np.tile(np.eye(3) * 1e-3, (L, 1, 1))
    return synth._finish("tie", 0, [-1, 0, 0, 0], axis, np.tile(np.eye(3), (L, 1, 1)), fp,
                         np.ones(L), z, inertia, [1, 2, 3], np.zeros((3, 3)), np.full(3, 0.0875))


def test_exact_tie_takes_lowest_pair(oracle):
    wb = _wb()
    rb = _tie_robot()
    r = _dev_robot(rb)
    B = 130
    q = torch.zeros((3, B), device="cuda")
    pose, sph = wb.wb_fk(r, q)
    mp, am, nc = wb.wb_self_collision(r, sph)
    torch.cuda.synchronize()
    s, t = oracle.pairs(rb)
    pens = oracle.self_collision_pens(rb, np.zeros((1, 3, 3)) + P.host(sph)[:1])
    assert pens[0, 0] < pens[0, 1] == pens[0, 2]          # pairs (1,2), (1,3), (2,3)
    assert np.all(am.cpu().numpy() == 1) and np.all(nc.cpu().numpy() == 2)
