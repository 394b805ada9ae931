"""GPU parity of the fused single-kernel iteration (wb_wholebody_step)
against the FP64 oracle, and against the plain per-operation launches."""
import numpy as np
import pytest
import torch

from paper_2603_05493_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu


def _robot(rb):
    from paper_2603_05493_amd import wb
    return wb.Robot(rb).to_device("cuda:0")


def _log(name, **kv):
    print(name, " ".join(f"{k}={v:.3g}" if isinstance(v, float) else f"{k}={v}" for k, v in kv.items()),
          flush=True)


def check_fused(O, rb, st, label, w=None, torque_weight=1e-3, margin=0.01, sample=None):
    from paper_2603_05493_amd.iteration import FusedIteration
    r = _robot(rb)
    it = FusedIteration(r, st.B, w=None if w is None else P.dev(w), torque_weight=torque_weight,
                        margin=margin, hinge_weight=1.0)
    q, qd, qdd = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
    it.run(q, qd, qdd, step=False)
    torch.cuda.synchronize()
    idx = np.arange(st.B) if sample is None else sample
    sub = lambda a: a[idx]
    g = lambda t: sub(P.host(t))
    ref = P.oracle_iteration(O, rb, sub(st.q), sub(st.qd), sub(st.qdd), None if w is None else sub(w),
                             torque_weight, margin, 1.0)
    pens = O.self_collision_pens(rb, ref["c"])
    ext = P.extent(ref["c"])
    e_tau = P.normwise(g(it.tau), ref["tau"], floor=1e-3).max()
    e_mp = P.scaled(g(it.max_pen)[:, None], ref["max_pen"][:, None], ext).max()
    e_cost = (np.abs(g(it.cost) - ref["cost"]) / P.cost_scale(ref, w, torque_weight, margin)).max()
    am = sub(it.argmax.cpu().numpy())
    nc = sub(it.n_coll.cpu().numpy())
    gq = P.check_grad_q(O, rb, sub(st.q), ref, g(it.g_q), am, margin, pens=pens)
    e_gqd = P.normwise(g(it.g_qd), ref["g_qd"], floor=1e-6).max()
    e_gqdd = P.normwise(g(it.g_qdd), ref["g_qdd"], floor=1e-6).max()
    lo, hi = P.count_band(pens)
    amb = P.unambiguous(pens)
    _log(label + " fused", e_tau=e_tau, e_mp=e_mp, e_cost=e_cost, e_gqd=e_gqd, e_gqdd=e_gqdd, **gq)
    for e in (e_tau, e_mp, e_cost, e_gqd, e_gqdd):
        assert e < P.TOL
    np.testing.assert_array_equal(am[amb], ref["argmax"][amb])
    assert np.all((nc >= lo) & (nc <= hi))
    return it, ref


@pytest.mark.parametrize("label,factory,B,qr,weighted", [
    ("chain7_B32", lambda: synth.serial_chain(7, 5, seed=0), 32, np.pi, True),
    ("chain7_B4096", lambda: synth.serial_chain(7, 5, seed=0), 4096, np.pi, True),
    ("humanoid48_B2048", lambda: synth.humanoid48(seed=0), 2048, 1.5, False),
    ("tree7_B8192", lambda: synth.random_tree(7, 6, seed=0), 8192, np.pi, False),
    ("tree12_B4096", lambda: synth.random_tree(12, 6, seed=1), 4096, np.pi, False),
    ("tree23_B2048", lambda: synth.random_tree(23, 6, seed=2), 2048, np.pi, False),
    ("tree48_B1024", lambda: synth.random_tree(48, 6, seed=3), 1024, np.pi, False),
    ("humanoid48_paper_scale_B1000", synth.humanoid48_paper_scale, 1000, 1.5, False),
    ("chain3_9spheres_B512", lambda: synth.serial_chain(3, 9, seed=4), 512, np.pi, True),
])
def test_fused_parity(oracle, label, factory, B, qr, weighted):
    rb = factory()
    st = synth.states(rb, B, seed=31, q_range=qr)
    w = synth.weights((B, rb.n_dof), seed=32) if weighted else None
    check_fused(oracle, rb, st, label, w=w)


def test_fused_breadth_first_numbering_and_fixed_rotations(oracle):
    """Links not in depth-first order exercise the lane permutation."""
    rb = synth.random_tree(20, 3, seed=33, random_fixed_rotation=True, dfs_order=False)
    assert any(rb.parent[k] != k - 1 for k in range(2, rb.n_links))
    check_fused(oracle, rb, synth.states(rb, 1500, seed=34), "bfs_tree20", w=synth.weights((1500, 20), seed=35))


def test_fused_fixed_links(oracle):
    rb = synth.with_fixed_links(synth.random_tree(16, 2, seed=36, random_fixed_rotation=True), [3, 7, 12])
    check_fused(oracle, rb, synth.states(rb, 700, seed=37), "fixed_links_tree16")


@pytest.mark.parametrize("B", [1, 17, 100, 1029])
def test_fused_ragged(oracle, B):
    rb = synth.humanoid48(seed=2)
    check_fused(oracle, rb, synth.states(rb, B, seed=B, q_range=1.5), f"humanoid_ragged_B{B}")


@pytest.mark.parametrize("k", [1, 3, 4, 6, 7, 8])
def test_fused_spheres_per_link(oracle, k):
    rb = synth.random_tree(10, k, seed=40 + k)
    check_fused(oracle, rb, synth.states(rb, 300, seed=k), f"tree10_k{k}")


def test_fused_optimizer_size_sampled(oracle):
    rb = synth.humanoid48(seed=0)
    B = 24576
    st = synth.states(rb, B, seed=21, q_range=1.5)
    sample = np.sort(np.random.default_rng(1).choice(B, 768, replace=False))
    check_fused(oracle, rb, st, "humanoid48_B24576_sampled", sample=sample)


def test_fused_matches_plain_and_steps():
    from paper_2603_05493_amd.iteration import FusedIteration, PlainIteration
    rb = synth.humanoid48(seed=0)
    r = _robot(rb)
    B = 3000
    st = synth.states(rb, B, seed=50, q_range=1.5)
    lr = 1e-3
    qa, qda, qdda = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
    qb, qdb, qddb = qa.clone(), qda.clone(), qdda.clone()
    pl = PlainIteration(r, B, lr=lr)
    fu = FusedIteration(r, B, lr=lr)
    pl.run(qa, qda, qdda, step=True)
    fu.run(qb, qdb, qddb, step=True)
    torch.cuda.synchronize()
    same = (pl.argmax == fu.argmax)
    assert same.float().mean() > 0.99
    g_pl = pl.g_q + pl.g_q_fk
    e = ((g_pl - fu.g_q).abs().amax(0) / g_pl.abs().amax(0).clamp_min(1e-6))[same]
    assert e.max().item() < 1e-4
    # the in-place step is x - lr * grad evaluated before the step
    x0 = P.dev(st.q)
    assert torch.allclose(qb, x0 - lr * fu.g_q, rtol=0, atol=1e-6)
    assert torch.allclose(qddb, P.dev(st.qdd) - lr * fu.g_qdd, rtol=0, atol=1e-6)
    assert ((qa - qb).abs().amax(0)[same] < 1e-6).all()


def _mimic_tree():
    rb = synth.random_tree(9, 3, seed=31, random_fixed_rotation=True)
    rb.joint_index = np.array([-1, 0, 1, 1, 2, 3, 4, 5, 5, 6], dtype=np.int32)
    rb.joint_mult = synth._f32([1.0, 1.0, 1.0, -0.5, 1.0, 2.0, 1.0, 1.0, 0.75, 1.0])
    rb.joint_offset = synth._f32([0.0, 0.0, 0.1, 0.25, 0.0, 0.0, -0.2, 0.0, 0.0, 0.0])
    return rb


def _humanoid_coupled_fingers():
    """The humanoid with each finger's distal joint following its proximal
    joint (ratio 0.8): 40 actuated joints drive 48 links."""
    rb = synth.humanoid48(seed=0)
    ji, jm = rb.joint_index.copy(), rb.joint_mult.copy()
    for wrist in (25, 40):
        for f in range(4):
            prox = wrist + 1 + 2 * f
            ji[prox + 1], jm[prox + 1] = ji[prox], 0.8
    used = sorted(set(int(j) for j in ji if j >= 0))
    remap = {j: i for i, j in enumerate(used)}
    rb.joint_index = np.array([remap[int(j)] if j >= 0 else -1 for j in ji], dtype=np.int32)
    rb.joint_mult = synth._f32(jm)
    return rb


@pytest.mark.parametrize("label,factory,B,qr,weighted", [
    ("mimic_tree9_B3000", _mimic_tree, 3000, np.pi, True),
    ("humanoid_coupled_fingers_B2048", _humanoid_coupled_fingers, 2048, 1.5, False),
])
def test_fused_mimic_joints(oracle, label, factory, B, qr, weighted):
    """Mimic joints (one actuator driving several links with a gain and an
    offset) in the fused iteration, against the oracle."""
    rb = factory()
    assert _robot(rb).fused_supported
    st = synth.states(rb, B, seed=17, q_range=qr)
    w = synth.weights((B, rb.n_dof), seed=18) if weighted else None
    check_fused(oracle, rb, st, label, w=w)


def test_fused_mimic_step_updates_each_joint_once():
    from paper_2603_05493_amd.iteration import FusedIteration
    rb = _humanoid_coupled_fingers()
    B = 1024
    st = synth.states(rb, B, seed=19, q_range=1.5)
    r = _robot(rb)
    fu = FusedIteration(r, B, torque_weight=1e-3, margin=0.01, hinge_weight=1.0)
    q, qd, qdd = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
    fu.run(q, qd, qdd, step=False)
    g_q, g_qd, g_qdd = fu.g_q.clone(), fu.g_qd.clone(), fu.g_qdd.clone()
    lr = 1e-3
    fu.lr = lr
    fu.run(q, qd, qdd, step=True)
    torch.cuda.synchronize()
    for x, x0, g in ((q, st.q, g_q), (qd, st.qd, g_qd), (qdd, st.qdd, g_qdd)):
        assert torch.allclose(x, P.dev(x0) - lr * g, rtol=0, atol=1e-6)


def test_fused_deterministic():
    from paper_2603_05493_amd.iteration import FusedIteration
    rb = synth.humanoid48(seed=0)
    r = _robot(rb)
    st = synth.states(rb, 2500, seed=60, q_range=1.5)
    outs = []
    for _ in range(2):
        it = FusedIteration(r, st.B)
        it.run(P.dev(st.q), P.dev(st.qd), P.dev(st.qdd), step=False)
        torch.cuda.synchronize()
        outs.append([t.clone() for t in (it.cost, it.max_pen, it.argmax, it.n_coll, it.tau, it.g_q)])
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_fused_no_collision_regime(oracle):
    rb = synth.humanoid48(seed=4)
    rb.sphere_r = synth._f32(rb.sphere_r * 0.3)
    check_fused(oracle, rb, synth.states(rb, 1500, seed=7, q_range=1.5), "humanoid_small_r")


def test_fused_exact_tie_takes_lowest_pair():
    from paper_2603_05493_amd.iteration import FusedIteration
    from tests.test_gpu_parity import _tie_robot
    rb = _tie_robot()
    r = _robot(rb)
    B = 70
    it = FusedIteration(r, B)
    z = torch.zeros((3, B), device="cuda")
    it.run(z, z.clone(), z.clone(), step=False)
    torch.cuda.synchronize()
    assert np.all(it.argmax.cpu().numpy() == 1) and np.all(it.n_coll.cpu().numpy() == 2)
