"""GPU checks of the launch-shape variants and the uneven multi-robot plan:
every shape agrees with the FP64 oracle; the persistent plan reproduces the
single-robot fused launch bit for bit with the same shapes; a plan captured
in a HIP graph replays identically."""
import numpy as np
import pytest
import torch

from paper_2603_05493_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu


def _robot(rb):
    from paper_2603_05493_amd import wb
    return wb.Robot(rb).to_device("cuda:0")


def _oracle_check(O, rb, st, out, label, margin=0.01, torque_weight=1e-3, fext=None):
    ref = P.oracle_iteration(O, rb, st.q, st.qd, st.qdd, None, torque_weight, margin, 1.0, fext=fext)
    if "g_fext" in out:
        g = np.transpose(out["g_fext"].cpu().numpy().astype(np.float64), (2, 0, 1))
        e = P.normwise(g, ref["g_fext"], floor=1e-6).max()
        print(label, f"e_gfext={e:.2e}", flush=True)
        assert e < P.TOL
    pens = O.self_collision_pens(rb, ref["c"])
    e_tau = P.normwise(P.host(out["tau"]), ref["tau"], floor=1e-3).max()
    gq = P.check_grad_q(O, rb, st.q, ref, P.host(out["g_q"]), out["argmax"].cpu().numpy(), margin, pens=pens)
    e_gqd = P.normwise(P.host(out["g_qd"]), ref["g_qd"], floor=1e-6).max()
    e_gqdd = P.normwise(P.host(out["g_qdd"]), ref["g_qdd"], floor=1e-6).max()
    e_cost = (np.abs(P.host(out["cost"]) - ref["cost"]) / P.cost_scale(ref, None, torque_weight, margin)).max()
    amb = P.unambiguous(pens)
    print(label, f"e_tau={e_tau:.2e} e_gqd={e_gqd:.2e} e_gqdd={e_gqdd:.2e} e_cost={e_cost:.2e}",
          " ".join(f"{k}={v}" for k, v in gq.items()), flush=True)
    for e in (e_tau, e_gqd, e_gqdd, e_cost):
        assert e < P.TOL
    np.testing.assert_array_equal(out["argmax"].cpu().numpy()[amb], ref["argmax"][amb])
    lo, hi = P.count_band(pens)
    nc = out["n_coll"].cpu().numpy()
    assert np.all((nc >= lo) & (nc <= hi))


@pytest.mark.parametrize("lanes,items", [(16, 4), (16, 16), (32, 8), (64, 16), (64, 1), (32, 64)])
def test_launch_shapes_small_tree(oracle, lanes, items):
    from paper_2603_05493_amd.iteration import FusedIteration
    rb = synth.random_tree(12, 6, seed=1)
    r = _robot(rb)
    r.set_tune(lanes, items)
    B = 777
    st = synth.states(rb, B, seed=5)
    it = FusedIteration(r, B)
    it.run(P.dev(st.q), P.dev(st.qd), P.dev(st.qdd), step=False)
    torch.cuda.synchronize()
    out = dict(tau=it.tau, g_q=it.g_q, g_qd=it.g_qd, g_qdd=it.g_qdd, cost=it.cost, argmax=it.argmax,
               n_coll=it.n_coll)
    _oracle_check(oracle, rb, st, out, f"tree12 G={lanes} c={items}")


def test_tune_validation():
    from paper_2603_05493_amd import _abi
    r = _robot(synth.random_tree(23, 2, seed=2))
    for bad in ((16, 8), (48, 8), (32, 0), (64, 5000)):
        with pytest.raises(_abi.WbError):
            r.set_tune(*bad)
    r.set_tune(32, 8, 12.5)
    assert r.get_tune() == {"lanes_per_state": 32, "states_per_item": 8, "ns_per_state": 12.5}


def _uneven():
    return [(synth.random_tree(n, 6, seed=i), b) for i, (n, b) in enumerate(synth.UNEVEN_TREES)]


def test_plan_uneven_trees_against_oracle(oracle):
    from paper_2603_05493_amd.iteration import PlanIteration
    jobs = _uneven()
    robots = [_robot(rb) for rb, _ in jobs]
    sts = [synth.states(rb, B, seed=80 + i) for i, (rb, B) in enumerate(jobs)]
    it = PlanIteration(robots, [B for _, B in jobs])
    it.run([(P.dev(s.q), P.dev(s.qd), P.dev(s.qdd)) for s in sts], step=False)
    torch.cuda.synchronize()
    assert it.plan.n_items >= 4
    for (rb, B), st, buf in zip(jobs, sts, it.bufs):
        _oracle_check(oracle, rb, st, buf, f"plan {rb.name} B={B}")


def test_plan_tune_shapes_against_oracle(oracle):
    """The plan shapes the benchmark uses (measured inside the plan when the
    tuned table has them, else the narrowest lanes with one round of the
    workgroup per work item) on the uneven trees, against the oracle."""
    from paper_2603_05493_amd import tune
    from paper_2603_05493_amd.iteration import PlanIteration
    jobs = _uneven()
    robots = [_robot(rb) for rb, _ in jobs]
    table = tune.load()
    tunes = tune.plan_shapes(robots, [B for _, B in jobs], table)
    for r, t in zip(robots, tunes):
        g = t["lanes_per_state"]
        assert g >= r.n_links and g in (16, 32, 64)
        assert t["states_per_item"] % (4 * (64 // g)) == 0
    sts = [synth.states(rb, B, seed=90 + i) for i, (rb, B) in enumerate(jobs)]
    it = PlanIteration(robots, [B for _, B in jobs], tunes=tunes)
    it.run([(P.dev(s.q), P.dev(s.qd), P.dev(s.qdd)) for s in sts], step=False)
    torch.cuda.synchronize()
    for (rb, B), st, buf in zip(jobs, sts, it.bufs):
        _oracle_check(oracle, rb, st, buf, f"plan (plan shapes) {rb.name} B={B}")


def test_plan_matches_single_robot_launch_bitwise():
    from paper_2603_05493_amd.iteration import FusedIteration, PlanIteration
    jobs = _uneven()
    robots = [_robot(rb) for rb, _ in jobs]
    tunes = [{"lanes_per_state": 16, "states_per_item": 8}, {"lanes_per_state": 16, "states_per_item": 16},
             {"lanes_per_state": 32, "states_per_item": 16}, {"lanes_per_state": 64, "states_per_item": 4}]
    sts = [synth.states(rb, B, seed=90 + i) for i, (rb, B) in enumerate(jobs)]
    lr = 1e-3
    pq = [(P.dev(s.q), P.dev(s.qd), P.dev(s.qdd)) for s in sts]
    it = PlanIteration(robots, [B for _, B in jobs], tunes=tunes, lr=lr)
    it.run(pq, step=True)
    for r, (rb, B), st, t, buf, (q, qd, qdd) in zip(robots, jobs, sts, tunes, it.bufs, pq):
        r.set_tune(t["lanes_per_state"], t["states_per_item"])
        fi = FusedIteration(r, B, lr=lr)
        q2, qd2, qdd2 = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
        fi.run(q2, qd2, qdd2, step=True)
        torch.cuda.synchronize()
        for k in ("tau", "g_q", "g_qd", "g_qdd", "cost", "max_pen", "argmax", "n_coll"):
            assert torch.equal(buf[k], getattr(fi, k)), (rb.name, k)
        assert torch.equal(q, q2) and torch.equal(qd, qd2) and torch.equal(qdd, qdd2)


def test_plan_graph_replays():
    from paper_2603_05493_amd.iteration import PlanIteration
    jobs = _uneven()
    robots = [_robot(rb) for rb, _ in jobs]
    sts = [synth.states(rb, B, seed=100 + i) for i, (rb, B) in enumerate(jobs)]
    pq = [(P.dev(s.q), P.dev(s.qd), P.dev(s.qdd)) for s in sts]
    it = PlanIteration(robots, [B for _, B in jobs], lr=0.0)
    it.run(pq, step=False)
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in b.items()} for b in it.bufs]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        it.run(pq, step=False)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        it.run(pq, step=False)
    for rep in range(3):
        for b in it.bufs:
            for v in b.values():
                v.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = torch.randn(1000, device="cuda").sum().item()   # unrelated eager work between replays
        for b, rb_ in zip(it.bufs, ref):
            for k in b:
                assert torch.equal(b[k], rb_[k]), (rep, k)


def test_autotuner_picks_a_valid_shape():
    from paper_2603_05493_amd import tune
    rb = synth.random_tree(7, 6, seed=0)
    r = _robot(rb)
    res = tune.tune_robot(r, rb, 2048, lanes=(16, 64), items=(8, 16), reps=2, rounds=2)
    assert res["lanes_per_state"] in (16, 64) and res["states_per_item"] in (8, 16)
    # (16 lanes, 8 states) is less than one round of the workgroup (16 states) and is not offered
    assert sorted((g, c) for g, c, _ in res["candidates"]) == [(16, 16), (64, 8), (64, 16)]
    assert res["ns_per_state"] > 0
    assert r.get_tune()["lanes_per_state"] == res["lanes_per_state"]
    assert tune.apply(r, {r.topology_key(): res})


def test_plan_mimic_tree_and_external_forces(oracle):
    """A plan holding a mimic robot, with external forces on two of its
    trees, runs the variant that carries both; every tree agrees with the
    oracle (torques, gradients and the gradient on the forces)."""
    from paper_2603_05493_amd import wb
    from tests.test_gpu_fused import _mimic_tree
    jobs = [(_mimic_tree(), 900), (synth.serial_chain(7, 5, seed=0), 1500), (synth.random_tree(12, 6, seed=1), 700)]
    robots = [_robot(rb) for rb, _ in jobs]
    plan = wb.Plan(robots, [B for _, B in jobs])
    rng = np.random.default_rng(90)
    ios, sts, fexts = [], [], []
    for i, (rb, B) in enumerate(jobs):
        st = synth.states(rb, B, seed=91 + i)
        n = rb.n_dof
        io = dict(q=P.dev(st.q), qd=P.dev(st.qd), qdd=P.dev(st.qdd))
        for key in ("tau", "g_q", "g_qd", "g_qdd"):
            io[key] = torch.empty((n, B), device="cuda")
        io["cost"] = torch.empty(B, device="cuda")
        io["argmax"] = torch.empty(B, dtype=torch.int32, device="cuda")
        io["n_coll"] = torch.empty(B, dtype=torch.int32, device="cuda")
        fe = None
        if i < 2:
            fe = synth._f32(rng.normal(scale=2.0, size=(B, rb.n_links, 6)))
            io["f_ext"] = torch.from_numpy(np.ascontiguousarray(np.transpose(fe, (1, 2, 0)), dtype=np.float32)).cuda()
            io["g_fext"] = torch.empty((rb.n_links, 6, B), device="cuda")
        ios.append(io)
        sts.append(st)
        fexts.append(fe)
    plan.run(ios, 1e-3, 0.01, 1.0, 0.0)
    torch.cuda.synchronize()
    for (rb, B), st, io, fe in zip(jobs, sts, ios, fexts):
        _oracle_check(oracle, rb, st, io, f"plan-ext {rb.name} B={B}", fext=fe)
