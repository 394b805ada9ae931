"""GPU checks of the optional parts of the C-ABI boundary against the FP64
oracle: forward kinematics without a link-pose output (branch links
recompose their parent's pose from q), RNEA without a cache (one group of
lanes per state; the backward recomputes every forward quantity, external
forces and mimic joints included), and a persistent plan captured into a
HIP graph by the library itself (wb_plan_capture / wb_graph_launch)."""
import numpy as np
import pytest
import torch

from paper_2603_05493_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu


def _robot(rb):
    from paper_2603_05493_amd import wb
    return wb.Robot(rb).to_device("cuda:0")


def _mimic_robot():
    rb = synth.random_tree(9, 3, seed=31, random_fixed_rotation=True)
    rb.joint_index = np.array([-1, 0, 1, 1, 2, 3, 4, 5, 5, 6], dtype=np.int32)
    rb.joint_mult = synth._f32([1.0, 1.0, 1.0, -0.5, 1.0, 2.0, 1.0, 1.0, 0.75, 1.0])
    rb.joint_offset = synth._f32([0.0, 0.0, 0.1, 0.25, 0.0, 0.0, -0.2, 0.0, 0.0, 0.0])
    return rb


def _fext(rb, B, seed):
    rng = np.random.default_rng(seed)
    f = np.empty((B, rb.n_links, 6))
    f[..., :3] = rng.normal(scale=0.5, size=(B, rb.n_links, 3))
    f[..., 3:] = rng.normal(scale=5.0, size=(B, rb.n_links, 3))
    return synth._f32(f)


CASES = [("chain7", lambda: synth.serial_chain(7, 5, seed=0), 777, np.pi),
         ("tree23_bfs", lambda: synth.random_tree(23, 3, seed=33, random_fixed_rotation=True, dfs_order=False),
          500, np.pi),
         ("humanoid48", lambda: synth.humanoid48(seed=0), 1500, 1.5),
         ("tree48", lambda: synth.random_tree(48, 6, seed=3), 333, np.pi),
         ("mimic_tree9", _mimic_robot, 640, np.pi)]


@pytest.mark.parametrize("label,factory,B,qr", CASES)
def test_fk_without_link_poses(oracle, label, factory, B, qr):
    from paper_2603_05493_amd import wb
    rb = factory()
    r = _robot(rb)
    st = synth.states(rb, B, seed=5, q_range=qr)
    q = P.dev(st.q)
    pose, sph_ref = wb.wb_fk(r, q)
    none, sph = wb.wb_fk(r, q, want_pose=False)
    torch.cuda.synchronize()
    assert none is None
    _, _, c = oracle.fk(rb, st.q)
    ext = P.extent(c)
    e = P.scaled(P.host(sph), c, ext).max()
    print(label, f"spheres without poses: e={e:.3g}", flush=True)
    assert e < P.TOL


@pytest.mark.parametrize("label,factory,B,qr", CASES)
@pytest.mark.parametrize("forces", [False, True])
def test_rnea_without_cache(oracle, label, factory, B, qr, forces):
    from paper_2603_05493_amd import wb
    rb = factory()
    r = _robot(rb)
    st = synth.states(rb, B, seed=6, q_range=qr)
    n, L = rb.n_dof, rb.n_links
    fe = _fext(rb, B, seed=7) if forces else None
    fe_d = None if fe is None else torch.from_numpy(np.ascontiguousarray(np.transpose(fe, (1, 2, 0))).astype(np.float32)).cuda()
    q, qd, qdd = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
    tau, cache = wb.wb_rnea(r, q, qd, qdd, f_ext=fe_d, want_cache=False)
    assert cache is None
    w = synth.weights((B, n), seed=8)
    g_fext = torch.full((L, 6, B), float("nan"), device="cuda") if forces else None
    gq, gqd, gqdd = wb.wb_rnea_backward(r, q, qd, qdd, None, P.dev(w), f_ext=fe_d, g_fext=g_fext)
    torch.cuda.synchronize()
    tau_ref = oracle.rnea(rb, st.q, st.qd, st.qdd, fe)
    rq, rqd, rqdd, rfe = oracle.rnea_vjp(rb, st.q, st.qd, st.qdd, w, fext=fe, want_fext=True)
    errs = dict(tau=P.normwise(P.host(tau), tau_ref, floor=1e-3).max(),
                g_q=P.normwise(P.host(gq), rq, floor=1e-6).max(),
                g_qd=P.normwise(P.host(gqd), rqd, floor=1e-6).max(),
                g_qdd=P.normwise(P.host(gqdd), rqdd, floor=1e-6).max())
    if forces:
        got = np.transpose(g_fext.cpu().numpy().astype(np.float64), (2, 0, 1))
        errs["g_fext"] = P.normwise(got, rfe, floor=1e-6).max()
    print(label, "forces" if forces else "", " ".join(f"{k}={v:.3g}" for k, v in errs.items()), flush=True)
    assert all(v < P.TOL for v in errs.values()), errs


def test_rnea_without_cache_agrees_with_cached_path(oracle):
    """Both forms of the same definition on one batch (floating-point sums
    are ordered differently, so to the parity tolerance, not bit for bit)."""
    from paper_2603_05493_amd import wb
    rb = synth.humanoid48(seed=0)
    r = _robot(rb)
    B = 2048
    st = synth.states(rb, B, seed=9, q_range=1.5)
    q, qd, qdd = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
    t0, cache = wb.wb_rnea(r, q, qd, qdd)
    t1, _ = wb.wb_rnea(r, q, qd, qdd, want_cache=False)
    g = P.dev(synth.weights((B, rb.n_dof), seed=10))
    a = wb.wb_rnea_backward(r, q, qd, qdd, cache, g)
    b = wb.wb_rnea_backward(r, q, qd, qdd, None, g)
    torch.cuda.synchronize()
    assert P.normwise(P.host(t1), P.host(t0), floor=1e-3).max() < P.TOL
    for x, y in zip(a, b):
        assert P.normwise(P.host(y), P.host(x), floor=1e-6).max() < P.TOL


def test_rnea_without_cache_rejects_large_robots():
    from paper_2603_05493_amd import _abi, wb
    rb = synth.serial_chain(70, 1, seed=2)
    r = _robot(rb)
    q = torch.zeros((70, 4), device="cuda")
    with pytest.raises(_abi.WbError) as e:
        wb.wb_rnea(r, q, q, q, want_cache=False)
    assert e.value.code == _abi.WB_ERR_UNSUPPORTED


def _plan_setup(seed0):
    jobs = [(synth.random_tree(n, 6, seed=i), b) for i, (n, b) in
            enumerate([(7, 1500), (12, 900), (23, 700), (48, 300)])]
    robots = [_robot(rb) for rb, _ in jobs]
    sts = [synth.states(rb, B, seed=seed0 + i) for i, (rb, B) in enumerate(jobs)]
    return jobs, robots, sts


def _io(rb, st, outputs=True):
    B, n = st.B, rb.n_dof
    e = lambda *shape, dt=torch.float32: torch.empty(shape, dtype=dt, device="cuda")
    io = dict(q=P.dev(st.q), qd=P.dev(st.qd), qdd=P.dev(st.qdd), cost=e(B), max_pen=e(B),
              argmax=e(B, dt=torch.int32), n_coll=e(B, dt=torch.int32))
    if outputs:
        io.update(tau=e(n, B), g_q=e(n, B), g_qd=e(n, B), g_qdd=e(n, B))
    return io


def test_plan_captured_by_the_library_matches_oracle(oracle):
    from paper_2603_05493_amd import wb
    jobs, robots, sts = _plan_setup(110)
    plan = wb.Plan(robots, [B for _, B in jobs])
    ios = [_io(rb, st) for (rb, _), st in zip(jobs, sts)]
    graph = plan.capture(ios, 1e-3, 0.01, 1.0, 0.0, iters=1)
    for i in ios:                       # poison the outputs: the launch must write them
        for k in ("tau", "g_q", "cost"):
            i[k].fill_(float("nan"))
    graph.launch()
    torch.cuda.synchronize()
    for (rb, B), st, io in zip(jobs, sts, ios):
        ref = P.oracle_iteration(oracle, rb, st.q, st.qd, st.qdd, None, 1e-3, 0.01, 1.0)
        pens = oracle.self_collision_pens(rb, ref["c"])
        gq = P.check_grad_q(oracle, rb, st.q, ref, P.host(io["g_q"]), io["argmax"].cpu().numpy(), 0.01, pens=pens)
        e_tau = P.normwise(P.host(io["tau"]), ref["tau"], floor=1e-3).max()
        e_cost = (np.abs(P.host(io["cost"]) - ref["cost"]) / P.cost_scale(ref, None, 1e-3, 0.01)).max()
        e_gqd = P.normwise(P.host(io["g_qd"]), ref["g_qd"], floor=1e-6).max()
        e_gqdd = P.normwise(P.host(io["g_qdd"]), ref["g_qdd"], floor=1e-6).max()
        print("captured plan", rb.name, B, f"e_tau={e_tau:.3g} e_cost={e_cost:.3g} e_gqd={e_gqd:.3g} "
              f"e_gqdd={e_gqdd:.3g}", " ".join(f"{k}={v}" for k, v in gq.items()), flush=True)
        assert e_tau < P.TOL and e_cost < P.TOL and e_gqd < P.TOL and e_gqdd < P.TOL
    graph.close()


def test_plan_capture_of_several_iterations_equals_eager_runs():
    """A graph of 3 stepping iterations, launched twice, leaves the states
    exactly where 6 eager wb_plan_run calls do."""
    from paper_2603_05493_amd import wb
    jobs, robots, sts = _plan_setup(120)
    plan = wb.Plan(robots, [B for _, B in jobs])
    ios_g = [_io(rb, st, outputs=False) for (rb, _), st in zip(jobs, sts)]
    ios_e = [_io(rb, st, outputs=False) for (rb, _), st in zip(jobs, sts)]
    graph = plan.capture(ios_g, 1e-3, 0.01, 1.0, 1e-3, iters=3)
    graph.launch()
    graph.launch()
    for _ in range(6):
        plan.run(ios_e, 1e-3, 0.01, 1.0, 1e-3)
    torch.cuda.synchronize()
    for a, b in zip(ios_g, ios_e):
        for k in ("q", "qd", "qdd", "cost", "max_pen", "argmax"):
            assert torch.equal(a[k], b[k]), k
    moved = [not torch.equal(a["q"], P.dev(st.q)) for a, st in zip(ios_g, sts)]
    assert all(moved)
    graph.close()


def test_plan_capture_rejects_bad_arguments():
    import ctypes as C
    from paper_2603_05493_amd import _abi, wb
    jobs, robots, sts = _plan_setup(130)
    plan = wb.Plan(robots, [B for _, B in jobs])
    ios = [_io(rb, st) for (rb, _), st in zip(jobs, sts)]
    with pytest.raises(_abi.WbError) as e:
        plan.capture(ios, iters=0)
    assert e.value.code == _abi.WB_ERR_INVALID_ARG
    ios[1]["q"] = None                  # a missing state array: refused before anything is recorded
    with pytest.raises((_abi.WbError, AttributeError, TypeError, ValueError)):
        plan.capture(ios, iters=2)
    assert _abi.lib().wb_graph_destroy(None) == _abi.WB_OK
    assert _abi.lib().wb_graph_launch(None, None) == _abi.WB_ERR_INVALID_ARG


def _pad(x: torch.Tensor, extra: int, fill=float("nan")) -> torch.Tensor:
    """x [..., B] -> a [..., B + extra] tensor holding x in its first B columns and `fill` after."""
    out = torch.full((*x.shape[:-1], x.shape[-1] + extra), fill, dtype=x.dtype, device=x.device)
    out[..., : x.shape[-1]] = x
    return out


def _same_and_untouched(padded, dense, extra, label):
    B = dense.shape[-1]
    assert torch.equal(padded[..., :B], dense), label
    tail = padded[..., B:]
    assert torch.isnan(tail).all() if tail.is_floating_point() else True, f"{label}: padding written"


@pytest.mark.parametrize("label,factory,B", [("humanoid48", lambda: synth.humanoid48(seed=0), 1000),
                                             ("tree12", lambda: synth.random_tree(12, 6, seed=1), 777)])
def test_padded_rows_give_the_dense_results(label, factory, B):
    """Every call that takes a leading dimension, run on arrays whose rows
    are padded by 37 columns of NaN: the first B columns equal the dense
    call's bit for bit and the padding is never written (or read: NaN
    there would spread)."""
    from paper_2603_05493_amd import wb
    rb = factory()
    r = _robot(rb)
    st = synth.states(rb, B, seed=140, q_range=1.5)
    X = 37
    n = rb.n_dof
    q, qd, qdd = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
    qp, qdp, qddp = _pad(q, X), _pad(qd, X), _pad(qdd, X)
    # forward kinematics, self-collision and its adjoint
    L, S = rb.n_links, rb.n_spheres
    nanpad = lambda *shape: _pad(torch.zeros((*shape, B), device="cuda"), X)
    pose, sph = wb.wb_fk(r, q)
    pose_p, sph_p = wb.wb_fk(r, qp, link_pose=nanpad(L, 12), spheres=nanpad(S, 3), nb=B)
    mp, am, nc = wb.wb_self_collision(r, sph)
    mp_p, am_p, nc_p = wb.wb_self_collision(r, sph_p, nb=B)
    gcost = torch.ones(B, device="cuda")
    gs = wb.wb_self_collision_backward(r, sph, am, mp, 0.01, gcost)
    gs_p = wb.wb_self_collision_backward(r, sph_p, am_p, mp_p, 0.01, gcost, g_spheres=_pad(torch.zeros_like(gs), X),
                                         nb=B)
    gfk = wb.wb_fk_backward(r, q, g_spheres=gs, link_pose=pose)
    gfk_p = wb.wb_fk_backward(r, qp, g_spheres=gs_p, link_pose=pose_p, g_q=_pad(torch.zeros_like(gfk), X), nb=B)
    # RNEA with and without its cache, the cost head and the step
    tau, cache = wb.wb_rnea(r, q, qd, qdd)
    tau_p, cache_p = wb.wb_rnea(r, qp, qdp, qddp, tau=_pad(torch.zeros_like(tau), X), cache=nanpad(L, 18), nb=B)
    tau2_p, _ = wb.wb_rnea(r, qp, qdp, qddp, tau=_pad(torch.zeros_like(tau), X), want_cache=False, nb=B)
    tau2, _ = wb.wb_rnea(r, q, qd, qdd, want_cache=False)
    cost, gtau, gmp = wb.wb_cost_head(tau, None, 1e-3, mp, 0.01, 1.0)
    cost_p, gtau_p, gmp_p = wb.wb_cost_head(tau_p, None, 1e-3, mp_p, 0.01, 1.0, g_tau=_pad(torch.zeros_like(tau), X),
                                            nb=B)
    z = lambda: _pad(torch.zeros((n, B), device="cuda"), X)
    g = wb.wb_rnea_backward(r, q, qd, qdd, cache, gtau)
    g_p = wb.wb_rnea_backward(r, qp, qdp, qddp, cache_p, gtau_p, z(), z(), z(), nb=B)
    g2 = wb.wb_rnea_backward(r, q, qd, qdd, None, gtau)
    g2_p = wb.wb_rnea_backward(r, qp, qdp, qddp, None, gtau_p, z(), z(), z(), nb=B)
    # the fused iteration with its step
    outs = lambda ld: dict(tau=torch.zeros((n, ld), device="cuda"), g_q=torch.zeros((n, ld), device="cuda"),
                           cost=torch.empty(B, device="cuda"), argmax=torch.empty(B, dtype=torch.int32, device="cuda"))
    fd, fp = outs(B), {k: (_pad(v, X) if v.dim() == 2 else v) for k, v in outs(B).items()}
    qf, qdf, qddf = q.clone(), qd.clone(), qdd.clone()
    qfp, qdfp, qddfp = qp.clone(), qdp.clone(), qddp.clone()
    wb.wb_wholebody_step(r, qf, qdf, qddf, torque_weight=1e-3, margin=0.01, hinge_weight=1.0, lr=1e-3, **fd)
    wb.wb_wholebody_step(r, qfp, qdfp, qddfp, torque_weight=1e-3, margin=0.01, hinge_weight=1.0, lr=1e-3, nb=B,
                         **fp)
    # the plain step
    qs, qs_p = q.clone(), qp.clone()
    wb.wb_sgd_step(1e-3, qs, qd.clone(), qdd.clone(), g[0], g[1], g[2], g_q2=gfk)
    wb.wb_sgd_step(1e-3, qs_p, qdp.clone(), qddp.clone(), g_p[0], g_p[1], g_p[2], g_q2=gfk_p, nb=B)
    torch.cuda.synchronize()
    for a, b, nm in ((pose_p, pose, "pose"), (sph_p, sph, "spheres"), (gs_p, gs, "g_spheres"), (gfk_p, gfk, "g_q_fk"),
                     (tau_p, tau, "tau"), (cache_p, cache, "cache"), (tau2_p, tau2, "tau (no cache)"),
                     (gtau_p, gtau, "g_tau"), (qs_p, qs, "sgd q"), (qfp, qf, "fused q"), (qdfp, qdf, "fused qd"),
                     (fp["tau"], fd["tau"], "fused tau"), (fp["g_q"], fd["g_q"], "fused g_q")):
        _same_and_untouched(a, b, X, f"{label} {nm}")
    for a, b in zip(g_p, g):
        _same_and_untouched(a, b, X, f"{label} rnea backward")
    for a, b in zip(g2_p, g2):
        _same_and_untouched(a, b, X, f"{label} rnea backward (no cache)")
    for a, b in ((mp_p, mp), (am_p, am), (nc_p, nc), (cost_p, cost), (gmp_p, gmp), (fp["cost"], fd["cost"]),
                 (fp["argmax"], fd["argmax"])):
        assert torch.equal(a, b), label


def test_padded_plan_rows():
    """A plan run on padded rows equals the run on dense rows, and the padding is left alone."""
    from paper_2603_05493_amd import wb
    jobs, robots, sts = _plan_setup(150)
    plan = wb.Plan(robots, [B for _, B in jobs])
    dense = [_io(rb, st) for (rb, _), st in zip(jobs, sts)]
    padded = [{k: (_pad(v, 13) if v.dim() == 2 else v.clone()) for k, v in d.items()} for d in dense]
    plan.run(dense, 1e-3, 0.01, 1.0, 1e-3)
    plan.run(padded, 1e-3, 0.01, 1.0, 1e-3)
    torch.cuda.synchronize()
    for d, p in zip(dense, padded):
        for k, v in d.items():
            if v.dim() == 2:
                _same_and_untouched(p[k], v, 13, f"plan {k}")
            else:
                assert torch.equal(p[k], v), k
