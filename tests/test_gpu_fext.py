"""GPU parity of external link forces (Alg. 4's f_ext, Alg. 5's gradient on
it) in the plain RNEA launches and the fused iteration, against the FP64
oracle.  Forces are in link coordinates, moment then force about the link
origin; device layout [L][6][B], oracle layout [B][L][6].

Tolerances are the parity module's: torques and gradients 1e-4 normwise per
state.  The gradient on f_ext comes from the torque cost alone (forces do
not move the collision spheres), so it is checked on every state."""
import numpy as np
import pytest
import torch

from paper_2603_05493_amd import synth
from tests import parity as P

pytestmark = pytest.mark.gpu


def _fext(rb, B, seed):
    """Forces of the order of the links' weights, moments of a lever arm's."""
    rng = np.random.default_rng(seed)
    f = np.empty((B, rb.n_links, 6))
    f[..., :3] = rng.normal(scale=0.5, size=(B, rb.n_links, 3))
    f[..., 3:] = rng.normal(scale=5.0, size=(B, rb.n_links, 3))
    return synth._f32(f)


def _dev_fext(f):               # [B, L, 6] -> [L][6][B]
    return torch.from_numpy(np.ascontiguousarray(np.transpose(f, (1, 2, 0)).astype(np.float32))).cuda()


def _host_fext(t):              # [L][6][B] -> [B, L, 6]
    return np.transpose(t.detach().cpu().numpy().astype(np.float64), (2, 0, 1))


CASES = [("chain7", lambda: synth.serial_chain(7, 5, seed=0), 3000, np.pi),
         ("tree23", lambda: synth.random_tree(23, 6, seed=2), 1024, np.pi),
         ("humanoid48", lambda: synth.humanoid48(seed=0), 777, 1.5)]


@pytest.mark.parametrize("label,factory,B,qr", CASES)
def test_plain_rnea_with_external_forces(oracle, label, factory, B, qr):
    from paper_2603_05493_amd import wb
    rb = factory()
    st = synth.states(rb, B, seed=31, q_range=qr)
    fe = _fext(rb, B, seed=32)
    r = wb.Robot(rb).to_device("cuda:0")
    q, qd, qdd = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
    tau, cache = wb.wb_rnea(r, q, qd, qdd, f_ext=_dev_fext(fe))
    rng = np.random.default_rng(33)
    g_tau = synth._f32(rng.normal(size=(B, rb.n_dof)))
    g_fext = torch.full((rb.n_links, 6, B), float("nan"), device="cuda")
    gq, gqd, gqdd = wb.wb_rnea_backward(r, q, qd, qdd, cache, P.dev(g_tau), g_fext=g_fext)
    torch.cuda.synchronize()
    ref = oracle.rnea(rb, st.q, st.qd, st.qdd, fe)
    ref0 = oracle.rnea(rb, st.q, st.qd, st.qdd)
    rq, rqd, rqdd, rfe = oracle.rnea_vjp(rb, st.q, st.qd, st.qdd, g_tau, fext=fe, want_fext=True)
    errs = dict(tau=P.normwise(P.host(tau), ref, floor=1e-3).max(),
                g_q=P.normwise(P.host(gq), rq, floor=1e-6).max(),
                g_qd=P.normwise(P.host(gqd), rqd, floor=1e-6).max(),
                g_qdd=P.normwise(P.host(gqdd), rqdd, floor=1e-6).max(),
                g_fext=P.normwise(_host_fext(g_fext), rfe, floor=1e-6).max())
    print(label, " ".join(f"{k}={v:.3g}" for k, v in errs.items()), flush=True)
    assert all(v < P.TOL for v in errs.values())
    assert P.normwise(ref, ref0, floor=1e-3).max() > 100 * P.TOL     # the forces really act
    # the base link carries no joint: its force never reaches a torque
    np.testing.assert_array_equal(_host_fext(g_fext)[:, 0], 0.0)


def _humanoid_coupled_fingers():
    from tests.test_gpu_fused import _humanoid_coupled_fingers as h
    return h()


@pytest.mark.parametrize("label,factory,B,qr,n_sample", [c + (None,) for c in CASES] + [
    # the EXT variant at the optimizer batch: mimic finger joints and forces
    # on every link, 512 sampled states against the oracle
    ("humanoid_coupled_fingers_B24576_sampled", _humanoid_coupled_fingers, 24576, 1.5, 512)])
def test_fused_iteration_with_external_forces(oracle, label, factory, B, qr, n_sample):
    from paper_2603_05493_amd import wb
    rb = factory()
    st = synth.states(rb, B, seed=41, q_range=qr)
    fe = _fext(rb, B, seed=42)
    sample = (np.sort(np.random.default_rng(43).choice(B, n_sample, replace=False)) if n_sample
              else np.arange(B))
    r = wb.Robot(rb).to_device("cuda:0")
    n, L = rb.n_dof, rb.n_links
    tw, margin, hw = 1e-3, 0.01, 1.0
    q, qd, qdd = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
    out = dict(tau=torch.empty((n, B), device="cuda"), cost=torch.empty(B, device="cuda"),
               max_pen=torch.empty(B, device="cuda"), argmax=torch.empty(B, dtype=torch.int32, device="cuda"),
               n_coll=torch.empty(B, dtype=torch.int32, device="cuda"),
               g_q=torch.empty((n, B), device="cuda"), g_qd=torch.empty((n, B), device="cuda"),
               g_qdd=torch.empty((n, B), device="cuda"))
    g_fext = torch.full((L, 6, B), float("nan"), device="cuda")
    wb.wb_wholebody_step(r, q, qd, qdd, torque_weight=tw, margin=margin, hinge_weight=hw,
                         f_ext=_dev_fext(fe), g_fext=g_fext, **out)
    torch.cuda.synchronize()
    ref = P.oracle_iteration(oracle, rb, st.q[sample], st.qd[sample], st.qdd[sample], None, tw, margin, hw,
                             fext=fe[sample])
    pens = oracle.self_collision_pens(rb, ref["c"])
    h = lambda x: P.host(x)[sample]
    gq = P.check_grad_q(oracle, rb, st.q[sample], ref, h(out["g_q"]), h(out["argmax"]), margin, hw, pens=pens)
    errs = dict(tau=P.normwise(h(out["tau"]), ref["tau"], floor=1e-3).max(),
                cost=(np.abs(h(out["cost"]) - ref["cost"]) / P.cost_scale(ref, None, tw, margin)).max(),
                g_qd=P.normwise(h(out["g_qd"]), ref["g_qd"], floor=1e-6).max(),
                g_qdd=P.normwise(h(out["g_qdd"]), ref["g_qdd"], floor=1e-6).max(),
                g_fext=P.normwise(_host_fext(g_fext)[sample], ref["g_fext"], floor=1e-6).max())
    print(label, "fused", " ".join(f"{k}={v:.3g}" for k, v in errs.items()),
          " ".join(f"{k}={v}" for k, v in gq.items()), flush=True)
    assert all(v < P.TOL for v in errs.values())


def test_fused_external_force_outputs_are_independent():
    """f_ext alone, g_fext alone and both give the same torques and gradients
    as the plain launches of the same definitions."""
    from paper_2603_05493_amd import wb
    rb = synth.random_tree(12, 6, seed=1)
    B = 2000
    st = synth.states(rb, B, seed=51, q_range=np.pi)
    fe = _dev_fext(_fext(rb, B, seed=52))
    r = wb.Robot(rb).to_device("cuda:0")
    n, L = rb.n_dof, rb.n_links
    q, qd, qdd = P.dev(st.q), P.dev(st.qd), P.dev(st.qdd)
    tw = 1e-3

    def fused(f_ext, want_g):
        tau = torch.empty((n, B), device="cuda")
        g_qdd = torch.empty((n, B), device="cuda")
        g = torch.empty((L, 6, B), device="cuda") if want_g else None
        wb.wb_wholebody_step(r, q, qd, qdd, torque_weight=tw, tau=tau, g_qdd=g_qdd, f_ext=f_ext, g_fext=g)
        return tau, g_qdd, g

    t_none, gqdd_none, _ = fused(None, False)
    t_g, gqdd_g, g_only = fused(None, True)
    t_f, gqdd_f, _ = fused(fe, False)
    t_fg, gqdd_fg, g_both = fused(fe, True)
    tau_p, cache = wb.wb_rnea(r, q, qd, qdd, f_ext=fe)
    gfe_p = torch.empty((L, 6, B), device="cuda")
    _, _, gqdd_p = wb.wb_rnea_backward(r, q, qd, qdd, cache, 2 * tw * tau_p, g_fext=gfe_p)
    torch.cuda.synchronize()
    close = lambda a, b, floor: P.normwise(P.host(a), P.host(b), floor=floor).max() < P.TOL
    assert close(t_g, t_none, 1e-3) and close(gqdd_g, gqdd_none, 1e-6)
    assert close(t_fg, t_f, 1e-3) and close(gqdd_fg, gqdd_f, 1e-6)
    assert close(t_fg, tau_p, 1e-3) and close(gqdd_fg, gqdd_p, 1e-6)
    assert P.normwise(P.host(g_both.reshape(L * 6, B)), P.host(gfe_p.reshape(L * 6, B)), floor=1e-6).max() < P.TOL
    assert not close(t_f, t_none, 1e-3)
    assert torch.isfinite(g_only).all()

