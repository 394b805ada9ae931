"""Host checks of the parity helpers the GPU tests rely on: the all-state
gradient check accepts the oracle's own results, accepts the alternative
subgradient at a tie or at the hinge kink, and rejects an argmax outside
the tie band or a gradient beyond the 1e-4 bound."""
import numpy as np
import pytest

from paper_2603_05493_amd import synth
from tests import parity as P


def _setup(O, B=300, seed=3):
    rb = synth.humanoid48(seed=0)
    st = synth.states(rb, B, seed=seed, q_range=1.5)
    ref = P.oracle_iteration(O, rb, st.q, st.qd, st.qdd, None, 1e-3, 0.01, 1.0)
    return rb, st, ref


def test_oracle_results_pass_with_no_allowance(oracle):
    rb, st, ref = _setup(oracle)
    info = P.check_grad_q(oracle, rb, st.q, ref, ref["g_q"], ref["argmax"], 0.01)
    assert info["e_gq_max"] < 1e-12 and info["checked"] == st.B


def test_alternative_subgradients_are_accepted(oracle):
    rb, st, ref = _setup(oracle)
    B = st.B
    pens = oracle.self_collision_pens(rb, ref["c"])
    # a state whose hinge is forced to the kink: the gradient without the hinge is valid there
    b = int(np.argmax(ref["max_pen"] > -0.01))
    ref_k = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in ref.items()}
    margin = float(-ref["max_pen"][b])          # max_pen + margin = 0 at state b
    got = ref["g_q"].copy()
    got[b] = ref["g_q_rnea"][b]
    g_ref, tied, kink, _ = P.reference_gq(oracle, rb, st.q, ref_k, got, ref["argmax"], margin, pens=pens)
    assert kink[b]
    np.testing.assert_allclose(g_ref[b], ref["g_q_rnea"][b])
    # a tie: declare the runner-up pair of a state tied by widening nothing but
    # the tie test's input -- a second pair given the maximum's penetration
    order = np.argsort(-pens, axis=1)
    b2 = 0
    p1, p2 = order[b2, 0], order[b2, 1]
    pens_t = pens.copy()
    pens_t[b2, p2] = pens_t[b2, p1]
    am = ref["argmax"].copy()
    am[b2] = p2
    g_ref2, tied2, _, alt = P.reference_gq(oracle, rb, st.q, ref, ref["g_q"], am, 0.01, pens=pens_t)
    assert tied2[b2] and alt[b2] == p2
    gc = oracle.self_collision_backward(rb, ref["c"][b2:b2 + 1], np.array([p2], np.int32),
                                        np.array([ref["max_pen"][b2]]), 0.01, np.ones(1))
    expect = ref["g_q_rnea"][b2] + oracle.fk_backward(rb, st.q[b2:b2 + 1], g_spheres=gc)[0]
    np.testing.assert_allclose(g_ref2[b2], expect, rtol=1e-12, atol=1e-12)


def test_wrong_argmax_and_large_errors_are_rejected(oracle):
    rb, st, ref = _setup(oracle)
    pens = oracle.self_collision_pens(rb, ref["c"])
    am = ref["argmax"].copy()
    gap = pens.max(1)[:, None] - pens
    b = int(np.argmax((gap > 1e-3).any(1)))
    am[b] = int(np.argmax(gap[b] > 1e-3))       # a pair far below the maximum
    with pytest.raises(AssertionError):
        P.check_grad_q(oracle, rb, st.q, ref, ref["g_q"], am, 0.01, pens=pens)
    got = ref["g_q"].copy()
    got[5] += P.TOL * 1.5 * np.abs(ref["g_q"][5]).max()
    with pytest.raises(AssertionError):
        P.check_grad_q(oracle, rb, st.q, ref, got, ref["argmax"], 0.01, pens=pens)
