"""Helpers shared by the GPU parity tests: layout conversion, the per-state
normwise error measure, the ambiguity band for integer decisions, and the
oracle's composition of the whole-body iteration (FK -> self-collision ->
hinge, RNEA -> torque cost, and their adjoints).

Tolerances (FP32 device arithmetic against the FP64 oracle):
  * every float output, per state: ||x - x_ref||_inf / max(||x_ref||_inf, floor)
    <= 1e-4 ("1e-4 relative", read normwise per output and state);
  * distances (sphere centres, link positions, max penetration) are scaled by
    the state's robot extent max_s |c_s| instead, since r_s + r_t - d
    cancels near contact;
  * argmax pair and collision counts are exact wherever the oracle's
    decision is farther than DELTA = 1e-5 m from a tie (about ten times the
    FP32 position error of an 18-deep chain); counts must lie in
    [#{pen > DELTA}, #{pen > -DELTA}];
  * the joint-position gradient is checked on every state at the same
    bound (check_grad_q): where the argmax pair is tied within DELTA, or the
    hinge sits within DELTA of its kink, the GPU's choice must be a valid
    one and its gradient is compared with the oracle's gradient for that
    same choice.
"""
from __future__ import annotations

import numpy as np
import torch

TOL = 1e-4
DELTA = 1e-5


def dev(a_Bk: np.ndarray) -> torch.Tensor:
    """State-major [B, ...] numpy -> device [..., B] float32 contiguous."""
    a = np.asarray(a_Bk, dtype=np.float32)
    return torch.from_numpy(np.ascontiguousarray(np.moveaxis(a, 0, -1))).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    """Device [..., B] -> state-major numpy float64 [B, ...]."""
    return np.moveaxis(t.detach().cpu().numpy().astype(np.float64), -1, 0)


def normwise(x: np.ndarray, ref: np.ndarray, floor: float = 1e-12) -> np.ndarray:
    B = x.shape[0]
    d = np.abs(x - ref).reshape(B, -1).max(1)
    s = np.maximum(np.abs(ref).reshape(B, -1).max(1), floor)
    return d / s


def scaled(x: np.ndarray, ref: np.ndarray, extent: np.ndarray) -> np.ndarray:
    B = x.shape[0]
    return np.abs(x - ref).reshape(B, -1).max(1) / np.maximum(extent, 1e-3)


def extent(c_ref: np.ndarray) -> np.ndarray:
    return np.linalg.norm(c_ref, axis=-1).max(-1)


def unambiguous(pens: np.ndarray, delta: float = DELTA) -> np.ndarray:
    """States whose maximum pair beats every other pair by at least delta."""
    if pens.shape[1] < 2:
        return np.ones(pens.shape[0], bool)
    part = -np.partition(-pens, 1, axis=1)[:, :2]
    return (part[:, 0] - part[:, 1]) >= delta


def count_band(pens: np.ndarray, delta: float = DELTA):
    return (pens > delta).sum(1), (pens > -delta).sum(1)


def cost_scale(ref, w, torque_weight, margin, floor=1e-3):
    """Magnitude the FP32 cost is accumulated from: sum |w tau| (or c tau^2) + hinge."""
    tau = ref["tau"]
    t = np.abs(w * tau).sum(1) if w is not None else torque_weight * (tau * tau).sum(1)
    return np.maximum(t + np.maximum(0.0, ref["max_pen"] + margin), floor)


def fk_grad_floor(ref, hinge_weight=1.0):
    """Floor for the hinge's FK gradient: 1 % of the magnitude of the terms it
    sums (extent x hinge weight).  For joints above both spheres of the pair
    the exact gradient is zero (the force is along the pair's centre line), so
    FP32 leaves rounding noise of order eps * |c| * |g| there."""
    return 1e-2 * float(np.median(extent(ref["c"]))) * hinge_weight


HINGE_D0 = 1e-2   # m: below this pair distance the hinge direction is ill-conditioned


def hinge_conditioning(ref, rb):
    """Amplification of centre errors into the hinge direction, HINGE_D0 / d at the argmax pair."""
    from oracle import oracle as O
    s, t = O.pairs(rb)
    am = ref["argmax"]
    c = ref["c"]
    cond = np.ones(len(am))
    for b in np.where(am >= 0)[0]:
        d = np.linalg.norm(c[b, s[am[b]]] - c[b, t[am[b]]])
        cond[b] = HINGE_D0 / max(d, 1e-9)
    return cond


def oracle_iteration(O, rb, q, qd, qdd, w=None, torque_weight=1e-3, margin=0.01, hinge_weight=1.0, fext=None):
    """FP64 reference of one iteration: costs and the gradient of
    sum_b cost_b with respect to q, qd, qdd (state-major arrays); with
    external link forces fext [B, L, 6] also the gradient on them."""
    R, p, c = O.fk(rb, q)
    mp, am, nc = O.self_collision(rb, c)
    tau = O.rnea(rb, q, qd, qdd, fext)
    g_tau = w if w is not None else 2.0 * torque_weight * tau
    tcost = np.sum(w * tau, 1) if w is not None else torque_weight * np.sum(tau * tau, 1)
    h = np.maximum(0.0, mp + margin)
    cost = tcost + hinge_weight * h
    g_c = O.self_collision_backward(rb, c, am, mp, margin, np.full(q.shape[0], hinge_weight))
    gq_fk = O.fk_backward(rb, q, g_spheres=g_c)
    gq, gqd, gqdd, gfe = O.rnea_vjp(rb, q, qd, qdd, g_tau, fext=fext, want_fext=True)
    return dict(R=R, p=p, c=c, max_pen=mp, argmax=am, n_coll=nc, tau=tau, cost=cost,
                g_q=gq + gq_fk, g_q_fk=gq_fk, g_q_rnea=gq, g_qd=gqd, g_qdd=gqdd, g_spheres=g_c, g_fext=gfe)



def reference_gq(O, rb, q, ref, got_gq, got_argmax, margin, hinge_weight=1.0, floor=1e-6, pens=None):
    """The oracle's joint-position gradient of the whole iteration (RNEA VJP
    plus FK through the hinge) for the choice the GPU made at each state:

      * unambiguous states: the oracle's own gradient;
      * argmax tied within DELTA: the GPU's pair must attain the maximum
        within DELTA, and the reference uses that pair (each tied pair gives
        a valid subgradient);
      * |max_pen + margin| < DELTA: the hinge may be on or off; the
        reference is whichever of the two the GPU's gradient is closer to.

    Returns (g_ref [B, n], tied mask, kink mask, the reference argmax)."""
    B = q.shape[0]
    if pens is None:
        pens = O.self_collision_pens(rb, ref["c"])
    mp = ref["max_pen"]
    tied = ~unambiguous(pens)
    kink = np.abs(mp + margin) < DELTA
    am = np.asarray(got_argmax, dtype=np.int64)
    if pens.shape[1] > 0:
        chosen = pens[np.arange(B), np.clip(am, 0, pens.shape[1] - 1)]
        valid = (am >= 0) & (chosen >= mp - DELTA)
        assert valid.all(), f"GPU argmax outside the tie band on {int((~valid).sum())} states"
    alt = np.where(tied, am, ref["argmax"]).astype(np.int32)
    hw = np.full(B, hinge_weight)
    on_mp = np.where(kink, np.abs(margin) + 1.0, mp)   # the hinge switched on at the kink
    g_on = ref["g_q_rnea"] + O.fk_backward(rb, q, g_spheres=O.self_collision_backward(rb, ref["c"], alt, on_mp,
                                                                                     margin, hw))
    if kink.any():
        e_on = normwise(got_gq, g_on, floor=floor)
        e_off = normwise(got_gq, ref["g_q_rnea"], floor=floor)
        g_on = np.where((kink & (e_off < e_on))[:, None], ref["g_q_rnea"], g_on)
    return g_on, tied, kink, alt


def check_grad_q(O, rb, q, ref, got_gq, got_argmax, margin, hinge_weight=1.0, floor=1e-6, pens=None):
    """Checks the GPU's joint-position gradient on every state against
    reference_gq at the plain bound: normwise error <= TOL per state, with
    no allowance for the hinge direction's conditioning.  Returns the counts
    the tests print: states checked, tied, at the kink, and close (argmax
    pair nearer than HINGE_D0, where an FP32 centre error e tilts the hinge
    direction by about e / d)."""
    g_ref, tied, kink, alt = reference_gq(O, rb, q, ref, got_gq, got_argmax, margin, hinge_weight, floor, pens)
    e = normwise(got_gq, g_ref, floor=floor)
    cond = hinge_conditioning(dict(argmax=alt, c=ref["c"]), rb)
    assert np.all(e <= TOL), f"g_q error {float(e.max()):.3g} on state {int(np.argmax(e))}"
    return dict(checked=int(q.shape[0]), tied=int(tied.sum()), kink=int(kink.sum()), close=int((cond > 1).sum()),
                e_gq_max=float(e.max()))
