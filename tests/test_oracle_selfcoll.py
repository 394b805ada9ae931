"""Pins for the oracle's self-collision (Sec. 6.2) and its backward.

The oracle is brute-force enumeration, i.e. the definition.  It is pinned to
an independently written vectorised computation on scipy's ``pdist``, to the
closed-form pair count of a chain with k spheres per link, and (for the
hinge backward) to central finite differences of the hinge cost.
"""
import numpy as np
import pytest
from scipy.spatial.distance import pdist

from paper_2603_05493_amd import synth


def _pdist_reference(rb, c):
    S = rb.n_spheres
    iu, ju = np.triu_indices(S, k=1)   # lexicographic (s, t), s < t
    la, lb = rb.sphere_link[iu], rb.sphere_link[ju]
    keep = (la != lb) & (rb.parent[lb] != la) & (rb.parent[la] != lb)
    rsum = (rb.sphere_r[:, None] + rb.sphere_r[None, :])[iu, ju]
    out = []
    for b in range(c.shape[0]):
        pen = (rsum - pdist(c[b]))[keep]
        out.append(pen)
    return np.stack(out), iu[keep], ju[keep]


@pytest.mark.parametrize("factory", [lambda: synth.serial_chain(7, 5, seed=0),
                                     lambda: synth.random_tree(23, 6, seed=2),
                                     lambda: synth.humanoid48(seed=0)])
def test_matches_pdist(oracle, factory):
    rb = factory()
    st = synth.states(rb, 6, seed=3, q_range=1.5)
    _, _, c = oracle.fk(rb, st.q)
    pen_ref, s_ref, t_ref = _pdist_reference(rb, c)
    s, t = oracle.pairs(rb)
    np.testing.assert_array_equal(s, s_ref)
    np.testing.assert_array_equal(t, t_ref)
    np.testing.assert_allclose(oracle.self_collision_pens(rb, c), pen_ref, atol=1e-12)
    mp, am, nc = oracle.self_collision(rb, c)
    np.testing.assert_allclose(mp, pen_ref.max(1), atol=1e-12)
    np.testing.assert_array_equal(am, pen_ref.argmax(1))   # argmax returns the first (lowest) index
    np.testing.assert_array_equal(nc, (pen_ref > 0).sum(1))


@pytest.mark.parametrize("n,k", [(7, 5), (3, 2), (12, 1)])
def test_chain_pair_count_closed_form(oracle, n, k):
    rb = synth.serial_chain(n, k, seed=1)
    S, L = rb.n_spheres, rb.n_links
    expected = S * (S - 1) // 2 - L * (k * (k - 1) // 2) - (L - 1) * k * k
    assert len(oracle.pairs(rb)[0]) == expected


def test_explicit_allow_matrix(oracle):
    rb = synth.random_tree(7, 2, seed=4)
    L = rb.n_links
    rng = np.random.default_rng(5)
    allow = (rng.uniform(size=(L, L)) < 0.5).astype(np.uint8)
    allow = np.triu(allow, 1)
    allow = allow + allow.T
    rb.allow = allow
    s, t = oracle.pairs(rb)
    ref = [(i, j) for i in range(rb.n_spheres) for j in range(i + 1, rb.n_spheres)
           if rb.sphere_link[i] != rb.sphere_link[j] and allow[rb.sphere_link[i], rb.sphere_link[j]]]
    assert list(zip(s.tolist(), t.tolist())) == ref


def test_degenerate_no_pairs(oracle):
    rb = synth.serial_chain(1, 3, seed=0)   # two links, parent and child: no pair allowed
    st = synth.states(rb, 3)
    _, _, c = oracle.fk(rb, st.q)
    mp, am, nc = oracle.self_collision(rb, c)
    assert np.all(np.isneginf(mp)) and np.all(am == -1) and np.all(nc == 0)


@pytest.mark.parametrize("r_scale,margin", [(1.0, 0.01), (0.5, 0.03)])
def test_hinge_backward_matches_fd(oracle, r_scale, margin):
    """The hinge gradient against central differences of the hinge cost: all
    three coordinates of both spheres of the most penetrating pair in every
    state away from the non-smooth points, and every other sphere (which
    must get exactly zero) in a few of them.  With smaller spheres and a
    wider margin, some states sit inside the margin without touching (the
    hinge is on) and some beyond it (the gradient is zero)."""
    rb = synth.random_tree(12, 3, seed=6)
    rb.sphere_r = synth._f32(rb.sphere_r * r_scale)
    B = 16
    st = synth.states(rb, B, seed=7)
    _, _, c = oracle.fk(rb, st.q)
    mp, am, _ = oracle.self_collision(rb, c)
    if r_scale < 1.0:
        assert ((mp < 0) & (mp + margin > 1e-4)).sum() >= 3 and (mp + margin < -1e-4).sum() >= 3
    pens = oracle.self_collision_pens(rb, c)
    srt = np.sort(pens, 1)
    gap = srt[:, -1] - srt[:, -2]
    ok = (gap > 1e-4) & (np.abs(mp + margin) > 1e-4)   # away from the non-smooth points
    assert ok.sum() >= 12
    w = synth.weights(B, seed=8)
    g = oracle.self_collision_backward(rb, c, am, mp, margin, w)
    ps, pt = oracle.pairs(rb)
    h = 1e-7

    def fd(b, s, i):
        cp, cm = c[b:b + 1].copy(), c[b:b + 1].copy()
        cp[0, s, i] += h
        cm[0, s, i] -= h
        return w[b] * (oracle.hinge(oracle.self_collision(rb, cp)[0], margin) -
                       oracle.hinge(oracle.self_collision(rb, cm)[0], margin))[0] / (2 * h)

    n_nonzero = 0
    for k, b in enumerate(np.where(ok)[0]):
        spheres = [ps[am[b]], pt[am[b]]]
        if k < 3:
            spheres = range(rb.n_spheres)
        for s in spheres:
            for i in range(3):
                ref = fd(b, s, i)
                assert abs(g[b, s, i] - ref) < 1e-6 * max(1.0, abs(w[b]))
                n_nonzero += abs(ref) > 1e-3
        others = np.setdiff1d(np.arange(rb.n_spheres), [ps[am[b]], pt[am[b]]])
        assert np.all(g[b, others] == 0.0)
    # both spheres of each colliding pair carry a gradient
    assert n_nonzero >= 2 * int((ok & (mp + margin > 0)).sum())
