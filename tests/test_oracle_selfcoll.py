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


def test_hinge_backward_matches_fd(oracle):
    rb = synth.random_tree(12, 3, seed=6)
    st = synth.states(rb, 16, seed=7)
    _, _, c = oracle.fk(rb, st.q)
    margin = 0.01
    mp, am, _ = oracle.self_collision(rb, c)
    pens = oracle.self_collision_pens(rb, c)
    srt = np.sort(pens, 1)
    gap = srt[:, -1] - srt[:, -2]
    ok = (gap > 1e-4) & (np.abs(mp + margin) > 1e-4)   # away from the non-smooth points
    w = synth.weights(16, seed=8)
    g = oracle.self_collision_backward(rb, c, am, mp, margin, w)
    h = 1e-7
    for b in np.where(ok)[0][:6]:
        for s in range(0, rb.n_spheres, 5):
            for i in range(3):
                cp, cm = c[b:b + 1].copy(), c[b:b + 1].copy()
                cp[0, s, i] += h
                cm[0, s, i] -= h
                fd = w[b] * (oracle.hinge(oracle.self_collision(rb, cp)[0], margin) -
                             oracle.hinge(oracle.self_collision(rb, cm)[0], margin)) / (2 * h)
                assert abs(g[b, s, i] - fd[0]) < 1e-6
    assert ok.sum() >= 6
