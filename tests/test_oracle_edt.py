"""Pins of the distance-transform oracle against what the mathematics and an
independent implementation fix: SciPy's exact Euclidean distance transform,
closed forms (one site, a plane of sites, two sites), empty and full grids,
and symmetry under axis permutation."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import edt
from paper_2603_05493_amd import sitegrid


@pytest.mark.parametrize("shape,p,seed", [((7, 9, 11), 0.05, 0), ((16, 5, 23), 0.01, 1), ((12, 12, 12), 0.3, 2),
                                          ((1, 1, 40), 0.1, 3), ((3, 30, 1), 0.1, 4)])
def test_matches_scipy_exact_edt(shape, p, seed):
    m = sitegrid.random_sites(*shape, p=p, seed=seed)
    if not m.any():
        m[0, 0, 0] = 1
    d2 = edt.d2_grid(m)
    ref = ndimage.distance_transform_edt(m == 0)            # distance of every voxel to the nearest site
    np.testing.assert_array_equal(d2, np.rint(ref ** 2).astype(np.int64))
    np.testing.assert_allclose(edt.dist(d2, 0.02), 0.02 * ref, rtol=1e-15)


def test_single_site_is_the_euclidean_norm():
    m = np.zeros((9, 10, 11), np.uint8)
    m[4, 2, 7] = 1
    z, y, x = np.meshgrid(np.arange(9), np.arange(10), np.arange(11), indexing="ij")
    np.testing.assert_array_equal(edt.d2_grid(m), (z - 4) ** 2 + (y - 2) ** 2 + (x - 7) ** 2)


def test_plane_of_sites_gives_the_distance_to_the_plane():
    m = np.zeros((13, 6, 7), np.uint8)
    m[5] = 1
    z = np.arange(13)[:, None, None]
    np.testing.assert_array_equal(edt.d2_grid(m), np.broadcast_to((z - 5) ** 2, m.shape))


def test_two_sites_split_space_at_the_bisector():
    m = np.zeros((5, 5, 20), np.uint8)
    m[2, 2, 3] = m[2, 2, 15] = 1
    x = np.arange(20)
    d2 = edt.d2_grid(m)[2, 2]
    np.testing.assert_array_equal(d2, np.minimum((x - 3) ** 2, (x - 15) ** 2))


def test_empty_and_full_grids():
    assert np.all(edt.d2_grid(np.zeros((3, 4, 5), np.uint8)) == edt.NONE)
    assert np.all(np.isinf(edt.dist(edt.d2_grid(np.zeros((2, 2, 2), np.uint8)))))
    assert np.all(edt.d2_grid(np.ones((3, 4, 5), np.uint8)) == 0)


def test_axis_permutation_symmetry():
    m = sitegrid.random_sites(6, 8, 10, p=0.04, seed=5)
    m[0, 0, 0] = 1
    d2 = edt.d2_grid(m)
    for perm in ((2, 1, 0), (1, 2, 0), (0, 2, 1)):
        np.testing.assert_array_equal(edt.d2_grid(np.ascontiguousarray(m.transpose(perm))), d2.transpose(perm))


def test_sampled_points_agree_with_the_grid():
    m = sitegrid.random_sites(10, 11, 12, p=0.02, seed=6)
    m[3, 3, 3] = 1
    pts = np.random.default_rng(7).integers(0, [10, 11, 12], size=(50, 3))
    np.testing.assert_array_equal(edt.d2_at(m, pts), edt.d2_grid(m)[pts[:, 0], pts[:, 1], pts[:, 2]])


def test_room_grid_is_seeded_and_surface_like():
    a, b = sitegrid.room(64, 64, 32, seed=3), sitegrid.room(64, 64, 32, seed=3)
    assert a.shape == (32, 64, 64) and a.dtype == np.uint8
    np.testing.assert_array_equal(a, b)
    frac = a.mean()
    assert 0.01 < frac < 0.2
    assert a[2].all()                                 # the floor
