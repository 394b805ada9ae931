"""Host-only checks of libwb (no GPU needed): the library loads and exports
every entry point the header declares, descriptors are validated with the
documented error codes, and the pair numbering rebuilt from the kernels'
link-block tables equals the oracle's lexicographic enumeration exactly."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2603_05493_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def abi():
    from paper_2603_05493_amd import _abi
    _abi.lib()
    return _abi


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "wb.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(wb_\w+)\s*\(", txt, flags=re.M)))


def test_exports_every_declared_symbol(abi):
    lib = abi.lib()
    names = _header_functions()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(abi.declared_symbols()) == set(names)


def _robot(rb):
    from paper_2603_05493_amd.wb import Robot
    return Robot(rb)


@pytest.mark.parametrize("factory", [lambda: synth.serial_chain(7, 5, seed=0),
                                     lambda: synth.humanoid48(seed=0),
                                     lambda: synth.random_tree(48, 6, seed=3),
                                     lambda: synth.random_tree(23, 6, seed=2),
                                     lambda: synth.random_tree(12, 3, seed=1)])
def test_pair_numbering_matches_oracle(abi, oracle, factory):
    rb = factory()
    r = _robot(rb)
    s, t = r.pairs()
    so, to = oracle.pairs(rb)
    np.testing.assert_array_equal(s, so)
    np.testing.assert_array_equal(t, to)
    assert r.n_pairs == len(so)


def test_sizes_of_the_workloads(abi):
    r = _robot(synth.humanoid48(seed=0))
    assert (r.n_links, r.n_dof, r.n_spheres, r.max_spheres_per_link) == (49, 48, 240, 5)
    assert r.n_pairs == 27040
    assert [_robot(synth.random_tree(n, 6, seed=i)).n_pairs
            for i, (n, _) in enumerate(synth.UNEVEN_TREES)] == [756, 2376, 9108, 40608]


def test_explicit_allow_matrix(abi, oracle):
    rb = synth.random_tree(9, 2, seed=4)
    L = rb.n_links
    rng = np.random.default_rng(5)
    allow = np.triu((rng.uniform(size=(L, L)) < 0.5).astype(np.uint8), 1)
    rb.allow = allow + allow.T
    s, t = _robot(rb).pairs()
    so, to = oracle.pairs(rb)
    np.testing.assert_array_equal(s, so)
    np.testing.assert_array_equal(t, to)


def _expect(abi, code, mutate):
    rb = synth.serial_chain(4, 2, seed=1)
    mutate(rb)
    from paper_2603_05493_amd.wb import Robot
    with pytest.raises(abi.WbError) as e:
        Robot(rb)
    assert e.value.code == code, str(e.value)


def test_rejects_bad_descriptors(abi):
    E = abi
    _expect(E, E.WB_ERR_INVALID_TREE, lambda rb: rb.parent.__setitem__(2, 3))      # parent after child
    _expect(E, E.WB_ERR_INVALID_TREE, lambda rb: rb.parent.__setitem__(3, 3))      # self loop / cycle
    _expect(E, E.WB_ERR_INVALID_TREE, lambda rb: rb.parent.__setitem__(0, 0))      # root has a parent
    _expect(E, E.WB_ERR_INVALID_TREE, lambda rb: rb.axis.__setitem__(2, [1.0, 1.0, 0.0]))  # non-unit axis
    _expect(E, E.WB_ERR_INVALID_TREE, lambda rb: rb.sphere_link.__setitem__(-1, 7))  # missing link
    _expect(E, E.WB_ERR_INVALID_TREE, lambda rb: rb.sphere_link.__setitem__(0, 3))   # not sorted
    _expect(E, E.WB_ERR_INVALID_TREE, lambda rb: rb.joint_index.__setitem__(3, 1))   # joint 2 unused
    _expect(E, E.WB_ERR_INVALID_TREE, lambda rb: rb.joint_type.__setitem__(0, 1))    # jointed root
    _expect(E, E.WB_ERR_INVALID_TREE, lambda rb: rb.fixed_R.__setitem__(1, 2 * np.eye(3)))
    _expect(E, E.WB_ERR_INVALID_ARG, lambda rb: rb.sphere_r.__setitem__(0, -0.1))
    _expect(E, E.WB_ERR_INVALID_ARG, lambda rb: rb.mass.__setitem__(1, np.nan))
    _expect(E, E.WB_ERR_INVALID_ARG, lambda rb: rb.inertia.__setitem__(1, np.array([[1, 2, 0], [0, 1, 0], [0, 0, 1.0]])))


def test_rejects_unsupported_sizes(abi):
    from paper_2603_05493_amd.wb import Robot
    rb = synth.serial_chain(3, 65, seed=0)                # 65 spheres on one link
    with pytest.raises(abi.WbError) as e:
        Robot(rb)
    assert e.value.code == abi.WB_ERR_UNSUPPORTED
    # nine per link are fine, padded to 12 slots, which the fused iteration takes;
    # thirteen pad to 16, which only the per-operation calls take
    r = Robot(synth.serial_chain(3, 9, seed=0))
    assert r.max_spheres_per_link == 9 and r.fused_supported
    r = Robot(synth.serial_chain(3, 13, seed=0))
    assert r.max_spheres_per_link == 13 and not r.fused_supported


def test_paper_scale_humanoid_sizes(abi):
    from paper_2603_05493_amd.wb import Robot
    r = Robot(synth.humanoid48_paper_scale())
    assert (r.n_links, r.n_dof, r.n_spheres) == (49, 48, 588)
    assert r.n_pairs == 162432 and r.max_spheres_per_link == 12 and r.n_blocks == 1128
    assert r.fused_supported


def test_asymmetric_allow_rejected(abi):
    rb = synth.serial_chain(3, 1, seed=0)
    a = np.zeros((4, 4), np.uint8)
    a[0, 2] = 1
    rb.allow = a
    from paper_2603_05493_amd.wb import Robot
    with pytest.raises(abi.WbError) as e:
        Robot(rb)
    assert e.value.code == abi.WB_ERR_INVALID_ARG


def test_null_descriptor_and_outputs(abi):
    lib = abi.lib()
    info = abi.WbRobotInfo()
    assert lib.wb_desc_analyze(None, C.byref(info)) == abi.WB_ERR_INVALID_ARG
    assert "null" in lib.wb_last_error().decode()
    r = _robot(synth.serial_chain(2, 1))
    assert lib.wb_desc_analyze(C.byref(r.desc), None) == abi.WB_ERR_INVALID_ARG
    h = C.c_void_p()
    assert lib.wb_robot_create(None, C.byref(h)) == abi.WB_ERR_INVALID_ARG
    assert lib.wb_robot_create(C.byref(r.desc), None) == abi.WB_ERR_INVALID_ARG


def test_launch_calls_reject_null_robot(abi):
    lib = abi.lib()
    assert lib.wb_fk(None, 4, 0, None, None, None, None) == abi.WB_ERR_INVALID_ARG
    assert lib.wb_self_collision(None, 4, 0, None, None, None, None, None) == abi.WB_ERR_INVALID_ARG
    assert lib.wb_cost_head(-1, 0, 3, None, None, 0.0, None, 0.0, 0.0, None, None, None, None) == \
        abi.WB_ERR_INVALID_ARG
    # B = 0 with no pointers is a valid no-op for the robot-free kernels
    assert lib.wb_sgd_step(0, 0, 3, 0.1, None, None, None, None, None, None, None, None) == abi.WB_OK


def test_leading_dimension_below_B_is_rejected(abi):
    """ld = 0 means ld = B; an ld below B is refused before any launch."""
    lib = abi.lib()
    E = abi.WB_ERR_INVALID_ARG
    assert lib.wb_cost_head(8, 7, 3, None, None, 0.0, None, 0.0, 0.0, None, None, None, None) == E
    assert "ld 7 is below B 8" in lib.wb_last_error().decode()
    assert lib.wb_sgd_step(8, 5, 3, 0.1, None, None, None, None, None, None, None, None) == E
    assert lib.wb_sgd_step(0, 0, 3, 0.1, None, None, None, None, None, None, None, None) == abi.WB_OK


def test_bspline_calls_validate_arguments(abi):
    lib = abi.lib()
    E = abi.WB_ERR_INVALID_ARG
    ev = lambda T, d, K, n, dt, rd, U=None, th=None, q=None: lib.wb_bspline_eval(T, d, K, n, dt, rd, U, th, None,
                                                                                  None, q, None, None, None)
    # empty batches are valid no-ops
    assert ev(0, 4, 9, 4, 0.05, 0) == abi.WB_OK
    assert lib.wb_bspline_backward(0, 4, 9, 4, 0.05, None, None, None, None, 0.0, 0, None, None) == abi.WB_OK
    # shape and parameter checks come before any launch
    assert ev(1, 4, 0, 4, 0.05, 0) == E                      # no control points
    assert ev(1, 4, 9, 0, 0.05, 0) == E                      # no samples per interval
    assert ev(1, 4, 9, 4, 0.0, 0) == E                       # dt must be > 0
    assert ev(1, 4, 9, 4, float("nan"), 0) == E
    assert ev(1, 4, 9, 4, 0.05, 2) == E                      # unknown ghost-knot reading
    assert ev(-1, 4, 9, 4, 0.05, 0) == E
    assert ev(1, 4, 9, 4, 0.05, 0) == E                      # U, theta0 and q are required
    assert "U" in lib.wb_last_error().decode()
    # the gradient needs somewhere to go: g_U, or U with a step
    assert lib.wb_bspline_backward(1, 4, 9, 4, 0.05, None, None, None, None, 0.0, 0, None, None) == E
    assert lib.wb_bspline_backward(1, 4, 9, 4, 0.05, None, None, None, None, 0.1, 0, None, None) == E
    assert lib.wb_bspline_backward(1, 4, 9, 4, 0.05, None, None, None, None, float("inf"), 0, None, None) == E
    # an unknown step rule, and the row-normalized step without g_U
    assert lib.wb_bspline_backward(1, 4, 9, 4, 0.05, None, None, None, None, 0.1, 2, None, None) == E
    assert "step rule" in lib.wb_last_error().decode()
    dummy = C.c_void_p(256)   # never dereferenced: the check fails first
    assert lib.wb_bspline_backward(1, 4, 9, 4, 0.05, None, None, None, None, 0.1, 1, dummy, None) == E
    assert "g_U" in lib.wb_last_error().decode()


def test_peak_probe_library_loads_and_rejects_bad_sizes():
    """The benchmark's FP32 FMA-rate probe (libwb_peak.so) loads, exports its
    two calls, counts its FLOP, and refuses empty launches without touching
    the device."""
    import ctypes as C
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2603_05493_amd",
                        "libwb_peak.so")
    lib = C.CDLL(path)
    lib.wb_peak_fma_flop.argtypes = [C.c_int64, C.c_int32]
    lib.wb_peak_fma_flop.restype = C.c_double
    assert lib.wb_peak_fma_flop(8192, 4096) == 8192 * 256 * 4096 * 16 * 2
    lib.wb_peak_fma.argtypes = [C.c_int64, C.c_int32, C.c_float, C.c_float, C.c_void_p, C.c_void_p]
    lib.wb_peak_fma.restype = C.c_int
    assert lib.wb_peak_fma(0, 10, 1.0, 0.0, None, None) != 0
    assert lib.wb_peak_fma(16, 0, 1.0, 0.0, None, None) != 0
