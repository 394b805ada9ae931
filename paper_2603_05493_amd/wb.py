"""Python binding of libwb: the C-ABI calls under the same names, taking torch
tensors for device memory and the current HIP stream, plus
``torch.autograd.Function`` wrappers.

Only argument marshalling happens here; every step runs in the HIP kernels
of libwb.  Batched tensors are [k, B] float32, contiguous, on the robot's
device (state index fastest), exactly as the C ABI documents.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Tuple

import numpy as np
import torch

from . import _abi
from ._abi import WbRobotDesc, WbRobotInfo, check, lib


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _p(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _chk(t: Optional[torch.Tensor], name: str, shape=None, dtype=torch.float32, device=None):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


class Robot:
    """A robot description bound to libwb.

    ``desc`` is any object with the fields of ``synth.Robot``.  The host
    tables (validation, pair numbering) need no GPU; ``to_device`` uploads
    the kernel tables to the current HIP device.
    """

    def __init__(self, desc):
        f = lambda a: np.ascontiguousarray(np.asarray(a), dtype=np.float32)
        i = lambda a: np.ascontiguousarray(np.asarray(a), dtype=np.int32)
        L = int(np.asarray(desc.parent).shape[0])
        S = int(np.asarray(desc.sphere_link).shape[0])
        sph = np.concatenate([np.asarray(desc.sphere_pos, dtype=np.float64).reshape(S, 3),
                              np.asarray(desc.sphere_r, dtype=np.float64).reshape(S, 1)], 1)
        self._keep = dict(
            parent=i(desc.parent), joint_type=i(desc.joint_type), joint_index=i(desc.joint_index),
            joint_mult=f(desc.joint_mult), joint_offset=f(desc.joint_offset), axis=f(desc.axis),
            fixed_R=f(desc.fixed_R).reshape(L, 9), fixed_p=f(desc.fixed_p), mass=f(desc.mass),
            com=f(desc.com), inertia=f(desc.inertia).reshape(L, 9), sphere_link=i(desc.sphere_link),
            sphere=f(sph) if S else np.zeros((1, 4), np.float32),
        )
        allow = getattr(desc, "allow", None)
        self._allow = None if allow is None else np.ascontiguousarray(allow, dtype=np.uint8)
        k = self._keep
        fp = lambda a: a.ctypes.data_as(C.POINTER(C.c_float))
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        g = np.asarray(desc.gravity, dtype=np.float32)
        self.desc = WbRobotDesc(
            L, ip(k["parent"]), ip(k["joint_type"]), ip(k["joint_index"]), fp(k["joint_mult"]),
            fp(k["joint_offset"]), fp(k["axis"]), fp(k["fixed_R"]), fp(k["fixed_p"]), fp(k["mass"]),
            fp(k["com"]), fp(k["inertia"]), S, ip(k["sphere_link"]), fp(k["sphere"]),
            self._allow.ctypes.data_as(C.POINTER(C.c_uint8)) if self._allow is not None else None,
            (C.c_float * 3)(*g.tolist()),
        )
        inf = WbRobotInfo()
        check(lib().wb_desc_analyze(C.byref(self.desc), C.byref(inf)))
        self.n_links, self.n_dof, self.n_spheres = inf.n_links, inf.n_dof, inf.n_spheres
        self.max_depth, self.n_pairs, self.n_blocks = inf.max_depth, inf.n_pairs, inf.n_blocks
        self.max_spheres_per_link = inf.max_spheres_per_link
        self.fused_supported = bool(inf.fused_supported)
        self.kinematics_supported = bool(inf.kinematics_supported)
        self.has_mimic = bool(inf.mimic)
        self.n_tools = 0
        self.handle = None
        self.device = None

    def pairs(self) -> Tuple[np.ndarray, np.ndarray]:
        P = self.n_pairs
        s = np.empty(max(P, 1), np.int32)
        t = np.empty(max(P, 1), np.int32)
        check(lib().wb_desc_pairs(C.byref(self.desc), s.ctypes.data_as(C.POINTER(C.c_int32)),
                                  t.ctypes.data_as(C.POINTER(C.c_int32))))
        return s[:P], t[:P]

    def to_device(self, device=None) -> "Robot":
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(dev):
            h = C.c_void_p()
            check(lib().wb_robot_create(C.byref(self.desc), C.byref(h)))
        self.handle, self.device = h, dev
        return self

    def workspace_bytes(self, B: int) -> int:
        n = C.c_size_t()
        check(lib().wb_workspace_bytes(self.handle, B, C.byref(n)))
        return n.value

    def rnea_cache_bytes(self, B: int) -> int:
        n = C.c_size_t()
        check(lib().wb_rnea_cache_bytes(self.handle, B, C.byref(n)))
        return n.value

    def set_tune(self, lanes_per_state: int, states_per_item: int, ns_per_state: float = 0.0) -> None:
        t = _abi.WbTune(int(lanes_per_state), int(states_per_item), float(ns_per_state))
        check(lib().wb_robot_set_tune(self.handle, C.byref(t)))

    def set_dispatch(self, sweep_split_below: int = -1, fk_groups_below: int = -1,
                     fk_pose_groups_below: int = -1) -> None:
        """Batch thresholds of the per-operation forms (wb_robot_set_dispatch):
        wb_self_collision sweeps one state per workgroup below the first,
        wb_fk / wb_fk_backward take one group of lanes per state below the
        second (no link poses involved) or the third (poses written or
        read); < 0 restores a default, 0 never takes the form."""
        self._dispatch = (int(sweep_split_below), int(fk_groups_below), int(fk_pose_groups_below))
        check(lib().wb_robot_set_dispatch(self.handle, *self._dispatch))

    def set_sweep_split(self, below: int) -> None:
        """Only the self-collision threshold of set_dispatch (the others kept)."""
        self.set_dispatch(below, *getattr(self, "_dispatch", (-1, -1, -1))[1:])

    def set_link_inertia(self, link: int, mass: float, com, inertia) -> None:
        """Replace one link's mass, CoM and inertia about the CoM (xx yy zz xy
        xz yz, link axes) on the device, e.g. for a payload; blocking, call
        between launches."""
        c = (C.c_float * 3)(*[float(x) for x in com])
        i6 = (C.c_float * 6)(*[float(x) for x in inertia])
        check(lib().wb_robot_set_link_inertia(self.handle, int(link), float(mass), c, i6))

    def set_tool_frames(self, links, R=None, p=None) -> None:
        """Tool frames fixed to `links` [T] with offsets R [T,3,3] (identity by
        default) and p [T,3] (zero by default) in the link frames; blocking,
        call between launches.  An empty list clears them."""
        links = np.ascontiguousarray(np.asarray(links, dtype=np.int32).reshape(-1))
        T = links.shape[0]
        R = np.tile(np.eye(3), (T, 1, 1)) if R is None else np.asarray(R, dtype=np.float64).reshape(T, 3, 3)
        p = np.zeros((T, 3)) if p is None else np.asarray(p, dtype=np.float64).reshape(T, 3)
        off = np.ascontiguousarray(np.concatenate([R.reshape(T, 9), p], 1), dtype=np.float32)
        check(lib().wb_robot_set_tool_frames(self.handle, T, links.ctypes.data_as(C.c_void_p),
                                             off.ctypes.data_as(C.c_void_p)))
        self.n_tools = T

    def get_tune(self) -> dict:
        t = _abi.WbTune()
        check(lib().wb_robot_get_tune(self.handle, C.byref(t)))
        return {"lanes_per_state": t.lanes_per_state, "states_per_item": t.states_per_item,
                "ns_per_state": t.ns_per_state}

    def topology_key(self) -> str:
        """Hash of what the launch shape depends on: topology, spheres per link."""
        import hashlib
        k = self._keep
        counts = np.bincount(k["sphere_link"], minlength=self.n_links) if self.n_spheres else np.zeros(1)
        h = hashlib.sha1(k["parent"].tobytes() + k["joint_type"].tobytes() + counts.astype(np.int32).tobytes())
        return f"L{self.n_links}_S{self.n_spheres}_{h.hexdigest()[:12]}"

    def workspace(self, B: int) -> torch.Tensor:
        return torch.empty(max(self.workspace_bytes(B) // 4, 1), dtype=torch.float32, device=self.device)

    def close(self):
        if self.handle is not None:
            check(lib().wb_robot_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _empty(shape, robot: Robot, dtype=torch.float32):
    return torch.empty(shape, dtype=dtype, device=robot.device)


# ------------------------------------------------------------------ the ABI
#
# The [k][B] arrays of the hot-path calls may have padded rows: their last
# dimension is the leading dimension ld, and `nb` (default ld) states are
# processed; per-state arrays have nb entries.


def _nb(ld: int, nb: Optional[int]) -> int:
    if nb is None:
        return ld
    if not 0 <= nb <= ld:
        raise ValueError(f"nb={nb} must be within [0, {ld}] (the arrays' last dimension)")
    return int(nb)


def wb_fk(robot: Robot, q: torch.Tensor, link_pose=None, spheres=None, want_spheres=True, want_pose=True,
          nb=None):
    n, ld = robot.n_dof, q.shape[-1]
    B = _nb(ld, nb)
    L, S = robot.n_links, robot.n_spheres
    if link_pose is None and want_pose:
        link_pose = _empty((L, 12, ld), robot)
    if spheres is None and want_spheres:
        spheres = _empty((S, 3, ld), robot)
    _chk(q, "q", (n, ld), device=robot.device)
    _chk(link_pose, "link_pose", (L, 12, ld), device=robot.device)
    _chk(spheres, "spheres", (S, 3, ld), device=robot.device)
    check(lib().wb_fk(robot.handle, B, ld, _p(q), _p(link_pose), _p(spheres), _stream()))
    return link_pose, spheres


def wb_kinematics(robot: Robot, q, link_pose=False, spheres=False, tool_pose=True, com=True, jacobian=True,
                  com_jacobian=False):
    """One launch of the kinematics outputs.  Each argument is False (skip),
    True (allocate) or a tensor to fill; returns a dict of the requested
    outputs: link_pose [L,12,B], spheres [S,3,B], tool_pose [T,12,B],
    com [3,B], and the state-major jacobian [B,T,6,n] and com_jacobian
    [B,3,n]."""
    n, B, L, S, T = robot.n_dof, q.shape[-1], robot.n_links, robot.n_spheres, robot.n_tools
    shapes = dict(link_pose=(L, 12, B), spheres=(S, 3, B), tool_pose=(T, 12, B), com=(3, B),
                  jacobian=(B, T, 6, n), com_jacobian=(B, 3, n))
    want = dict(link_pose=link_pose, spheres=spheres, tool_pose=tool_pose, com=com, jacobian=jacobian,
                com_jacobian=com_jacobian)
    out = {}
    for k, v in want.items():
        if v is True:
            out[k] = _empty(shapes[k], robot)
        elif v is not False and v is not None:
            _chk(v, k, shapes[k], device=robot.device)
            out[k] = v
    _chk(q, "q", (n, B), device=robot.device)
    check(lib().wb_kinematics(robot.handle, B, _p(q), *[_p(out.get(k)) for k in shapes], _stream()))
    return out


def wb_kinematics_backward(robot: Robot, q, g_tool_pose=None, g_com=None, g_q=None):
    """dL/dq [n,B] for L = <g_tool_pose, tool_pose> + <g_com, com>."""
    n, B, T = robot.n_dof, q.shape[-1], robot.n_tools
    g_q = _empty((n, B), robot) if g_q is None else g_q
    _chk(q, "q", (n, B), device=robot.device)
    _chk(g_tool_pose, "g_tool_pose", (T, 12, B), device=robot.device)
    _chk(g_com, "g_com", (3, B), device=robot.device)
    _chk(g_q, "g_q", (n, B), device=robot.device)
    check(lib().wb_kinematics_backward(robot.handle, B, _p(q), _p(g_tool_pose), _p(g_com), _p(g_q), _stream()))
    return g_q


EDT_NONE = -1


def edt_workspace_bytes(nx: int, ny: int, nz: int) -> int:
    n = C.c_size_t()
    check(lib().wb_edt_workspace_bytes(int(nx), int(ny), int(nz), C.byref(n)))
    return n.value


def wb_edt(sites: torch.Tensor, voxel_size: float = 1.0, nearest=True, dist=True, workspace=None):
    """Exact Euclidean distance transform of a uint8 site grid [nz, ny, nx]:
    returns (nearest [nz, ny, nx] int32 packed x | y << 10 | z << 20 or -1,
    dist [nz, ny, nx] float32, voxel_size * distance or +inf); either may be
    False to skip or a tensor to fill."""
    if sites.dim() != 3:
        raise ValueError("sites must be [nz, ny, nx]")
    nz, ny, nx = sites.shape
    _chk(sites, "sites", (nz, ny, nx), torch.uint8)
    dev = sites.device
    if nearest is True:
        nearest = torch.empty((nz, ny, nx), dtype=torch.int32, device=dev)
    if dist is True:
        dist = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
    nearest = None if nearest is False else nearest
    dist = None if dist is False else dist
    _chk(nearest, "nearest", (nz, ny, nx), torch.int32)
    _chk(dist, "dist", (nz, ny, nx))
    need = edt_workspace_bytes(nx, ny, nz)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError("workspace too small")
    check(lib().wb_edt(nx, ny, nz, _p(sites), float(voxel_size), _p(nearest), _p(dist), _p(workspace), _stream()))
    return nearest, dist


EDT_NOALLOC_MAX_VOXELS = 1 << 23


def wb_edt_noalloc(sites: torch.Tensor, voxel_size: float = 1.0, nearest=None, dist=None):
    """wb_edt without a workspace: the library's per-device scratch array
    serves as one (grids of at most EDT_NOALLOC_MAX_VOXELS voxels).  The
    outputs must be given as tensors (or None to skip); nothing is
    allocated, so the call may run where allocation is not allowed."""
    if sites.dim() != 3:
        raise ValueError("sites must be [nz, ny, nx]")
    nz, ny, nx = sites.shape
    _chk(sites, "sites", (nz, ny, nx), torch.uint8)
    _chk(nearest, "nearest", (nz, ny, nx), torch.int32)
    _chk(dist, "dist", (nz, ny, nx))
    check(lib().wb_edt_noalloc(nx, ny, nz, _p(sites), float(voxel_size), _p(nearest), _p(dist), _stream()))
    return nearest, dist


def wb_rnea(robot: Robot, q, qd, qdd, tau=None, cache=None, f_ext=None, want_cache=True, nb=None):
    """tau [n,B] and the cache for the backward (None with want_cache=False:
    nothing is stored and the backward recomputes); f_ext [L,6,B] external
    link forces in link coordinates (moment, force), or None."""
    n, ld, L = robot.n_dof, q.shape[-1], robot.n_links
    B = _nb(ld, nb)
    tau = _empty((n, ld), robot) if tau is None else tau
    if cache is None and want_cache:
        cache = _empty((L, 18, ld), robot)
    for t, nm in ((q, "q"), (qd, "qd"), (qdd, "qdd"), (tau, "tau")):
        _chk(t, nm, (n, ld), device=robot.device)
    _chk(cache, "cache", (L, 18, ld), device=robot.device)
    _chk(f_ext, "f_ext", (L, 6, ld), device=robot.device)
    check(lib().wb_rnea(robot.handle, B, ld, _p(q), _p(qd), _p(qdd), _p(f_ext), _p(tau), _p(cache), _stream()))
    return tau, cache


def wb_self_collision(robot: Robot, spheres, max_pen=None, argmax=None, n_coll=None, nb=None):
    S, ld = robot.n_spheres, spheres.shape[-1]
    B = _nb(ld, nb)
    max_pen = _empty((B,), robot) if max_pen is None else max_pen
    argmax = _empty((B,), robot, torch.int32) if argmax is None else argmax
    n_coll = _empty((B,), robot, torch.int32) if n_coll is None else n_coll
    _chk(spheres, "spheres", (S, 3, ld), device=robot.device)
    _chk(max_pen, "max_pen", (B,), device=robot.device)
    _chk(argmax, "argmax", (B,), torch.int32, device=robot.device)
    _chk(n_coll, "n_coll", (B,), torch.int32, device=robot.device)
    check(lib().wb_self_collision(robot.handle, B, ld, _p(spheres), _p(max_pen), _p(argmax), _p(n_coll),
                                  _stream()))
    return max_pen, argmax, n_coll


def wb_self_collision_backward(robot: Robot, spheres, argmax, max_pen, margin: float, g_cost,
                               g_spheres=None, nb=None):
    S, ld = robot.n_spheres, spheres.shape[-1]
    B = _nb(ld, nb)
    g_spheres = _empty((S, 3, ld), robot) if g_spheres is None else g_spheres
    _chk(spheres, "spheres", (S, 3, ld), device=robot.device)
    _chk(argmax, "argmax", (B,), torch.int32, device=robot.device)
    _chk(max_pen, "max_pen", (B,), device=robot.device)
    _chk(g_cost, "g_cost", (B,), device=robot.device)
    _chk(g_spheres, "g_spheres", (S, 3, ld), device=robot.device)
    check(lib().wb_self_collision_backward(robot.handle, B, ld, _p(spheres), _p(argmax), _p(max_pen),
                                           float(margin), _p(g_cost), _p(g_spheres), _stream()))
    return g_spheres


def wb_fk_backward(robot: Robot, q, g_spheres=None, g_link_pose=None, link_pose=None, g_q=None,
                   workspace=None, nb=None):
    n, ld, L, S = robot.n_dof, q.shape[-1], robot.n_links, robot.n_spheres
    B = _nb(ld, nb)
    g_q = _empty((n, ld), robot) if g_q is None else g_q
    workspace = robot.workspace(ld) if workspace is None else workspace
    _chk(q, "q", (n, ld), device=robot.device)
    _chk(g_spheres, "g_spheres", (S, 3, ld), device=robot.device)
    _chk(g_link_pose, "g_link_pose", (L, 12, ld), device=robot.device)
    _chk(link_pose, "link_pose", (L, 12, ld), device=robot.device)
    _chk(g_q, "g_q", (n, ld), device=robot.device)
    if workspace.numel() * workspace.element_size() < robot.workspace_bytes(ld):
        raise ValueError("workspace too small")
    check(lib().wb_fk_backward(robot.handle, B, ld, _p(q), _p(link_pose), _p(g_link_pose), _p(g_spheres),
                               _p(g_q), _p(workspace), _stream()))
    return g_q


def wb_rnea_backward(robot: Robot, q, qd, qdd, cache, g_tau, g_q=None, g_qd=None, g_qdd=None,
                     workspace=None, g_fext=None, f_ext=None, nb=None):
    """g_q, g_qd, g_qdd [n,B]; with g_fext [L,6,B] also the gradient on the
    external forces.  cache: the forward call's (its forces included), or
    None to recompute every forward quantity from q, qd, qdd and f_ext."""
    n, ld, L = robot.n_dof, q.shape[-1], robot.n_links
    B = _nb(ld, nb)
    g_q = _empty((n, ld), robot) if g_q is None else g_q
    g_qd = _empty((n, ld), robot) if g_qd is None else g_qd
    g_qdd = _empty((n, ld), robot) if g_qdd is None else g_qdd
    if cache is not None and workspace is None:
        workspace = robot.workspace(ld)
    for t, nm in ((q, "q"), (qd, "qd"), (qdd, "qdd"), (g_tau, "g_tau"), (g_q, "g_q"), (g_qd, "g_qd"),
                  (g_qdd, "g_qdd")):
        _chk(t, nm, (n, ld), device=robot.device)
    _chk(cache, "cache", (L, 18, ld), device=robot.device)
    _chk(g_fext, "g_fext", (L, 6, ld), device=robot.device)
    _chk(f_ext, "f_ext", (L, 6, ld), device=robot.device)
    if workspace is not None and workspace.numel() * workspace.element_size() < robot.workspace_bytes(ld):
        raise ValueError("workspace too small")
    check(lib().wb_rnea_backward(robot.handle, B, ld, _p(q), _p(qd), _p(qdd), _p(f_ext), _p(cache), _p(g_tau),
                                 _p(g_q), _p(g_qd), _p(g_qdd), _p(g_fext), _p(workspace), _stream()))
    return g_q, g_qd, g_qdd


def wb_cost_head(tau, w=None, torque_weight=0.0, max_pen=None, margin=0.0, hinge_weight=0.0,
                 cost=None, g_tau=None, g_maxpen=None, nb=None):
    n, ld = tau.shape
    B = _nb(ld, nb)
    dev = tau.device
    cost = torch.empty(B, dtype=torch.float32, device=dev) if cost is None else cost
    g_tau = torch.empty_like(tau) if g_tau is None else g_tau
    if max_pen is not None and g_maxpen is None:
        g_maxpen = torch.empty(B, dtype=torch.float32, device=dev)
    for t, nm, shp in ((tau, "tau", (n, ld)), (w, "w", (n, ld)), (max_pen, "max_pen", (B,)), (cost, "cost", (B,)),
                       (g_tau, "g_tau", (n, ld)), (g_maxpen, "g_maxpen", (B,))):
        _chk(t, nm, shp, device=dev)
    check(lib().wb_cost_head(B, ld, n, _p(tau), _p(w), float(torque_weight), _p(max_pen), float(margin),
                             float(hinge_weight), _p(cost), _p(g_tau), _p(g_maxpen), _stream()))
    return cost, g_tau, g_maxpen


def wb_sgd_step(lr: float, q, qd, qdd, g_q, g_qd, g_qdd, g_q2=None, nb=None):
    n, ld = q.shape
    B = _nb(ld, nb)
    for t, nm in ((q, "q"), (qd, "qd"), (qdd, "qdd"), (g_q, "g_q"), (g_qd, "g_qd"), (g_qdd, "g_qdd"),
                  (g_q2, "g_q2")):
        _chk(t, nm, (n, ld), device=q.device)
    check(lib().wb_sgd_step(B, ld, n, float(lr), _p(q), _p(qd), _p(qdd), _p(g_q), _p(g_q2), _p(g_qd),
                            _p(g_qdd), _stream()))


GHOST_EXACT, GHOST_PRINTED = 0, 1
BSPLINE_MAX_K = 65536


def bspline_horizon(K: int, n_interp: int) -> int:
    """Samples per trajectory: K + 3 segments of n_interp samples."""
    return (K + 3) * n_interp


def wb_bspline_eval(U, theta0, dt: float, n_interp: int = 4, dtheta0=None, ddtheta0=None, q=None, qd=None,
                    qdd=None, reading: int = GHOST_EXACT):
    """Sample the control points U [d][T][K] into q, qd, qdd [d][T*H]
    (allocated when None; qd and qdd are skipped when passed as False)."""
    d, T, K = U.shape
    H = bspline_horizon(K, n_interp)
    _chk(U, "U", (d, T, K), device=U.device)
    for t, nm in ((theta0, "theta0"), (dtheta0, "dtheta0"), (ddtheta0, "ddtheta0")):
        _chk(t, nm, (d, T), device=U.device)
    outs = []
    for t, nm in ((q, "q"), (qd, "qd"), (qdd, "qdd")):
        if t is False:
            outs.append(None)
            continue
        if t is None:
            t = torch.empty((d, T * H), dtype=torch.float32, device=U.device)
        _chk(t, nm, (d, T * H), device=U.device)
        outs.append(t)
    check(lib().wb_bspline_eval(T, d, K, n_interp, float(dt), int(reading), _p(U), _p(theta0), _p(dtheta0),
                                _p(ddtheta0), _p(outs[0]), _p(outs[1]), _p(outs[2]), _stream()))
    return tuple(outs)


STEP_PLAIN, STEP_ROW_RMS = 0, 1


def wb_bspline_backward(K: int, T: int, dt: float, n_interp: int = 4, g_q=None, g_qd=None, g_qdd=None, g_U=None,
                        lr: float = 0.0, U=None, step_rule: int = STEP_PLAIN):
    """Control-point gradient [d][T][K] of upstream sample gradients
    [d][T*H]; with lr != 0 also the step on U in place: U -= lr * g_U
    (STEP_PLAIN), or each (joint, trajectory) row of K control points moved
    by lr * g / rms(g) (STEP_ROW_RMS)."""
    ref = next(t for t in (g_q, g_qd, g_qdd) if t is not None)
    d = ref.shape[0]
    H = bspline_horizon(K, n_interp)
    for t, nm in ((g_q, "g_q"), (g_qd, "g_qd"), (g_qdd, "g_qdd")):
        _chk(t, nm, (d, T * H), device=ref.device)
    if g_U is None and (lr == 0.0 or step_rule == STEP_ROW_RMS):
        g_U = torch.empty((d, T, K), dtype=torch.float32, device=ref.device)
    _chk(g_U, "g_U", (d, T, K), device=ref.device)
    _chk(U, "U", (d, T, K), device=ref.device)
    check(lib().wb_bspline_backward(T, d, K, n_interp, float(dt), _p(g_q), _p(g_qd), _p(g_qdd), _p(g_U),
                                    float(lr), int(step_rule), _p(U), _stream()))
    return g_U


def wb_wholebody_step(robot: Robot, q, qd, qdd, w=None, torque_weight=0.0, margin=0.0, hinge_weight=0.0,
                      lr=0.0, tau=None, cost=None, max_pen=None, argmax=None, n_coll=None, g_q=None,
                      g_qd=None, g_qdd=None, f_ext=None, g_fext=None, nb=None):
    """One fused iteration (FK, self-collision, RNEA, cost head, adjoints,
    optional in-place step on q, qd, qdd).  Outputs left as None are skipped.
    f_ext [L,6,B]: external link forces (link coordinates, moment then force);
    g_fext [L,6,B]: their gradient."""
    n, ld, L = robot.n_dof, q.shape[-1], robot.n_links
    B = _nb(ld, nb)
    _chk(f_ext, "f_ext", (L, 6, ld), device=robot.device)
    _chk(g_fext, "g_fext", (L, 6, ld), device=robot.device)
    for t, nm in ((q, "q"), (qd, "qd"), (qdd, "qdd"), (w, "w"), (tau, "tau"), (g_q, "g_q"), (g_qd, "g_qd"),
                  (g_qdd, "g_qdd")):
        _chk(t, nm, (n, ld), device=robot.device)
    _chk(cost, "cost", (B,), device=robot.device)
    _chk(max_pen, "max_pen", (B,), device=robot.device)
    _chk(argmax, "argmax", (B,), torch.int32, device=robot.device)
    _chk(n_coll, "n_coll", (B,), torch.int32, device=robot.device)
    check(lib().wb_wholebody_step(robot.handle, B, ld, _p(q), _p(qd), _p(qdd), _p(w), float(torque_weight),
                                  float(margin), float(hinge_weight), float(lr), _p(tau), _p(cost),
                                  _p(max_pen), _p(argmax), _p(n_coll), _p(g_q), _p(g_qd), _p(g_qdd),
                                  _p(f_ext), _p(g_fext), _stream()))


def wb_wholebody_step_bspline(robot: Robot, U, theta0, dt: float, dtheta0=None, ddtheta0=None,
                              reading: int = GHOST_EXACT, w=None, torque_weight=0.0, margin=0.0, hinge_weight=0.0,
                              g_U=None, lr: float = 0.0, step_rule: int = STEP_PLAIN, tau=None, cost=None,
                              max_pen=None, argmax=None, n_coll=None, g_q=None, g_qd=None, g_qdd=None):
    """The B-spline iteration in one launch: the fused iteration over the
    four-per-interval samples of the splines U [d][T][K] (formed in the
    kernel), and with g_U or lr != 0 the control-point gradient reduced in
    the kernel and the step on U; per-state outputs as wb_wholebody_step for
    the T * H states, None to skip."""
    d, T, K = U.shape
    H = bspline_horizon(K, 4)
    B = T * H
    _chk(U, "U", (d, T, K), device=robot.device)
    for t, nm in ((theta0, "theta0"), (dtheta0, "dtheta0"), (ddtheta0, "ddtheta0")):
        _chk(t, nm, (d, T), device=robot.device)
    for t, nm in ((w, "w"), (tau, "tau"), (g_q, "g_q"), (g_qd, "g_qd"), (g_qdd, "g_qdd")):
        _chk(t, nm, (d, B), device=robot.device)
    _chk(cost, "cost", (B,), device=robot.device)
    _chk(max_pen, "max_pen", (B,), device=robot.device)
    _chk(argmax, "argmax", (B,), torch.int32, device=robot.device)
    _chk(n_coll, "n_coll", (B,), torch.int32, device=robot.device)
    _chk(g_U, "g_U", (d, T, K), device=robot.device)
    check(lib().wb_wholebody_step_bspline(robot.handle, T, K, float(dt), int(reading), _p(U), _p(theta0),
                                          _p(dtheta0), _p(ddtheta0), _p(w), float(torque_weight), float(margin),
                                          float(hinge_weight), _p(g_U), float(lr), int(step_rule), _p(tau), _p(cost),
                                          _p(max_pen), _p(argmax), _p(n_coll), _p(g_q), _p(g_qd), _p(g_qdd),
                                          _stream()))


class Plan:
    """An uneven batch of robots run by one persistent launch (wb_plan_*)."""

    def __init__(self, robots, B, tunes=None):
        self.robots, self.B = list(robots), [int(b) for b in B]
        n = len(self.robots)
        handles = (C.c_void_p * n)(*[r.handle.value for r in self.robots])
        bs = (C.c_int64 * n)(*self.B)
        tn = None
        if tunes is not None:
            tn = (_abi.WbTune * n)(*[_abi.WbTune(int(t["lanes_per_state"]), int(t["states_per_item"]),
                                                 float(t.get("ns_per_state", 0.0))) for t in tunes])
        h = C.c_void_p()
        check(lib().wb_plan_create(C.cast(handles, C.POINTER(C.c_void_p)), bs, n, tn, C.byref(h)))
        self.handle = h
        ni, nw = C.c_int32(), C.c_int32()
        check(lib().wb_plan_get_info(h, C.byref(ni), C.byref(nw)))
        self.n_items, self.n_workgroups = ni.value, nw.value

    def run(self, ios, torque_weight=0.0, margin=0.0, hinge_weight=0.0, lr=0.0):
        """ios: one dict per robot with keys q, qd, qdd and optional w, tau,
        cost, max_pen, argmax, n_coll, g_q, g_qd, g_qdd, f_ext, g_fext
        (device tensors)."""
        arr = self._io_array(ios)
        check(lib().wb_plan_run(self.handle, arr, float(torque_weight), float(margin), float(hinge_weight),
                                float(lr), _stream()))

    def capture(self, ios, torque_weight=0.0, margin=0.0, hinge_weight=0.0, lr=0.0, iters=1) -> "PlanGraph":
        """`iters` runs with these buffers captured into an executable HIP
        graph by the library (wb_plan_capture); the tensors must outlive it."""
        arr = self._io_array(ios)
        g = C.c_void_p()
        check(lib().wb_plan_capture(self.handle, arr, float(torque_weight), float(margin), float(hinge_weight),
                                    float(lr), int(iters), C.byref(g)))
        return PlanGraph(g, ios)

    def _io_array(self, ios):
        n = len(self.robots)
        arr = (_abi.WbTreeIO * n)()
        for i, (r, b, io) in enumerate(zip(self.robots, self.B, ios)):
            nd = r.n_dof
            ld = io["q"].shape[-1] if io.get("q") is not None else b   # padded rows: the arrays' last dimension
            if ld < b:
                raise ValueError(f"tree {i}: arrays of {ld} columns for {b} states")
            for key in ("q", "qd", "qdd", "w", "tau", "g_q", "g_qd", "g_qdd"):
                _chk(io.get(key), key, (nd, ld), device=r.device)
            for key in ("f_ext", "g_fext"):
                _chk(io.get(key), key, (r.n_links, 6, ld), device=r.device)
            for key in ("cost", "max_pen"):
                _chk(io.get(key), key, (b,), device=r.device)
            for key in ("argmax", "n_coll"):
                _chk(io.get(key), key, (b,), torch.int32, device=r.device)
            for key in _abi.TREE_IO_POINTERS:
                t = io.get(key)
                setattr(arr[i], key, None if t is None else t.data_ptr())
            arr[i].ld = ld
        return arr

    def close(self):
        if getattr(self, "handle", None) is not None:
            check(lib().wb_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PlanGraph:
    """An executable graph made by wb_plan_capture; launch() enqueues it on
    the current stream (wb_graph_launch)."""

    def __init__(self, handle, ios):
        self.handle, self._ios = handle, ios   # the graph holds the buffers' addresses

    def launch(self) -> None:
        check(lib().wb_graph_launch(self.handle, _stream()))

    def close(self):
        if getattr(self, "handle", None) is not None:
            check(lib().wb_graph_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- autograd

class ForwardKinematics(torch.autograd.Function):
    """q [n,B] -> sphere centres [S,3,B]; backward runs wb_fk_backward."""

    @staticmethod
    def forward(ctx, q, robot: Robot):
        q = q.contiguous()
        pose, sph = wb_fk(robot, q)
        ctx.robot = robot
        ctx.save_for_backward(q, pose)
        return sph

    @staticmethod
    def backward(ctx, g_sph):
        q, pose = ctx.saved_tensors
        g_q = wb_fk_backward(ctx.robot, q, g_spheres=g_sph.contiguous(), link_pose=pose)
        return g_q, None


class SelfCollision(torch.autograd.Function):
    """spheres [S,3,B] -> max penetration [B] (argmax and counts as extra,
    non-differentiable outputs); the gradient flows through the argmax pair."""

    @staticmethod
    def forward(ctx, sph, robot: Robot):
        sph = sph.contiguous()
        mp, am, nc = wb_self_collision(robot, sph)
        ctx.robot = robot
        ctx.save_for_backward(sph, am, mp)
        ctx.mark_non_differentiable(am, nc)
        return mp, am, nc

    @staticmethod
    def backward(ctx, g_mp, g_am, g_nc):
        sph, am, mp = ctx.saved_tensors
        # an effectively infinite margin makes the hinge transparent: d max_pen / d spheres
        g = wb_self_collision_backward(ctx.robot, sph, am, mp, 3.0e38, g_mp.contiguous())
        return g, None


class InverseDynamics(torch.autograd.Function):
    """(q, qd, qdd) [n,B] -> tau [n,B]; backward runs wb_rnea_backward."""

    @staticmethod
    def forward(ctx, q, qd, qdd, robot: Robot):
        q, qd, qdd = q.contiguous(), qd.contiguous(), qdd.contiguous()
        tau, cache = wb_rnea(robot, q, qd, qdd)
        ctx.robot = robot
        ctx.save_for_backward(q, qd, qdd, cache)
        return tau

    @staticmethod
    def backward(ctx, g_tau):
        q, qd, qdd, cache = ctx.saved_tensors
        g_q, g_qd, g_qdd = wb_rnea_backward(ctx.robot, q, qd, qdd, cache, g_tau.contiguous())
        return g_q, g_qd, g_qdd, None


def forward_kinematics(robot, q):
    return ForwardKinematics.apply(q, robot)


def self_collision(robot, spheres):
    return SelfCollision.apply(spheres, robot)


def inverse_dynamics(robot, q, qd, qdd):
    return InverseDynamics.apply(q, qd, qdd, robot)
