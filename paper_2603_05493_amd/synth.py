"""Seeded synthetic robots and joint states.

This module only draws inputs: robot descriptions (topology, joint axes,
fixed offsets, inertial parameters, collision spheres) and joint-space
states (q, qd, qdd).  It holds none of the whole-body arithmetic (no
kinematics, no dynamics, no distances, no pair selection), so it can feed
both the HIP path and the FP64 oracle without coupling them.

Every floating-point value is rounded to float32 and returned as a float64
array, so the FP32 device path and the FP64 oracle consume bit-identical
inputs.

Workload shapes follow the paper's robots as the whole-body section and the
inverse-dynamics comparison describe them (a 7-DoF arm, a 12-DoF bimanual
system, a 48-DoF humanoid with branching hands); the robots themselves are
synthetic stand-ins, since no robot models ship with the paper.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

JOINT_FIXED = 0
JOINT_REVOLUTE = 1


def _f32(x) -> np.ndarray:
    """Round to float32 and hand back float64 holding exactly those values."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclass
class Robot:
    """A kinematic tree with collision spheres.

    Links are numbered so that ``parent[k] < k``; link 0 is the fixed root
    (world-attached base) with ``parent[0] == -1``.  Link ``k >= 1`` hangs
    off its parent through a fixed transform ``(fixed_R[k], fixed_p[k])``
    (child joint frame expressed in the parent link frame) followed by a
    rotation of angle ``joint_mult[k] * q[joint_index[k]] + joint_offset[k]``
    about ``axis[k]`` (a unit vector in the child frame).  Inertia is about
    the link's centre of mass, in link axes.  Spheres are listed in
    nondecreasing link order, each with a centre in its link's frame.
    """

    name: str
    parent: np.ndarray          # int32 [L]
    joint_type: np.ndarray      # int32 [L]
    joint_index: np.ndarray     # int32 [L], -1 for fixed links
    joint_mult: np.ndarray      # [L]
    joint_offset: np.ndarray    # [L]
    axis: np.ndarray            # [L,3]
    fixed_R: np.ndarray         # [L,3,3]
    fixed_p: np.ndarray         # [L,3]
    mass: np.ndarray            # [L]
    com: np.ndarray             # [L,3]
    inertia: np.ndarray         # [L,3,3]
    sphere_link: np.ndarray     # int32 [S]
    sphere_pos: np.ndarray      # [S,3]
    sphere_r: np.ndarray        # [S]
    gravity: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, -9.81]))
    allow: Optional[np.ndarray] = None   # optional uint8 [L,L] link-pair allow matrix
    seed: int = 0

    @property
    def n_links(self) -> int:
        return int(self.parent.shape[0])

    @property
    def n_dof(self) -> int:
        ji = self.joint_index
        return int(ji.max()) + 1 if (ji >= 0).any() else 0

    @property
    def n_spheres(self) -> int:
        return int(self.sphere_link.shape[0])

    def depth(self) -> np.ndarray:
        d = np.zeros(self.n_links, dtype=np.int32)
        for k in range(1, self.n_links):
            d[k] = d[self.parent[k]] + 1
        return d


@dataclass
class States:
    """A batch of joint states, state-major ``[B, n]`` float64 (float32 values)."""

    q: np.ndarray
    qd: np.ndarray
    qdd: np.ndarray
    seed: int = 0

    @property
    def B(self) -> int:
        return int(self.q.shape[0])


# ---------------------------------------------------------------- helpers

def _unit(rng: np.random.Generator, n: int = 1) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    # QR of a Gaussian matrix with sign fix gives a Haar-distributed rotation.
    a = rng.normal(size=(3, 3))
    qm, r = np.linalg.qr(a)
    qm = qm * np.sign(np.diag(r))
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


def _spd_inertia(rng: np.random.Generator, lo=1e-3, hi=1e-2) -> np.ndarray:
    qm = _random_rotation(rng)
    d = rng.uniform(lo, hi, size=3)
    i = qm @ np.diag(d) @ qm.T
    return 0.5 * (i + i.T)


def _spheres_along(rng, seg_end: np.ndarray, count: int, r_lo: float, r_hi: float,
                   jitter: float) -> (np.ndarray, np.ndarray):
    """Sphere centres spread along the segment from the link origin to seg_end."""
    t = (np.arange(count) + 0.5) / count
    pos = t[:, None] * seg_end[None, :] + rng.uniform(-jitter, jitter, size=(count, 3))
    r = rng.uniform(r_lo, r_hi, size=count)
    return pos, r


def _finish(name: str, seed: int, parent: List[int], axis, fixed_R, fixed_p, mass, com,
            inertia, sph_link, sph_pos, sph_r, allow=None) -> Robot:
    L = len(parent)
    jt = np.array([JOINT_FIXED] + [JOINT_REVOLUTE] * (L - 1), dtype=np.int32)
    ji = np.array([-1] + list(range(L - 1)), dtype=np.int32)
    order = np.argsort(np.asarray(sph_link), kind="stable")
    return Robot(
        name=name,
        parent=np.asarray(parent, dtype=np.int32),
        joint_type=jt,
        joint_index=ji,
        joint_mult=np.ones(L),
        joint_offset=np.zeros(L),
        axis=_f32(axis),
        fixed_R=_f32(fixed_R),
        fixed_p=_f32(fixed_p),
        mass=_f32(mass),
        com=_f32(com),
        inertia=_f32(inertia),
        sphere_link=np.asarray(sph_link, dtype=np.int32)[order],
        sphere_pos=_f32(np.asarray(sph_pos)[order]),
        sphere_r=_f32(np.asarray(sph_r)[order]),
        gravity=_f32([0.0, 0.0, -9.81]),
        allow=allow,
        seed=seed,
    )


def _dfs_preorder(parent: List[int]) -> List[int]:
    L = len(parent)
    children = [[] for _ in range(L)]
    for k in range(1, L):
        children[parent[k]].append(k)
    order, stack = [], [0]
    while stack:
        k = stack.pop()
        order.append(k)
        stack.extend(reversed(children[k]))
    return order


# ---------------------------------------------------------------- robots

def serial_chain(n_dof: int = 7, spheres_per_link: int = 5, seed: int = 0,
                 random_fixed_rotation: bool = False) -> Robot:
    """Serial revolute chain (the 7-joint arm workload).

    Link offsets U[-0.2,0.2] m per axis, unit random axes, masses U[0.5,3] kg,
    inertia Q diag(U[1e-3,1e-2]) Q^T, CoM U[-0.1,0.1] m, sphere radii
    U[0.03,0.08] m, spheres spread along each link toward its child (the leaf
    extends 0.1 m along a random direction).
    """
    rng = np.random.default_rng(seed)
    L = n_dof + 1
    parent = [-1] + list(range(L - 1))
    fixed_p = np.zeros((L, 3))
    fixed_p[1:] = rng.uniform(-0.2, 0.2, size=(L - 1, 3))
    fixed_R = np.tile(np.eye(3), (L, 1, 1))
    if random_fixed_rotation:
        for k in range(1, L):
            fixed_R[k] = _random_rotation(rng)
    axis = np.zeros((L, 3))
    axis[0] = [0.0, 0.0, 1.0]
    axis[1:] = _unit(rng, L - 1)
    mass = rng.uniform(0.5, 3.0, size=L)
    com = rng.uniform(-0.1, 0.1, size=(L, 3))
    inertia = np.stack([_spd_inertia(rng) for _ in range(L)])
    sl, sp, sr = [], [], []
    for k in range(L):
        seg = fixed_p[k + 1] if k + 1 < L else 0.1 * _unit(rng)[0]
        pos, r = _spheres_along(rng, seg, spheres_per_link, 0.03, 0.08, 0.02)
        sl += [k] * spheres_per_link
        sp.append(pos)
        sr.append(r)
    return _finish(f"chain{n_dof}", seed, parent, axis, fixed_R, fixed_p, mass, com,
                   inertia, sl, np.concatenate(sp), np.concatenate(sr))


def random_tree(n_dof: int, spheres_per_link: int = 6, seed: int = 0,
                min_children: int = 1, max_children: int = 3,
                random_fixed_rotation: bool = False, dfs_order: bool = True) -> Robot:
    """Random tree: breadth-first growth, each node taking 1-3 children, then
    renumbered in depth-first pre-order (or kept in breadth-first order).
    Geometry and inertia as the chain."""
    rng = np.random.default_rng(seed)
    parent_bfs = [-1]
    frontier = [0]
    while len(parent_bfs) < n_dof + 1:
        nxt = []
        for node in frontier:
            c = int(rng.integers(min_children, max_children + 1))
            for _ in range(c):
                if len(parent_bfs) >= n_dof + 1:
                    break
                parent_bfs.append(node)
                nxt.append(len(parent_bfs) - 1)
        frontier = nxt if nxt else [len(parent_bfs) - 1]
    order = _dfs_preorder(parent_bfs) if dfs_order else list(range(len(parent_bfs)))
    new_of = {old: i for i, old in enumerate(order)}
    parent = [-1] + [new_of[parent_bfs[old]] for old in order[1:]]
    L = n_dof + 1
    fixed_p = np.zeros((L, 3))
    fixed_p[1:] = rng.uniform(-0.2, 0.2, size=(L - 1, 3))
    fixed_R = np.tile(np.eye(3), (L, 1, 1))
    if random_fixed_rotation:
        for k in range(1, L):
            fixed_R[k] = _random_rotation(rng)
    axis = np.zeros((L, 3))
    axis[0] = [0.0, 0.0, 1.0]
    axis[1:] = _unit(rng, L - 1)
    mass = rng.uniform(0.5, 3.0, size=L)
    com = rng.uniform(-0.1, 0.1, size=(L, 3))
    inertia = np.stack([_spd_inertia(rng) for _ in range(L)])
    first_child = {}
    for k in range(1, L):
        first_child.setdefault(parent[k], k)
    sl, sp, sr = [], [], []
    for k in range(L):
        seg = fixed_p[first_child[k]] if k in first_child else 0.1 * _unit(rng)[0]
        pos, r = _spheres_along(rng, seg, spheres_per_link, 0.03, 0.08, 0.02)
        sl += [k] * spheres_per_link
        sp.append(pos)
        sr.append(r)
    return _finish(f"tree{n_dof}", seed, parent, axis, fixed_R, fixed_p, mass, com,
                   inertia, sl, np.concatenate(sp), np.concatenate(sr))


def humanoid48(seed: int = 0, n_spheres: int = 240) -> Robot:
    """48-DoF humanoid tree with a fixed root (pelvis).

    Waist 3, neck 3, two legs of 6, two arms of 7, two hands of 8 (four
    two-joint fingers on each wrist).  Legs and waist attach to the root;
    neck and arms to the waist tip.  Links are in depth-first pre-order.
    Segment lengths are nominal human-like values with U[-0.01,0.01] m
    jitter; masses, CoM offsets and inertias are drawn as for the chain
    (fingers scaled down); ``n_spheres`` spheres are spread 4-5 per link.
    """
    rng = np.random.default_rng(seed)
    parent: List[int] = [-1]
    offs: List[np.ndarray] = [np.zeros(3)]
    axes: List[np.ndarray] = [np.array([0.0, 0.0, 1.0])]
    kind: List[str] = ["torso"]
    ex, ey, ez = np.eye(3)

    def chain(par: int, segs, knd: str) -> int:
        last = par
        for off, ax in segs:
            parent.append(last)
            offs.append(np.asarray(off, dtype=np.float64) + rng.uniform(-0.01, 0.01, 3))
            a = np.asarray(ax, dtype=np.float64) + rng.uniform(-0.05, 0.05, 3)
            axes.append(a / np.linalg.norm(a))
            kind.append(knd)
            last = len(parent) - 1
        return last

    for side in (+1.0, -1.0):  # legs
        chain(0, [((0, 0.09 * side, -0.05), ez), ((0, 0, -0.04), ex), ((0, 0, -0.04), ey),
                  ((0, 0, -0.36), ey), ((0, 0, -0.36), ey), ((0, 0, -0.04), ex)], "leg")
    waist = chain(0, [((0, 0, 0.10), ez), ((0, 0, 0.05), ex), ((0, 0, 0.05), ey)], "torso")
    chain(waist, [((0, 0, 0.28), ez), ((0, 0, 0.04), ey), ((0, 0, 0.04), ex)], "head")
    for side in (+1.0, -1.0):  # arm then hand
        wrist = chain(waist, [((0, 0.18 * side, 0.22), ey), ((0, 0.04 * side, 0), ex),
                              ((0, 0.04 * side, 0), ey), ((0, 0.24 * side, 0), ez),
                              ((0, 0.20 * side, 0), ey), ((0, 0.03 * side, 0), ex),
                              ((0, 0.03 * side, 0), ez)], "arm")
        for f in range(4):
            chain(wrist, [((-0.03 + 0.02 * f, 0.06 * side, 0), ex),
                          ((0, 0.04 * side, 0), ex)], "finger")
    L = len(parent)
    assert L == 49, L
    fixed_p = np.stack(offs)
    fixed_R = np.tile(np.eye(3), (L, 1, 1))
    axis = np.stack(axes)
    scale = np.array([0.02 if kd == "finger" else 1.0 for kd in kind])
    mass = rng.uniform(0.5, 3.0, size=L) * scale
    com = rng.uniform(-0.1, 0.1, size=(L, 3)) * np.sqrt(scale)[:, None]
    inertia = np.stack([_spd_inertia(rng) * s for s in scale])
    first_child = {}
    for k in range(1, L):
        first_child.setdefault(parent[k], k)
    leaf_dir = {"leg": 0.10 * ex, "head": 0.10 * ez, "finger": None, "arm": None, "torso": 0.1 * ez}
    segs = []
    for k in range(L):
        if k in first_child:
            segs.append(fixed_p[first_child[k]])
        elif kind[k] == "finger":
            segs.append(0.03 * fixed_p[k] / np.linalg.norm(fixed_p[k]))
        else:
            segs.append(leaf_dir[kind[k]])
    seg_len = np.array([np.linalg.norm(s) for s in segs])
    per_link = np.full(L, n_spheres // L)
    extra = n_spheres - per_link.sum()
    per_link[np.argsort(-seg_len, kind="stable")[:extra]] += 1
    sl, sp, sr = [], [], []
    for k in range(L):
        small = kind[k] == "finger"
        pos, r = _spheres_along(rng, segs[k], int(per_link[k]),
                                0.008 if small else 0.03, 0.015 if small else 0.08,
                                0.005 if small else 0.02)
        sl += [k] * int(per_link[k])
        sp.append(pos)
        sr.append(r)
    return _finish("humanoid48", seed, parent, axis, fixed_R, fixed_p, mass, com, inertia,
                   sl, np.concatenate(sp), np.concatenate(sr))


# The 48-DoF humanoid at the paper's self-collision scale: 588 spheres (12
# on the 31 longest links, 11 on the others) give 162,432 checked pairs, the
# paper's 162k pairs of its 48-DoF humanoid.
PAPER_SCALE_SPHERES = 588


def humanoid48_paper_scale(seed: int = 0) -> Robot:
    """humanoid48 with PAPER_SCALE_SPHERES spheres (162,432 checked pairs)."""
    return humanoid48(seed=seed, n_spheres=PAPER_SCALE_SPHERES)


def humanoid48_tool_links() -> dict:
    """Links of humanoid48 that carry its natural tool frames, by the
    generator's depth-first numbering: the last link of each leg (feet), of
    each arm (wrists) and of the neck (head)."""
    return {"left_foot": 6, "right_foot": 12, "head": 18, "left_wrist": 25, "right_wrist": 40}


def with_fixed_links(rb: Robot, links) -> Robot:
    """Turn the given links' joints into fixed joints (actuated indices renumbered)."""
    fixed = set(int(k) for k in links)
    jt = rb.joint_type.copy()
    ji = np.full_like(rb.joint_index, -1)
    nxt = 0
    for k in range(rb.n_links):
        if k in fixed or k == 0:
            jt[k] = JOINT_FIXED
        else:
            ji[k] = nxt
            nxt += 1
    rb.joint_type, rb.joint_index = jt, ji
    return rb


def planar_2r(l1: float = 0.5, l2: float = 0.4, m1: float = 1.0, m2: float = 0.7,
              izz1: float = 0.01, izz2: float = 0.02) -> Robot:
    """Textbook planar two-link arm: joints about z, links along x, CoM at mid-link,
    gravity along -y.  One sphere at each link's tip (for distance checks)."""
    L = 3
    parent = [-1, 0, 1]
    fixed_p = np.array([[0, 0, 0], [0, 0, 0], [l1, 0, 0]], dtype=np.float64)
    axis = np.array([[0, 0, 1], [0, 0, 1], [0, 0, 1]], dtype=np.float64)
    mass = np.array([0.0, m1, m2])
    com = np.array([[0, 0, 0], [l1 / 2, 0, 0], [l2 / 2, 0, 0]], dtype=np.float64)
    inertia = np.zeros((3, 3, 3))
    inertia[1] = np.diag([1e-4, 1e-4, izz1])
    inertia[2] = np.diag([1e-4, 1e-4, izz2])
    rb = _finish("planar2r", 0, parent, axis, np.tile(np.eye(3), (L, 1, 1)), fixed_p, mass, com,
                 inertia, [1, 2], np.array([[l1, 0, 0], [l2, 0, 0]]), np.array([0.01, 0.01]))
    rb.gravity = _f32([0.0, -9.81, 0.0])
    return rb


# ---------------------------------------------------------------- states

def states(robot: Robot, B: int, seed: int = 1, q_range: float = np.pi,
           qd_std: float = 1.0, qdd_std: float = 1.0) -> States:
    """q ~ U[-q_range, q_range], qd ~ N(0, qd_std^2), qdd ~ N(0, qdd_std^2)."""
    rng = np.random.default_rng(seed)
    n = robot.n_dof
    q = rng.uniform(-q_range, q_range, size=(B, n))
    qd = rng.normal(0.0, qd_std, size=(B, n))
    qdd = rng.normal(0.0, qdd_std, size=(B, n))
    return States(q=_f32(q), qd=_f32(qd), qdd=_f32(qdd), seed=seed)


def weights(shape, seed: int = 2) -> np.ndarray:
    """Random N(0,1) upstream weights (float32 values)."""
    return _f32(np.random.default_rng(seed).normal(size=shape))


# ---------------------------------------------------------------- workloads

WORKLOADS = {
    # name: (robot factory, B, q_range)
    "chain7_fwd_B32": (lambda: serial_chain(7, 5, seed=0), 32, np.pi),
    "chain7_fwdbwd_B4096": (lambda: serial_chain(7, 5, seed=0), 4096, np.pi),
    "humanoid48_fwdbwd_B2048": (lambda: humanoid48(seed=0), 2048, 1.5),
    "humanoid48_optimizer_B24576": (lambda: humanoid48(seed=0), 24576, 1.5),
}

UNEVEN_TREES = [(7, 8192), (12, 4096), (23, 2048), (48, 1024)]


def uneven_trees(seed: int = 0):
    """The uneven multi-tree batch: random trees of 7/12/23/48 DoF with
    8192/4096/2048/1024 states, six spheres per link."""
    return [(random_tree(n, 6, seed=seed + i), b) for i, (n, b) in enumerate(UNEVEN_TREES)]
