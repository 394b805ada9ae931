"""FP64 oracle of the kinematics outputs that complete a forward-kinematics
call besides link poses and sphere centres (cuRoboV2 Sec. 6.1, "adaptive
kernel dispatch", and Alg. 2): tool poses, the centre of mass, the
tool-frame Jacobian with its topology caches, the Jacobian of the centre of
mass, and the gradient of losses on tool poses and the centre of mass.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the HIP
library or its binding; it shares no code with the HIP path.  Link poses
come from the oracle's own forward kinematics (``oracle.fk``).

Definitions (frames as in the robot description: link k's origin is its
joint's origin, and its joint turns about axis_k in link k's frame):
  * tool frame t = (link e_t, fixed offset (R_off, p_off) in that link's
    frame); its world pose is R = R_e R_off, x = p_e + R_e p_off;
  * centre of mass: the mass-weighted mean of every link's CoM in world
    coordinates, fixed base included, sum_k m_k (R_k c_k + p_k) / sum_k m_k;
  * Jacobian of tool t (Alg. 2): column j sums, over the links l that joint j
    drives (connectedLinks[j]; more than one for mimic joints) and that lie
    on the chain from the root to e_t (linkChain[e_t]; the joint's own link
    e_t included), mult_l [s_l x (x - o_l); s_l], with s_l = R_l axis_l the
    world axis and o_l = p_l the world origin of that joint.  Rows are the
    linear velocity of the tool point then the angular velocity;
    affects[j, e] (the coarse filter) is true when any of those links is on
    the chain;
  * CoM Jacobian: column j = sum over l in connectedLinks[j] of
    mult_l s_l x (C_l - M_l o_l) / M, with M_l and C_l the mass and first
    moment (sum m_k c_k^world) of l's subtree and M the total mass;
  * gradient of L = sum_t <G_t, R_t> + g_t . x_t + g_com . com: for a joint
    turning by dtheta about (s, o) a rotation changes by [s]x R dtheta, so
    dL/dq = sum_t J_t^T [g_t; w_t] + J_com^T g_com with
    w_t = sum_c r_c x G_c over the columns r_c of R_t and G_c of G_t.

Arrays are state-major: q [B, n]; tool_R [T, 3, 3], tool_p [T, 3]; outputs
[B, T, 3, 3], [B, T, 3], [B, 3], [B, T, 6, n], [B, 3, n].
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

REVOLUTE = 1


def _n_dof(rb) -> int:
    j = np.asarray(rb.joint_index)
    return int(j.max()) + 1 if (j >= 0).any() else 0


def link_chain(rb, e: int) -> list:
    """Links from e up to the root (e included): linkChain[e]."""
    out = []
    k = int(e)
    while k >= 0:
        out.append(k)
        k = int(rb.parent[k])
    return out


def connected_links(rb) -> list:
    """connectedLinks[j]: the revolute links whose angle joint j sets."""
    n = _n_dof(rb)
    conn = [[] for _ in range(n)]
    for k in range(1, len(rb.parent)):
        if int(rb.joint_type[k]) == REVOLUTE and int(rb.joint_index[k]) >= 0:
            conn[int(rb.joint_index[k])].append(k)
    return conn


def affects(rb, tool_link) -> np.ndarray:
    """affects[j, t]: joint j moves tool t's link (bool [n, T])."""
    conn = connected_links(rb)
    out = np.zeros((len(conn), len(tool_link)), dtype=bool)
    for t, e in enumerate(tool_link):
        chain = set(link_chain(rb, e))
        for j, links in enumerate(conn):
            out[j, t] = any(l in chain for l in links)
    return out


def _poses(rb, q):
    R, p, _ = O.fk(rb, q)
    return R, p


def tool_poses(rb, q, tool_link, tool_R, tool_p):
    R, p = _poses(rb, q)
    tool_R = np.asarray(tool_R, float)
    tool_p = np.asarray(tool_p, float)
    Re = R[:, list(tool_link)]                                        # [B, T, 3, 3]
    Rt = Re @ tool_R[None]
    xt = p[:, list(tool_link)] + np.einsum("btij,tj->bti", Re, tool_p)
    return Rt, xt


def _total_mass(rb) -> float:
    M = float(np.sum(np.asarray(rb.mass, float)))
    if not M > 0.0:
        raise ValueError("the robot has no mass")
    return M


def _link_coms(rb, R, p):
    """World CoM of every link: [B, L, 3]."""
    return np.einsum("blij,lj->bli", R, np.asarray(rb.com, float)) + p


def center_of_mass(rb, q):
    R, p = _poses(rb, q)
    m = np.asarray(rb.mass, float)
    return np.einsum("l,bli->bi", m, _link_coms(rb, R, p)) / _total_mass(rb)


def jacobian(rb, q, tool_link, tool_R, tool_p):
    """Alg. 2: one column per joint, coarse filter affects[j, e], fine filter
    linkChain[e], contributions summed over connectedLinks[j]."""
    R, p = _poses(rb, q)
    _, xt = tool_poses(rb, q, tool_link, tool_R, tool_p)
    B = R.shape[0]
    conn = connected_links(rb)
    aff = affects(rb, tool_link)
    axis = np.asarray(rb.axis, float)
    mult = np.asarray(rb.joint_mult, float)
    J = np.zeros((B, len(tool_link), 6, len(conn)))
    for t, e in enumerate(tool_link):
        chain = set(link_chain(rb, e))
        for j, links in enumerate(conn):
            if not aff[j, t]:
                continue
            for l in links:
                if l not in chain:
                    continue
                s = R[:, l] @ axis[l]                                 # [B, 3]
                J[:, t, :3, j] += mult[l] * np.cross(s, xt[:, t] - p[:, l])
                J[:, t, 3:, j] += mult[l] * s
    return J


def _subtree(rb, l: int) -> list:
    return [k for k in range(len(rb.parent)) if l in link_chain(rb, k)]


def com_jacobian(rb, q):
    R, p = _poses(rb, q)
    m = np.asarray(rb.mass, float)
    M = _total_mass(rb)
    cw = _link_coms(rb, R, p)
    axis = np.asarray(rb.axis, float)
    mult = np.asarray(rb.joint_mult, float)
    conn = connected_links(rb)
    Jc = np.zeros((R.shape[0], 3, len(conn)))
    for j, links in enumerate(conn):
        for l in links:
            sub = _subtree(rb, l)
            Ml = float(np.sum(m[sub]))
            Cl = np.einsum("k,bki->bi", m[sub], cw[:, sub])
            s = R[:, l] @ axis[l]
            Jc[:, :, j] += mult[l] * np.cross(s, Cl - Ml * p[:, l]) / M
    return Jc


def backward(rb, q, tool_link, tool_R, tool_p, g_R=None, g_p=None, g_com=None):
    """dL/dq [B, n] for L = sum_t <g_R[t], R_t> + g_p[t] . x_t + g_com . com."""
    q = np.asarray(q, float)
    B = q.shape[0]
    gq = np.zeros((B, _n_dof(rb)))
    if len(tool_link) and (g_R is not None or g_p is not None):
        Rt, _ = tool_poses(rb, q, tool_link, tool_R, tool_p)
        J = jacobian(rb, q, tool_link, tool_R, tool_p)
        T = len(tool_link)
        gp = np.zeros((B, T, 3)) if g_p is None else np.asarray(g_p, float)
        gR = np.zeros((B, T, 3, 3)) if g_R is None else np.asarray(g_R, float)
        w = np.cross(np.swapaxes(Rt, -1, -2), np.swapaxes(gR, -1, -2)).sum(-2)   # sum over columns
        gq += np.einsum("btrj,btr->bj", J, np.concatenate([gp, w], -1))
    if g_com is not None:
        gq += np.einsum("bij,bi->bj", com_jacobian(rb, q), np.asarray(g_com, float))
    return gq
