"""ctypes front end of the FP64 CPU oracle (``wb_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the HIP library or its binding.  The
oracle shares no code with the HIP path; both only consume the same seeded
inputs (plain numpy arrays describing a robot and its states).

All arrays here are state-major: q [B, n], sphere centres [B, S, 3], link
rotations [B, L, 3, 3], link positions [B, L, 3].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _OrcRobot(C.Structure):
    _fields_ = [
        ("L", C.c_int), ("n", C.c_int), ("S", C.c_int),
        ("parent", _ip), ("jtype", _ip), ("jidx", _ip),
        ("jmult", _dp), ("joff", _dp), ("axis", _dp), ("fR", _dp), ("fp", _dp),
        ("mass", _dp), ("com", _dp), ("inertia", _dp),
        ("sph_link", _ip), ("sph_pos", _dp), ("sph_r", _dp), ("gravity", _dp),
        ("allow", C.POINTER(C.c_ubyte)),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over states)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _lib.orc_pairs.restype = C.c_int
        _lib.orc_num_threads.restype = C.c_int
    return _lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _pd(a: Optional[np.ndarray]):
    return a.ctypes.data_as(_dp) if a is not None else None


def _pi(a: Optional[np.ndarray]):
    return a.ctypes.data_as(_ip) if a is not None else None


class OracleRobot:
    """Holds FP64 copies of a robot description and the C struct pointing at them."""

    def __init__(self, rb):
        self.L = int(rb.parent.shape[0])
        self.n = int(rb.joint_index.max()) + 1 if (rb.joint_index >= 0).any() else 0
        self.S = int(rb.sphere_link.shape[0])
        self._keep = dict(
            parent=_i(rb.parent), jtype=_i(rb.joint_type), jidx=_i(rb.joint_index),
            jmult=_d(rb.joint_mult), joff=_d(rb.joint_offset), axis=_d(rb.axis),
            fR=_d(rb.fixed_R).reshape(-1), fp=_d(rb.fixed_p), mass=_d(rb.mass), com=_d(rb.com),
            inertia=_d(rb.inertia).reshape(-1), sph_link=_i(rb.sphere_link),
            sph_pos=_d(rb.sphere_pos), sph_r=_d(rb.sphere_r), gravity=_d(rb.gravity),
        )
        allow = getattr(rb, "allow", None)
        self._allow = None if allow is None else np.ascontiguousarray(allow, dtype=np.uint8)
        k = self._keep
        self.c = _OrcRobot(
            self.L, self.n, self.S, _pi(k["parent"]), _pi(k["jtype"]), _pi(k["jidx"]),
            _pd(k["jmult"]), _pd(k["joff"]), _pd(k["axis"]), _pd(k["fR"]), _pd(k["fp"]),
            _pd(k["mass"]), _pd(k["com"]), _pd(k["inertia"]), _pi(k["sph_link"]),
            _pd(k["sph_pos"]), _pd(k["sph_r"]), _pd(k["gravity"]),
            self._allow.ctypes.data_as(C.POINTER(C.c_ubyte)) if self._allow is not None else None,
        )

    @property
    def ref(self):
        return C.byref(self.c)


def _robot(rb) -> OracleRobot:
    return rb if isinstance(rb, OracleRobot) else OracleRobot(rb)


def fk(rb, q) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """World rotations [B,L,3,3], positions [B,L,3], sphere centres [B,S,3]."""
    o = _robot(rb)
    q = _d(q)
    B = q.shape[0]
    R = np.empty((B, o.L, 3, 3))
    p = np.empty((B, o.L, 3))
    c = np.empty((B, o.S, 3))
    lib().orc_fk(o.ref, B, _pd(q), _pd(R), _pd(p), _pd(c))
    return R, p, c


def fk_backward(rb, q, g_spheres=None, g_R=None, g_p=None) -> np.ndarray:
    o = _robot(rb)
    q = _d(q)
    B = q.shape[0]
    gq = np.empty((B, o.n))
    gc = None if g_spheres is None else _d(g_spheres)
    gR = None if g_R is None else _d(g_R)
    gp = None if g_p is None else _d(g_p)
    lib().orc_fk_backward(o.ref, B, _pd(q), _pd(gR), _pd(gp), _pd(gc), _pd(gq))
    return gq


def rnea(rb, q, qd, qdd, fext=None) -> np.ndarray:
    o = _robot(rb)
    q, qd, qdd = _d(q), _d(qd), _d(qdd)
    B = q.shape[0]
    tau = np.empty((B, o.n))
    fe = None if fext is None else _d(fext)
    lib().orc_rnea(o.ref, B, _pd(q), _pd(qd), _pd(qdd), _pd(fe), _pd(tau))
    return tau


def rnea_vjp(rb, q, qd, qdd, g_tau, fext=None, want_fext=False):
    o = _robot(rb)
    q, qd, qdd, gt = _d(q), _d(qd), _d(qdd), _d(g_tau)
    B = q.shape[0]
    gq, gqd, gqdd = np.empty((B, o.n)), np.empty((B, o.n)), np.empty((B, o.n))
    gfe = np.empty((B, o.L, 6)) if want_fext else None
    fe = None if fext is None else _d(fext)
    lib().orc_rnea_vjp(o.ref, B, _pd(q), _pd(qd), _pd(qdd), _pd(fe), _pd(gt), _pd(gq), _pd(gqd),
                       _pd(gqdd), _pd(gfe))
    return (gq, gqd, gqdd, gfe) if want_fext else (gq, gqd, gqdd)


def pairs(rb) -> Tuple[np.ndarray, np.ndarray]:
    o = _robot(rb)
    P = lib().orc_pairs(o.ref, None, None)
    s = np.empty(max(P, 1), dtype=np.int32)
    t = np.empty(max(P, 1), dtype=np.int32)
    lib().orc_pairs(o.ref, _pi(s), _pi(t))
    return s[:P], t[:P]


def self_collision(rb, c):
    """(max_pen [B], argmax [B] int32, n_coll [B] int32) over all allowed pairs."""
    o = _robot(rb)
    c = _d(c)
    B = c.shape[0]
    mp = np.empty(B)
    am = np.empty(B, dtype=np.int32)
    nc = np.empty(B, dtype=np.int32)
    lib().orc_self_collision(o.ref, B, _pd(c), _pd(mp), _pi(am), _pi(nc))
    return mp, am, nc


def self_collision_pens(rb, c) -> np.ndarray:
    """Penetration of every allowed pair, [B, P]."""
    o = _robot(rb)
    c = _d(c)
    B = c.shape[0]
    P = lib().orc_pairs(o.ref, None, None)
    pen = np.empty((B, P))
    lib().orc_self_collision_pens(o.ref, B, _pd(c), _pd(pen))
    return pen


def self_collision_backward(rb, c, argmax, max_pen, margin, g_cost) -> np.ndarray:
    o = _robot(rb)
    c = _d(c)
    B = c.shape[0]
    gc = np.empty((B, o.S, 3))
    lib().orc_self_collision_backward(o.ref, B, _pd(c), _pi(_i(argmax)), _pd(_d(max_pen)),
                                      C.c_double(margin), _pd(_d(g_cost)), _pd(gc))
    return gc


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's loops over states (used for timing only)."""
    lib().orc_set_num_threads(C.c_int(int(n)))


# ------------------------------------------------------------- cost heads
# Upstream adjoints of the scalar costs the optimizer-shaped workload uses:
# L = sum(w * tau) -> tau-bar = w;  L = c ||tau||^2 -> tau-bar = 2 c tau;
# hinge h = max(0, max_pen + margin) -> h-bar = 1[h > 0].

def hinge(max_pen, margin):
    return np.maximum(0.0, np.asarray(max_pen) + margin)
