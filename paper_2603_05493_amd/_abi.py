"""ctypes view of the C ABI in include/wb.h (argument marshalling only).

The shared library must have been built (``python -m paper_2603_05493_amd.build``
or ``__graft_entry__.build()``); importing this module without it raises, so
no caller can silently fall back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwb.so")

WB_OK, WB_ERR_INVALID_ARG, WB_ERR_INVALID_TREE, WB_ERR_UNSUPPORTED, WB_ERR_HIP = range(5)
WB_JOINT_FIXED, WB_JOINT_REVOLUTE = 0, 1

_i32p = C.POINTER(C.c_int32)
_f32p = C.POINTER(C.c_float)
_u8p = C.POINTER(C.c_uint8)
_vp = C.c_void_p


class WbRobotDesc(C.Structure):
    _fields_ = [
        ("n_links", C.c_int32), ("parent", _i32p), ("joint_type", _i32p), ("joint_index", _i32p),
        ("joint_mult", _f32p), ("joint_offset", _f32p), ("axis", _f32p), ("fixed_R", _f32p),
        ("fixed_p", _f32p), ("mass", _f32p), ("com", _f32p), ("inertia", _f32p),
        ("n_spheres", C.c_int32), ("sphere_link", _i32p), ("sphere", _f32p), ("allow", _u8p),
        ("gravity", C.c_float * 3),
    ]


class WbRobotInfo(C.Structure):
    _fields_ = [
        ("n_links", C.c_int32), ("n_dof", C.c_int32), ("n_spheres", C.c_int32),
        ("max_depth", C.c_int32), ("n_pairs", C.c_int64), ("n_blocks", C.c_int32),
        ("max_spheres_per_link", C.c_int32), ("fused_supported", C.c_int32),
        ("kinematics_supported", C.c_int32), ("mimic", C.c_int32),
    ]


class WbTune(C.Structure):
    _fields_ = [("lanes_per_state", C.c_int32), ("states_per_item", C.c_int32), ("ns_per_state", C.c_float)]


TREE_IO_POINTERS = ("q", "qd", "qdd", "w", "tau", "cost", "max_pen", "argmax", "n_coll", "g_q", "g_qd", "g_qdd",
                    "f_ext", "g_fext")


class WbTreeIO(C.Structure):
    _fields_ = [(nm, _vp) for nm in TREE_IO_POINTERS] + [("ld", C.c_int64)]


class WbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"wb error {code}: {msg}")
        self.code = code


# name -> (argtypes)
_SIGS = {
    "wb_desc_analyze": [C.POINTER(WbRobotDesc), C.POINTER(WbRobotInfo)],
    "wb_desc_pairs": [C.POINTER(WbRobotDesc), _i32p, _i32p],
    "wb_robot_create": [C.POINTER(WbRobotDesc), C.POINTER(_vp)],
    "wb_robot_destroy": [_vp],
    "wb_robot_get_info": [_vp, C.POINTER(WbRobotInfo)],
    "wb_workspace_bytes": [_vp, C.c_int64, C.POINTER(C.c_size_t)],
    "wb_rnea_cache_bytes": [_vp, C.c_int64, C.POINTER(C.c_size_t)],
    "wb_fk": [_vp, C.c_int64, C.c_int64, _vp, _vp, _vp, _vp],
    "wb_rnea": [_vp, C.c_int64, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "wb_self_collision": [_vp, C.c_int64, C.c_int64, _vp, _vp, _vp, _vp, _vp],
    "wb_self_collision_backward": [_vp, C.c_int64, C.c_int64, _vp, _vp, _vp, C.c_float, _vp, _vp, _vp],
    "wb_fk_backward": [_vp, C.c_int64, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "wb_rnea_backward": [_vp, C.c_int64, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "wb_cost_head": [C.c_int64, C.c_int64, C.c_int32, _vp, _vp, C.c_float, _vp, C.c_float, C.c_float, _vp, _vp,
                     _vp, _vp],
    "wb_sgd_step": [C.c_int64, C.c_int64, C.c_int32, C.c_float, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "wb_robot_set_link_inertia": [_vp, C.c_int32, C.c_float, _vp, _vp],
    "wb_robot_set_tool_frames": [_vp, C.c_int32, _vp, _vp],
    "wb_robot_get_tool_count": [_vp, _i32p],
    "wb_kinematics": [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "wb_kinematics_backward": [_vp, C.c_int64, _vp, _vp, _vp, _vp, _vp],
    "wb_edt_workspace_bytes": [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)],
    "wb_edt": [C.c_int32, C.c_int32, C.c_int32, _vp, C.c_float, _vp, _vp, _vp, _vp],
    "wb_edt_noalloc": [C.c_int32, C.c_int32, C.c_int32, _vp, C.c_float, _vp, _vp, _vp],
    "wb_bspline_eval": [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_int32, _vp, _vp, _vp, _vp,
                        _vp, _vp, _vp, _vp],
    "wb_bspline_backward": [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_float, _vp, _vp, _vp, _vp, C.c_float,
                            C.c_int32, _vp, _vp],
    "wb_wholebody_step": [_vp, C.c_int64, C.c_int64, _vp, _vp, _vp, _vp, C.c_float, C.c_float, C.c_float, C.c_float,
                          _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "wb_wholebody_step_bspline": [_vp, C.c_int64, C.c_int32, C.c_float, C.c_int32, _vp, _vp, _vp, _vp, _vp,
                                  C.c_float, C.c_float, C.c_float, _vp, C.c_float, C.c_int32, _vp, _vp, _vp, _vp,
                                  _vp, _vp, _vp, _vp, _vp],
    "wb_robot_set_tune": [_vp, C.POINTER(WbTune)],
    "wb_robot_set_dispatch": [_vp, C.c_int64, C.c_int64, C.c_int64],
    "wb_robot_get_tune": [_vp, C.POINTER(WbTune)],
    "wb_plan_create": [C.POINTER(_vp), C.POINTER(C.c_int64), C.c_int32, C.POINTER(WbTune), C.POINTER(_vp)],
    "wb_plan_run": [_vp, C.POINTER(WbTreeIO), C.c_float, C.c_float, C.c_float, C.c_float, _vp],
    "wb_plan_capture": [_vp, C.POINTER(WbTreeIO), C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32,
                        C.POINTER(_vp)],
    "wb_graph_launch": [_vp, _vp],
    "wb_graph_destroy": [_vp],
    "wb_plan_get_info": [_vp, _i32p, _i32p],
    "wb_plan_destroy": [_vp],
}

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2603_05493_amd.build`")
        _lib = C.CDLL(LIB_PATH)
        _lib.wb_last_error.restype = C.c_char_p
        _lib.wb_last_error.argtypes = []
        for name, args in _SIGS.items():
            fn = getattr(_lib, name)
            fn.argtypes = args
            fn.restype = C.c_int
    return _lib


def declared_symbols():
    """The entry points this binding expects the library to export."""
    return ["wb_last_error", *_SIGS.keys()]


def check(rc: int) -> None:
    if rc != WB_OK:
        raise WbError(rc, lib().wb_last_error().decode(errors="replace"))
