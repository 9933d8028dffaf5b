"""ctypes loader of libnbody.so (built in-tree by paper_2411_18889_amd/build.py).

There is no fallback: if the library is not built, every call raises.
"""

from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbody.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "nbody.h")

NB_OK, NB_EINVAL, NB_EWORKSPACE, NB_EUNSUPPORTED, NB_ENODEV, NB_EDEVICE = range(6)
NB_OP_ACCEL, NB_OP_STEP, NB_OP_ADJOINT, NB_OP_DIAG = range(4)
NB_ACC_VALID = 0x1
NB_GRAPH = 0x2
NB_ADJ_ENTRY_HALF = 0x1
NB_ADJ_EXIT_FULL = 0x2

PREC = {"f64": 0, "f32": 1, "mix_acc32": 2, "mix_kahan": 3, "mix_acc64": 4, "mix_tilec": 5}


class nb_launch(ctypes.Structure):
    _fields_ = [("i_per_lane", ctypes.c_int32), ("block", ctypes.c_int32),
                ("split", ctypes.c_int32), ("symmetric", ctypes.c_int32)]


class nb_pass_info(ctypes.Structure):
    _fields_ = [("symmetric", ctypes.c_int32), ("block", ctypes.c_int32),
                ("i_per_lane", ctypes.c_int32), ("split", ctypes.c_int32),
                ("block_particles", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t)]


class NBodyError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__("%s: %s (status %d%s)" % (
            what, strerror(status), status,
            ", hip error %d" % last_hip_error() if status == NB_EDEVICE else ""))


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libnbody.so is not built (%s); run `python -m paper_2411_18889_amd.build` "
            "or __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    i64, vp, dbl, i32, sz, u32 = (ctypes.c_int64, ctypes.c_void_p, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_size_t, ctypes.c_uint)
    L.nbody_accel.argtypes = [i64, vp, i64, vp, vp, dbl, dbl, i32, vp, vp, vp, sz, vp]
    L.nbody_accel_noalloc.argtypes = [i64, vp, i64, vp, vp, dbl, dbl, i32, vp, vp, vp]
    L.nbody_accel_ex.argtypes = [i64, vp, i64, vp, vp, dbl, dbl, i32, vp, vp,
                                 ctypes.POINTER(nb_launch), vp, sz, vp]
    L.nbody_step.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, dbl, i64, i32, u32, vp, i64,
                             vp, sz, vp]
    L.nbody_step_adjoint.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, dbl, dbl, dbl, i64,
                                     i32, u32, vp, i64, i64, vp, sz, vp]
    L.nbody_step_adjoint_ex.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, dbl, dbl, dbl, i64,
                                        i32, u32, vp, i64, i64, ctypes.POINTER(nb_launch), vp,
                                        sz, vp]
    L.nbody_diag.argtypes = [i64, vp, vp, vp, dbl, dbl, i32, vp, vp, sz, vp]
    L.nbody_workspace_size.argtypes = [i32, i64, i32]
    L.nbody_workspace_size.restype = sz
    L.nbody_pass_workspace_size.argtypes = [i32, i64, i64, i32, i32, i32, ctypes.POINTER(nb_launch)]
    L.nbody_pass_workspace_size.restype = sz
    L.nbody_strerror.argtypes = [i32]
    L.nbody_strerror.restype = ctypes.c_char_p
    L.nbody_last_hip_error.argtypes = []
    L.nbody_device_info.argtypes = [ctypes.c_char_p, sz]
    L.diffusion3d_step.argtypes = [i64, i64, i64, dbl, dbl, dbl, dbl, dbl, vp, vp, vp]
    L.diffusion3d_step.restype = ctypes.c_int
    L.nbody_profile_begin.argtypes = []
    L.nbody_profile_end.argtypes = [ctypes.POINTER(nb_profile_t)]
    L.nbody_graph_cache_clear.argtypes = []
    L.nbody_pass_info.argtypes = [i32, i64, i32, ctypes.POINTER(nb_pass_info)]
    for f in ("nbody_accel", "nbody_accel_noalloc", "nbody_accel_ex", "nbody_step", "nbody_step_adjoint",
              "nbody_step_adjoint_ex",
              "nbody_diag", "nbody_last_hip_error", "nbody_device_info",
              "nbody_profile_begin", "nbody_profile_end", "nbody_graph_cache_clear",
              "nbody_pass_info"):
        getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().nbody_strerror(int(status)).decode()


def last_hip_error() -> int:
    return int(lib().nbody_last_hip_error())


def check(status: int, what: str) -> None:
    if status != NB_OK:
        raise NBodyError(status, what)


def declared_functions() -> list:
    """Names of the functions the headers under include/ declare."""
    names = set()
    inc = os.path.dirname(HEADER)
    for h in sorted(os.listdir(inc)):
        if h.endswith(".h"):
            text = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, h)).read(), flags=re.S)
            names.update(re.findall(r"\b((?:nbody|diffusion3d)_\w+)\s*\(", text))
    return sorted(names)


class nb_profile_t(ctypes.Structure):
    """Mirror of nb_profile: summed device ms and call counts per kind
    (force, adjoint, update, diag, copy)."""
    _fields_ = [("ms", ctypes.c_double * 5), ("calls", ctypes.c_int64 * 5)]
