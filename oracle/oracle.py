"""ctypes front end of the FP64 CPU oracle (oracle/nbody_oracle.c).

TEST INFRASTRUCTURE ONLY. Arrays are float64 numpy arrays in
structure-of-arrays layout: positions/velocities/adjoints (3, n), masses (n,).
Inputs of another dtype are promoted to float64 exactly (FP32 -> FP64 is
exact), so a GPU run in FP32 can be compared against the oracle on the very
values it saw. The library is built on first use if it is not there yet.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

DIAG_FIELDS = ("KE", "PE", "E", "Px", "Py", "Pz", "Lx", "Ly", "Lz",
               "COMx", "COMy", "COMz", "M")

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("NBODY_ORACLE_LIB")  # a mutant build, for the pin tests
    if not path:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
    lib = ctypes.CDLL(path)
    i64, dbl = ctypes.c_int64, ctypes.c_double
    lib.oracle_accel.argtypes = [i64, _D, _I64, i64, _D, _D, dbl, dbl, _D, _D]
    lib.oracle_kdk.argtypes = [i64, _D, _D, _D, dbl, dbl, dbl, i64, _D, _D, _D]
    lib.oracle_diag.argtypes = [i64, _D, _D, _D, dbl, dbl, _D]
    lib.oracle_vjp.argtypes = [i64, _D, _D, _D, dbl, dbl, _D, _D]
    lib.oracle_vjp_sampled.argtypes = [i64, i64, _I64, _D, _D, _D, dbl, dbl, _D, _D]
    lib.oracle_jvp.argtypes = [i64, _D, _D, _D, dbl, dbl, _D]
    lib.oracle_adjoint.argtypes = [i64, i64, _D, _D, dbl, dbl, dbl, _D, _D, _D]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    for f in ("oracle_accel", "oracle_kdk", "oracle_diag", "oracle_vjp", "oracle_vjp_sampled",
              "oracle_jvp", "oracle_adjoint"):
        getattr(lib, f).restype = None
    _lib = lib
    return lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def _p(a):
    return None if a is None else a.ctypes.data_as(_D)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(k: int) -> None:
    """Threads used by later calls (the results do not depend on it)."""
    _load().oracle_set_num_threads(int(k))


def accel(x, m, eps, G=1.0, xj=None, potential=False):
    """Eq. (1) at every particle of x (3, n) against sources xj (default: x
    itself, with j = i skipped). Returns a (3, n), or (a, phi) with
    ``potential=True``."""
    lib = _load()
    xi = _f64(x)
    ni = xi.shape[1]
    if xj is None:
        src, self_idx = xi, np.arange(ni, dtype=np.int64)
    else:
        src, self_idx = _f64(xj), None
    nj = src.shape[1]
    mj = _f64(m, (nj,))
    acc = np.empty((3, ni))
    pot = np.empty(ni) if potential else None
    lib.oracle_accel(ni, _p(xi), None if self_idx is None else self_idx.ctypes.data_as(_I64),
                     nj, _p(src), _p(mj), float(eps), float(G), _p(acc), _p(pot))
    return (acc, pot) if potential else acc


def accel_sampled(x, m, eps, idx, G=1.0, potential=False):
    """Eq. (1) at the particles ``idx`` of the set x against the whole set
    (each sample's own term skipped). Returns a (3, len(idx))."""
    lib = _load()
    src = _f64(x)
    n = src.shape[1]
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    xi = np.ascontiguousarray(src[:, idx])
    mj = _f64(m, (n,))
    acc = np.empty((3, idx.size))
    pot = np.empty(idx.size) if potential else None
    lib.oracle_accel(idx.size, _p(xi), idx.ctypes.data_as(_I64), n, _p(src), _p(mj),
                     float(eps), float(G), _p(acc), _p(pot))
    return (acc, pot) if potential else acc


def kdk(x, v, m, eps, dt, nsteps, G=1.0, trajectory=False):
    """nsteps KDK leapfrog steps. Returns (x, v, a) at the end, plus the
    (nsteps+1, 3, n) position and velocity trajectories with
    ``trajectory=True``."""
    lib = _load()
    x = _f64(x).copy()
    v = _f64(v).copy()
    n = x.shape[1]
    mm = _f64(m, (n,))
    acc = np.empty((3, n))
    tx = np.empty((nsteps + 1, 3, n)) if trajectory else None
    tv = np.empty((nsteps + 1, 3, n)) if trajectory else None
    lib.oracle_kdk(n, _p(x), _p(v), _p(mm), float(eps), float(G), float(dt), int(nsteps),
                   _p(acc), _p(tx), _p(tv))
    if trajectory:
        return x, v, acc, tx, tv
    return x, v, acc


def diag(x, v, m, eps, G=1.0):
    """dict of KE, PE, E, P, L, COM and total mass."""
    lib = _load()
    x = _f64(x)
    n = x.shape[1]
    out = np.empty(13)
    lib.oracle_diag(n, _p(x), _p(_f64(v)), _p(_f64(m, (n,))), float(eps), float(G), _p(out))
    return dict(zip(DIAG_FIELDS, out.tolist()))


def vjp(x, m, lam, eps, G=1.0):
    """(J^T lam, G^T lam): transposed position and mass Jacobians of Eq. (1)."""
    lib = _load()
    x = _f64(x)
    n = x.shape[1]
    jt = np.empty((3, n))
    gt = np.empty(n)
    lib.oracle_vjp(n, _p(x), _p(_f64(m, (n,))), _p(_f64(lam)), float(eps), float(G),
                   _p(jt), _p(gt))
    return jt, gt


def vjp_sampled(x, m, lam, eps, idx, G=1.0):
    """Rows ``idx`` of vjp: (J^T lam)[:, idx] (3, len(idx)) and (G^T lam)[idx]."""
    lib = _load()
    x = _f64(x)
    n = x.shape[1]
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    jt = np.empty((3, idx.size))
    gt = np.empty(idx.size)
    lib.oracle_vjp_sampled(n, idx.size, idx.ctypes.data_as(_I64), _p(x), _p(_f64(m, (n,))),
                           _p(_f64(lam)), float(eps), float(G), _p(jt), _p(gt))
    return jt, gt


def jvp(x, m, u, eps, G=1.0):
    """J u: the position Jacobian of Eq. (1) applied to u (3, n)."""
    lib = _load()
    x = _f64(x)
    n = x.shape[1]
    ju = np.empty((3, n))
    lib.oracle_jvp(n, _p(x), _p(_f64(m, (n,))), _p(_f64(u)), float(eps), float(G), _p(ju))
    return ju


def adjoint(traj_x, m, eps, dt, lamx, lamv, G=1.0):
    """Reverse-mode derivative of the KDK trajectory traj_x (S+1, 3, n).
    Given lamx, lamv = dL/dx_S, dL/dv_S, returns (dL/dx_0, dL/dv_0, dL/dm)."""
    lib = _load()
    traj = _f64(traj_x)
    S = traj.shape[0] - 1
    n = traj.shape[2]
    lx = _f64(lamx).copy()
    lv = _f64(lamv).copy()
    lm = np.zeros(n)
    lib.oracle_adjoint(n, S, _p(traj), _p(_f64(m, (n,))), float(eps), float(G), float(dt),
                       _p(lx), _p(lv), _p(lm))
    return lx, lv, lm


def diffusion3d(f, dx, dy, dz, dt, kappa):
    """One explicit step of the 3-D diffusion equation on the grid f (nx, ny, nz),
    k fastest, clamped neighbours; returns fn (float64)."""
    lib = _load()
    if not hasattr(lib.oracle_diffusion3d, "_typed"):
        i64, dbl = ctypes.c_int64, ctypes.c_double
        lib.oracle_diffusion3d.argtypes = [i64, i64, i64, dbl, dbl, dbl, dbl, dbl, _D, _D]
        lib.oracle_diffusion3d.restype = None
        lib.oracle_diffusion3d._typed = True
    g = _f64(f)
    nx, ny, nz = g.shape
    out = np.empty_like(g)
    lib.oracle_diffusion3d(nx, ny, nz, float(dx), float(dy), float(dz), float(dt), float(kappa),
                           _p(g), _p(out))
    return out
