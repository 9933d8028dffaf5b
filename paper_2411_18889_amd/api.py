"""Tensor-level binding of libnbody: argument checks and marshalling only.

Every computation runs in the library's HIP kernels; this module only checks
tensor dtypes, devices and shapes, sizes the workspace, and passes pointers
and the current HIP stream through the C ABI.

Layout: positions, velocities, accelerations and adjoints are (3, n)
contiguous tensors (rows x, y, z); masses and potentials are (n,).
Precision names: "f64", "f32", "mix_acc32", "mix_kahan", "mix_acc64",
"mix_tilec" (see include/nbody.h).
"""

from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import PREC, check, nb_launch


def pos_dtype(prec: str):
    return torch.float32 if prec == "f32" else torch.float64


def mass_dtype(prec: str):
    return torch.float64 if prec == "f64" else torch.float32


def _prec(prec: str) -> int:
    if prec not in PREC:
        raise ValueError("unknown precision %r (one of %s)" % (prec, sorted(PREC)))
    return PREC[prec]


def _vec(t, name, n, dtype, rows=3):
    shape = (rows, n) if rows else (n,)
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != shape or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s tensor, got %s" % (name, shape, tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def workspace_size(op: int, n: int, prec: str) -> int:
    return int(_lib.lib().nbody_workspace_size(op, int(n), _prec(prec)))


def _workspace(op, n, prec, device):
    nbytes = workspace_size(op, n, prec)
    if nbytes == 0:
        return None, ctypes.c_void_p(0), 0
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    return ws, ctypes.c_void_p(ws.data_ptr()), nbytes


def _user_workspace(workspace):
    if workspace.dtype != torch.uint8 or not workspace.is_contiguous() or workspace.device.type != "cuda":
        raise ValueError("workspace: contiguous uint8 CUDA tensor")
    return ctypes.c_void_p(workspace.data_ptr() if workspace.numel() else 0), workspace.numel()


def _launch(launch):
    """An nb_launch from a dict with any of the keys i_per_lane, block, split,
    symmetric (missing = 0 = the library's choice), or None."""
    if launch is None:
        return None
    bad = set(launch) - {"i_per_lane", "block", "split", "symmetric"}
    if bad:
        raise ValueError("unknown launch fields %s" % sorted(bad))
    return nb_launch(*[int(launch.get(k, 0)) for k in ("i_per_lane", "block", "split", "symmetric")])


def accel(x, m, eps, G=1.0, prec="mix_tilec", xj=None, potential=False, launch=None,
          out=None, stream=None, workspace=None):
    """a (3, ni) of the sinks x (3, ni) from the sources xj (3, nj) with masses m
    (nj,) -- Eq. (1). xj=None: the set x acts on itself. potential=True also
    returns phi (ni,). workspace: optional uint8 device tensor (the library
    checks that it is large enough); by default one of the size the library
    asks for is allocated."""
    p = _prec(prec)
    pdt, mdt = pos_dtype(prec), mass_dtype(prec)
    ni = x.shape[1]
    src = x if xj is None else xj
    nj = src.shape[1]
    px = _vec(x, "x", ni, pdt)
    pj = px if xj is None else _vec(xj, "xj", nj, pdt)
    pm = _vec(m, "m", nj, mdt, rows=0)
    acc = torch.empty((3, ni), dtype=pdt, device=x.device) if out is None else out
    pa = _vec(acc, "out", ni, pdt)
    pot = torch.empty(ni, dtype=pdt, device=x.device) if potential else None
    pp = _vec(pot, "pot", ni, pdt, rows=0) if potential else ctypes.c_void_p(0)
    L = _lib.lib()
    ln = _launch(launch)
    if workspace is not None:
        pws, nws = _user_workspace(workspace)
    else:
        nws = int(L.nbody_pass_workspace_size(_lib.NB_OP_ACCEL, ni, nj, p, int(xj is None),
                                              int(bool(potential)),
                                              None if ln is None else ctypes.byref(ln)))
        ws = torch.empty(nws, dtype=torch.uint8, device=x.device) if nws else None
        pws = ctypes.c_void_p(ws.data_ptr() if nws else 0)
    if ln is None:
        st = L.nbody_accel(ni, px, nj, pj, pm, float(eps), float(G), p, pa, pp, pws, nws,
                           _stream(stream))
    else:
        st = L.nbody_accel_ex(ni, px, nj, pj, pm, float(eps), float(G), p, pa, pp,
                              ctypes.byref(ln), pws, nws, _stream(stream))
    check(st, "nbody_accel")
    return (acc, pot) if potential else acc


def step(x, v, m, acc, eps, dt, nsteps, G=1.0, prec="mix_tilec", acc_valid=False,
         ckpt=None, ckpt_every=0, stream=None, graph=False, workspace=None):
    """nsteps KDK steps in place on x, v, acc. ckpt: optional tensor of
    (nsteps // ckpt_every + 1, 9 n) pos elements receiving (x, v, acc) every
    ckpt_every steps. graph=True replays the loop as a cached HIP graph
    (NB_GRAPH); pass the same `workspace` (uint8 tensor of at least
    workspace_size(NB_OP_STEP, n, prec) bytes) on every call so that the
    cached graph is found again."""
    p = _prec(prec)
    pdt, mdt = pos_dtype(prec), mass_dtype(prec)
    n = x.shape[1]
    args = [_vec(x, "x", n, pdt), _vec(v, "v", n, pdt), _vec(m, "m", n, mdt, rows=0),
            _vec(acc, "acc", n, pdt)]
    if ckpt is not None:
        slots = nsteps // ckpt_every + 1
        pc = _vec(ckpt, "ckpt", 9 * n, pdt, rows=slots)
    else:
        pc = ctypes.c_void_p(0)
    if workspace is not None:
        pws, nws = _user_workspace(workspace)
    else:
        ws, pws, nws = _workspace(_lib.NB_OP_STEP, n, prec, x.device)
    flags = (_lib.NB_ACC_VALID if acc_valid else 0) | (_lib.NB_GRAPH if graph else 0)
    st = _lib.lib().nbody_step(n, *args, float(eps), float(G), float(dt), int(nsteps), p,
                               flags, pc, int(ckpt_every), pws, nws, _stream(stream))
    check(st, "nbody_step")


def step_adjoint(x, v, m, acc, lam_x, lam_v, lam_m, eps, dt, nsteps, G=1.0,
                 prec="mix_tilec", entry_half=False, exit_full=False, ckpt=None,
                 ckpt_every=0, step_end=0, stream=None, workspace=None, launch=None):
    """Walk nsteps KDK steps back from (x, v, acc), updating the adjoints
    lam_x, lam_v (3, n) and lam_m (n, float64) in place. workspace: as
    accel; launch: an explicit shape of the fused adjoint passes (as
    accel's)."""
    p = _prec(prec)
    pdt, mdt = pos_dtype(prec), mass_dtype(prec)
    n = x.shape[1]
    args = [_vec(x, "x", n, pdt), _vec(v, "v", n, pdt), _vec(m, "m", n, mdt, rows=0),
            _vec(acc, "acc", n, pdt), _vec(lam_x, "lam_x", n, pdt), _vec(lam_v, "lam_v", n, pdt),
            _vec(lam_m, "lam_m", n, torch.float64, rows=0)]
    if ckpt is not None:
        slots = ckpt.shape[0]
        pc = _vec(ckpt, "ckpt", 9 * n, pdt, rows=slots)
    else:
        pc = ctypes.c_void_p(0)
    flags = (_lib.NB_ADJ_ENTRY_HALF if entry_half else 0) | (_lib.NB_ADJ_EXIT_FULL if exit_full else 0)
    L = _lib.lib()
    ln = _launch(launch)
    if workspace is not None:
        pws, nws = _user_workspace(workspace)
    elif ln is None:
        ws, pws, nws = _workspace(_lib.NB_OP_ADJOINT, n, prec, x.device)
    else:
        nws = int(L.nbody_pass_workspace_size(_lib.NB_OP_ADJOINT, n, n, p, 1, 0, ctypes.byref(ln)))
        ws = torch.empty(nws, dtype=torch.uint8, device=x.device) if nws else None
        pws = ctypes.c_void_p(ws.data_ptr() if nws else 0)
    if ln is None:
        st = L.nbody_step_adjoint(n, *args, float(eps), float(G), float(dt), int(nsteps), p, flags,
                                  pc, int(ckpt_every), int(step_end), pws, nws, _stream(stream))
    else:
        st = L.nbody_step_adjoint_ex(n, *args, float(eps), float(G), float(dt), int(nsteps), p,
                                     flags, pc, int(ckpt_every), int(step_end), ctypes.byref(ln),
                                     pws, nws, _stream(stream))
    check(st, "nbody_step_adjoint")


DIAG_FIELDS = ("KE", "PE", "E", "Px", "Py", "Pz", "Lx", "Ly", "Lz",
               "COMx", "COMy", "COMz", "M")


def diag(x, v, m, eps, G=1.0, prec="mix_tilec", stream=None, out=None):
    """FP64 conserved quantities as a (13,) float64 device tensor (fields in
    DIAG_FIELDS order)."""
    p = _prec(prec)
    pdt, mdt = pos_dtype(prec), mass_dtype(prec)
    n = x.shape[1]
    res = torch.empty(13, dtype=torch.float64, device=x.device) if out is None else out
    ws, pws, nws = _workspace(_lib.NB_OP_DIAG, n, prec, x.device)
    st = _lib.lib().nbody_diag(n, _vec(x, "x", n, pdt), _vec(v, "v", n, pdt),
                               _vec(m, "m", n, mdt, rows=0), float(eps), float(G), p,
                               _vec(res, "out", 13, torch.float64, rows=0), pws, nws,
                               _stream(stream))
    check(st, "nbody_diag")
    return res


def diag_dict(res) -> dict:
    return dict(zip(DIAG_FIELDS, res.tolist()))


def diffusion3d_step(f, dx, dy, dz, dt, kappa, out=None, stream=None):
    """One explicit step of the 3-D diffusion equation on the FP32 grid f
    (nx, ny, nz), k fastest, clamped neighbours; returns fn (nx, ny, nz)."""
    if not isinstance(f, torch.Tensor) or f.device.type != "cuda" or f.dtype != torch.float32 \
            or f.dim() != 3 or not f.is_contiguous():
        raise ValueError("f must be a contiguous float32 CUDA tensor of shape (nx, ny, nz)")
    fn = torch.empty_like(f) if out is None else out
    if fn.shape != f.shape or fn.dtype != f.dtype or not fn.is_contiguous() or fn.device != f.device:
        raise ValueError("out must match f")
    nx, ny, nz = f.shape
    st = _lib.lib().diffusion3d_step(nx, ny, nz, float(dx), float(dy), float(dz), float(dt),
                                     float(kappa), ctypes.c_void_p(f.data_ptr()),
                                     ctypes.c_void_p(fn.data_ptr()), _stream(stream))
    check(st, "diffusion3d_step")
    return fn


def device_info() -> str:
    buf = ctypes.create_string_buffer(256)
    st = _lib.lib().nbody_device_info(buf, 256)
    check(st, "nbody_device_info")
    return buf.value.decode()


def graph_cache_clear():
    """Free the HIP graphs that step(graph=True) cached (after their last
    launches finish)."""
    check(_lib.lib().nbody_graph_cache_clear(), "nbody_graph_cache_clear")


def pass_info(op: int, n: int, prec: str) -> dict:
    """The pair pass the library runs for n particles on themselves
    (op 1 = force of a leapfrog, 2 = fused adjoint): nbody_pass_info."""
    info = _lib.nb_pass_info()
    check(_lib.lib().nbody_pass_info(int(op), int(n), _prec(prec), ctypes.byref(info)),
          "nbody_pass_info")
    return {f: getattr(info, f) for f, _ in info._fields_}
