"""C-ABI contract of libnbody.so, checked without a GPU.

The library must load, export every function include/nbody.h declares, and
reject bad arguments before it makes any HIP call. The pointers below are
fake (never dereferenced): every call here fails validation, except the
no-device case, which only runs where no GPU is present.
"""

import ctypes
import subprocess

import pytest

from paper_2411_18889_amd import _lib
from paper_2411_18889_amd._lib import (NB_EINVAL, NB_ENODEV, NB_EUNSUPPORTED, NB_EWORKSPACE,
                                       NB_OK, nb_launch)

P = ctypes.c_void_p
A = P(0x100000)  # placeholder aligned addresses, for calls that must stop in validation
B = P(0x200000)
C = P(0x300000)
D = P(0x400000)
F64, F32, TILEC = 0, 1, 5


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


@pytest.fixture
def Lv(L):
    """The library, for tests that hand it placeholder pointers: they are
    meant for a host without a GPU (where nothing can be launched); with a
    device present they are skipped."""
    _skip_if_device(L)
    return L


def test_every_declared_symbol_is_exported(L):
    names = _lib.declared_functions()
    assert {"nbody_accel", "nbody_step", "nbody_step_adjoint", "nbody_diag"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in names:
        assert name in exported, name
        assert hasattr(L, name)


def test_strerror(L):
    texts = {_lib.strerror(s) for s in range(6)}
    assert len(texts) == 6
    assert _lib.strerror(NB_OK) == "success"
    assert _lib.strerror(99) == "unknown status"


def test_workspace_size(L):
    assert L.nbody_workspace_size(9, 1000, F64) == 0        # unknown op
    assert L.nbody_workspace_size(0, 1000, 17) == 0         # unknown precision
    assert L.nbody_workspace_size(0, 0, F64) == 0           # n < 1
    assert L.nbody_workspace_size(3, 1000, F64) > 0         # diagnostics always need some
    assert L.nbody_workspace_size(0, 64, F64) == 0          # one source tile: no partials
    assert L.nbody_workspace_size(0, 1024, F64) > 0         # small N: short source ranges
    assert L.nbody_workspace_size(0, 4096, TILEC) > 0       # split source ranges: partials
    assert L.nbody_workspace_size(0, 1 << 20, TILEC) > 0
    assert L.nbody_workspace_size(2, 4096, TILEC) > 0
    # a set acting on itself with the tile-compensated policy from 12288 on:
    # the symmetric pass, one FP32 partial per particle, component and block
    # (blocks of at most min(n/48, 512) particles below 81920, 1024 up to 2^18,
    # 2048 from there); the whole set of partials up to 4 GiB
    assert L.nbody_workspace_size(1, 12288, TILEC) == 48 * 3 * 12288 * 4
    assert L.nbody_workspace_size(1, 16384, TILEC) == 64 * 3 * 16384 * 4
    assert L.nbody_workspace_size(1, 24576, TILEC) == 48 * 3 * 24576 * 4
    assert L.nbody_workspace_size(1, 32768, TILEC) == 64 * 3 * 32768 * 4
    assert L.nbody_workspace_size(1, 1 << 17, TILEC) == 128 * 3 * (1 << 17) * 4
    assert L.nbody_workspace_size(1, 1 << 18, TILEC) == 128 * 3 * (1 << 18) * 4
    # beyond 4 GiB of partials the pass runs in bands of about 4 GiB, after
    # FP64 running sums (3 per particle)
    G4 = 4 << 30
    for n in (1 << 20, 1 << 21, 3 << 20, 5 << 20):
        assert L.nbody_workspace_size(1, n, TILEC) == 3 * n * 8 + G4, n
    # ... or one row of blocks per band where a row needs more (2^28: blocks
    # of 2048, a row holds the slot of every particle and the 131071 other
    # slots of its own 2048)
    n = 1 << 28
    assert L.nbody_workspace_size(1, n, TILEC) == 3 * n * 8 + 3 * 4 * (n + 131071 * 2048)
    # FP32: FP32 running sums; FP64: FP64 partials
    assert L.nbody_workspace_size(1, 1 << 20, F32) == 3 * (1 << 20) * 4 + G4
    assert L.nbody_workspace_size(1, 1 << 20, F64) == 3 * (1 << 20) * 8 + G4
    assert L.nbody_workspace_size(1, 1 << 17, F64) == 128 * 3 * (1 << 17) * 8
    # nbody_accel covers the symmetric pass with the potential too: four
    # partials (and running sums) per particle
    assert L.nbody_workspace_size(0, 1 << 20, TILEC) == 4 * (1 << 20) * 8 + G4
    assert L.nbody_workspace_size(0, 1 << 18, TILEC) == 128 * 4 * (1 << 18) * 4
    # and a small sink set against up to n sources: at most 64 one-tile source
    # ranges below 16384 sources, n / 512 above, <= 2^24 sink-ranges in all,
    # 4 FP64 partials each
    assert L.nbody_workspace_size(0, 16384, TILEC) == 64 * 16384 * 4 * 8
    assert L.nbody_workspace_size(0, 1 << 30, TILEC) == (1 << 24) * 4 * 8
    assert L.nbody_workspace_size(0, 1 << 30, F64) == (1 << 24) * 4 * 8
    # and the symmetric adjoint pass: seven FP32 partials per particle and
    # block (blocks of min(n/64, 512) below 163840, 1024 from there at every
    # n), all of them up to 4 GiB, then seven FP64 running sums and bands of
    # about 4 GiB
    assert L.nbody_workspace_size(2, 12288, TILEC) == 48 * 7 * 12288 * 4
    assert L.nbody_workspace_size(2, 16384, TILEC) == 64 * 7 * 16384 * 4
    assert L.nbody_workspace_size(2, 32768, TILEC) == 64 * 7 * 32768 * 4
    assert L.nbody_workspace_size(2, 1 << 17, TILEC) == 256 * 7 * (1 << 17) * 4
    assert L.nbody_workspace_size(2, 1 << 18, TILEC) == 256 * 7 * (1 << 18) * 4
    for n in (1 << 19, 1 << 20, 1 << 21, 3 << 20):
        assert L.nbody_workspace_size(2, n, TILEC) == 7 * n * 8 + G4, n
    n = 1 << 28
    assert L.nbody_workspace_size(2, n, TILEC) == 7 * n * 8 + 7 * 4 * (n + 262143 * 1024)
    # FP32 and FP64 take the symmetric adjoint too (FP64: FP64 partials, in
    # blocks of 256 below 24576, 512 below 98304, 1024 from there; FP32 as
    # the tile-compensated policy); the running sums are FP64 for all three
    assert L.nbody_workspace_size(2, 16384, F64) == 64 * 7 * 16384 * 8
    assert L.nbody_workspace_size(2, 32768, F64) == 64 * 7 * 32768 * 8
    assert L.nbody_workspace_size(2, 1 << 17, F64) == 128 * 7 * (1 << 17) * 8
    assert L.nbody_workspace_size(2, 1 << 18, F64) == 256 * 7 * (1 << 18) * 8
    assert L.nbody_workspace_size(2, 1 << 20, F64) == 7 * (1 << 20) * 8 + G4
    assert L.nbody_workspace_size(2, 65536, F32) == 128 * 7 * 65536 * 4
    assert L.nbody_workspace_size(2, 1 << 20, F32) == 7 * (1 << 20) * 8 + G4
    # the one-sided adjoint kernel (other policies, and below 12288):
    # split partials or none
    assert L.nbody_workspace_size(2, 1 << 20, 3) == 8 * 7 * (1 << 20) * 8
    assert L.nbody_workspace_size(2, 8192, F64) == 32 * 7 * 8192 * 8


def _skip_if_device(L):
    """Calls whose arguments pass validation launch kernels when a device is
    present; with the placeholder pointers of these tests that would be an
    access to memory nobody allocated. Such checks run only without a GPU."""
    buf = ctypes.create_string_buffer(128)
    if L.nbody_device_info(buf, 128) != NB_ENODEV:
        pytest.skip("a GPU is present: valid calls would launch on placeholder pointers")


def test_accel_workspace_covers_every_set_size(Lv):
    L = Lv
    """nbody_workspace_size(NB_OP_ACCEL, max(ni, nj)) is enough for every
    ni, nj up to it. Checked through the library's own validation, which
    rejects a short workspace (NB_EWORKSPACE) before it looks for a device,
    so without a GPU every sufficient call ends at NB_ENODEV."""
    base = 1 << 40
    xi, xj, mj, acc, pot, ws = (base + (k << 38) for k in range(6))
    sinks = {1, 16, 63, 64, 65, 255, 256, 257, 1000, 3071, 3072, 4095, 12288, 12289, 16383,
             16384, 65535, 65536, 65537, 1 << 20}
    sinks |= {g * 1024 for g in range(4096, 8193, 257)} | {8191 * 1024, 4097 * 1024 - 1}
    for prec in range(6):
        for nmax in (100, 1000, 5000, 20000, 70000, 1 << 20, 1 << 22, 1 << 24, 1 << 30):
            w = L.nbody_workspace_size(0, nmax, prec)
            for ni in sorted(k for k in sinks if k <= nmax) + [nmax]:
                for nj in {nmax, max(1, nmax // 3)}:
                    if max(ni, nj) != nmax:
                        continue
                    srcs = (xj, xi) if ni == nj else (xj,)  # and the set on itself
                    for src in srcs:
                        for p in (None, pot):
                            st = L.nbody_accel(ni, xi, nj, src, mj, 0.01, 1.0, prec, acc, p,
                                               ws if w else None, w, None)
                            assert st == NB_ENODEV, (prec, nmax, ni, nj, src == xi, p, st)


def _accel(L, ni=64, xi=A, nj=64, xj=B, mj=C, eps=0.1, G=1.0, prec=F64, acc=D, pot=None,
           ws=None, wsb=0):
    return L.nbody_accel(ni, xi, nj, xj, mj, eps, G, prec, acc, pot, ws, wsb, None)


def test_accel_validation(Lv):
    L = Lv
    assert _accel(L, ni=0) == NB_EINVAL
    assert _accel(L, nj=0) == NB_EINVAL
    assert _accel(L, ni=(1 << 30) + 1) == NB_EINVAL
    assert _accel(L, eps=0.0) == NB_EINVAL
    assert _accel(L, eps=-1.0) == NB_EINVAL
    assert _accel(L, eps=float("nan")) == NB_EINVAL
    assert _accel(L, eps=float("inf")) == NB_EINVAL
    assert _accel(L, eps=2.0 ** -41, prec=F32) == NB_EINVAL   # FP32 needs eps >= 2^-40
    assert _accel(L, G=float("inf")) == NB_EINVAL
    assert _accel(L, xi=None) == NB_EINVAL
    assert _accel(L, acc=None) == NB_EINVAL
    assert _accel(L, xi=P(0x100004)) == NB_EINVAL              # misaligned for double
    assert _accel(L, mj=P(0x300002), prec=F32) == NB_EINVAL     # misaligned for float
    assert _accel(L, xi=A, xj=A, ni=64, nj=65) == NB_EINVAL     # same set, different counts
    assert _accel(L, acc=P(0x100000 + 8)) == NB_EINVAL         # output overlaps the sinks
    assert _accel(L, pot=P(0x400000 + 8)) == NB_EINVAL         # potential overlaps acc
    assert _accel(L, prec=9) == NB_EUNSUPPORTED


def test_accel_workspace_checked_before_device(L):
    bound = L.nbody_workspace_size(0, 4096, TILEC)
    args = dict(ni=4096, nj=4096, xi=P(0x1000000), xj=P(0x2000000), mj=P(0x3000000),
                acc=P(0x4000000), prec=TILEC)
    assert _accel(L, **args) == NB_EWORKSPACE
    assert _accel(L, ws=P(0x5000000), wsb=1024, **args) == NB_EWORKSPACE
    assert _accel(L, ws=P(0x5000000 + 128), wsb=bound, **args) == NB_EWORKSPACE  # not 256-aligned
    _skip_if_device(L)
    assert _accel(L, ws=P(0x5000000), wsb=bound, **args) == NB_ENODEV
    # the exact need of this call, found through the validation itself:
    # 16 source ranges x 4 FP64 partials per sink
    lo, hi = 0, bound
    while hi - lo > 1:
        mid = (lo + hi) // 2
        lo, hi = (lo, mid) if _accel(L, ws=P(0x5000000), wsb=mid, **args) == NB_ENODEV else (mid, hi)
    assert hi == 16 * 4 * 4096 * 8 <= bound
    assert _accel(L, ws=P(0x5000000), wsb=hi - 1, **args) == NB_EWORKSPACE
    assert _accel(L, ws=P(0x5000000 + 128), wsb=hi, **args) == NB_EWORKSPACE  # not 256-aligned


def test_accel_ex_rejects_bad_shapes(Lv):
    L = Lv
    for shape in ((3, 256, 1), (2, 96, 1), (2, 256, 0x1000), (2, 2048, 1)):
        ln = nb_launch(*shape)
        st = L.nbody_accel_ex(64, A, 64, B, C, 0.1, 1.0, F64, D, None, ctypes.byref(ln), None,
                              0, None)
        assert st == NB_EUNSUPPORTED, shape


def test_step_validation(Lv):
    L = Lv
    def step(n=64, x=A, v=B, m=C, acc=D, eps=0.1, dt=0.01, nsteps=1, prec=F64, flags=0,
             ckpt=None, every=0):
        return L.nbody_step(n, x, v, m, acc, eps, 1.0, dt, nsteps, prec, flags, ckpt, every,
                            None, 0, None)
    assert step(n=0) == NB_EINVAL
    assert step(nsteps=-1) == NB_EINVAL
    assert step(dt=float("nan")) == NB_EINVAL
    assert step(flags=0x8) == NB_EINVAL
    assert step(flags=0x4 | 0x2) == NB_EINVAL                    # unknown bit beside NB_GRAPH
    assert step(v=P(0x100000 + 64)) == NB_EINVAL                 # v overlaps x
    assert step(ckpt=P(0x800000), every=0) == NB_EINVAL         # interval must be >= 1
    assert step(ckpt=P(0x400000 + 64), every=1) == NB_EINVAL     # checkpoints overlap acc
    assert step(prec=6) == NB_EUNSUPPORTED


def test_adjoint_validation(Lv):
    L = Lv
    E, Fp, Gp = P(0x500000), P(0x600000), P(0x700000)

    def adj(n=64, lam_m=Gp, flags=0, ckpt=None, every=0, step_end=0, nsteps=1):
        return L.nbody_step_adjoint(n, A, B, C, D, E, Fp, lam_m, 0.1, 1.0, 0.01, nsteps, F64,
                                    flags, ckpt, every, step_end, None, 0, None)
    assert adj(n=0) == NB_EINVAL
    assert adj(flags=0x4) == NB_EINVAL
    assert adj(lam_m=P(0x500000 + 8)) == NB_EINVAL               # lam_m overlaps lam_x
    assert adj(ckpt=P(0x900000), every=4, step_end=0, nsteps=1) == NB_EINVAL  # step_end < nsteps


def test_diag_validation(Lv):
    L = Lv
    assert L.nbody_diag(0, A, B, C, 0.1, 1.0, F64, D, None, 0, None) == NB_EINVAL
    assert L.nbody_diag(64, A, B, C, 0.1, 1.0, F64, None, None, 0, None) == NB_EINVAL
    assert L.nbody_diag(64, A, B, C, 0.1, 1.0, F64, D, None, 0, None) == NB_EWORKSPACE


def test_no_device_is_reported():
    L = _lib.lib()
    _skip_if_device(L)
    # valid arguments: the call gets as far as the device check and stops there
    assert _accel(L) == NB_ENODEV
    assert L.nbody_step(64, A, B, C, D, 0.1, 1.0, 0.01, 1, F64, 0, None, 0, None, 0, None) == NB_ENODEV
    assert L.nbody_step(64, A, B, C, D, 0.1, 1.0, 0.01, 1, F64, 0x2, None, 0, None, 0, None) == NB_ENODEV


def test_diffusion_validation(Lv):
    L = Lv
    def step(nx=8, ny=8, nz=8, dx=1.0, dy=1.0, dz=1.0, dt=0.1, kappa=1.0, f=A, fn=B):
        return L.diffusion3d_step(nx, ny, nz, dx, dy, dz, dt, kappa, f, fn, None)
    assert step(nx=0) == NB_EINVAL
    assert step(nx=(1 << 21) + 1) == NB_EINVAL
    assert step(ny=524281) == NB_EINVAL
    assert step(nx=2048, ny=2048, nz=1024) == NB_EINVAL   # more than 2^31 - 1 points
    assert step(dx=0.0) == NB_EINVAL
    assert step(dz=float("nan")) == NB_EINVAL
    assert step(dt=float("inf")) == NB_EINVAL
    assert step(f=None) == NB_EINVAL
    assert step(fn=P(0x200002)) == NB_EINVAL                  # misaligned
    assert step(fn=P(0x100000 + 64)) == NB_EINVAL              # overlaps f


def test_pass_info(L):
    from paper_2411_18889_amd import _lib
    info = _lib.nb_pass_info()
    assert L.nbody_pass_info(1, 1 << 20, TILEC, ctypes.byref(info)) == 0
    assert (info.symmetric, info.block, info.i_per_lane, info.block_particles) == (1, 256, 8, 2048)
    assert info.workspace_bytes == L.nbody_workspace_size(1, 1 << 20, TILEC)
    assert L.nbody_pass_info(2, 1 << 20, TILEC, ctypes.byref(info)) == 0
    assert (info.symmetric, info.block, info.i_per_lane, info.block_particles) == (1, 256, 4, 1024)
    assert L.nbody_pass_info(2, 1 << 17, TILEC, ctypes.byref(info)) == 0
    assert (info.symmetric, info.block, info.i_per_lane, info.block_particles) == (1, 256, 2, 512)
    assert L.nbody_pass_info(1, 1 << 16, TILEC, ctypes.byref(info)) == 0
    assert (info.symmetric, info.block, info.i_per_lane, info.block_particles) == (1, 256, 2, 512)
    assert L.nbody_pass_info(1, 1 << 17, TILEC, ctypes.byref(info)) == 0
    assert (info.symmetric, info.block, info.i_per_lane, info.block_particles) == (1, 256, 4, 1024)
    assert L.nbody_pass_info(1, 1 << 20, 2, ctypes.byref(info)) == 0  # FP32 running sums
    assert info.symmetric == 0 and info.block_particles == 0 and info.split >= 1
    assert L.nbody_pass_info(1, 1 << 18, TILEC, ctypes.byref(info)) == 0
    assert (info.symmetric, info.block, info.i_per_lane, info.block_particles) == (1, 256, 8, 2048)
    # FP64: the same shapes, FP64 partials
    assert L.nbody_pass_info(1, 1 << 17, F64, ctypes.byref(info)) == 0
    assert (info.i_per_lane, info.block_particles) == (4, 1024)
    assert L.nbody_pass_info(1, 1 << 20, F64, ctypes.byref(info)) == 0
    assert (info.symmetric, info.i_per_lane, info.block_particles) == (1, 8, 2048)
    assert info.workspace_bytes == 3 * (1 << 20) * 8 + (4 << 30)
    assert L.nbody_pass_info(1, 1 << 21, F64, ctypes.byref(info)) == 0
    assert (info.symmetric, info.block, info.i_per_lane, info.block_particles) == (1, 256, 8, 2048)
    # the symmetric passes serve every size up to 2^28: blocks of 2048
    # (force) and 1024 (adjoint) at the top
    for op, b in ((1, 2048), (2, 1024)):
        assert L.nbody_pass_info(op, 1 << 28, TILEC, ctypes.byref(info)) == 0
        assert (info.symmetric, info.block_particles) == (1, b)
    assert L.nbody_pass_info(1, (1 << 28) + 1, TILEC, ctypes.byref(info)) == 0
    assert info.symmetric == 0
    # the FP64 and FP32 adjoint: symmetric too (FP64 with four sinks per
    # lane from 49152); the compensated policies keep the one-sided kernel
    assert L.nbody_pass_info(2, 1 << 20, F64, ctypes.byref(info)) == 0
    assert (info.symmetric, info.block, info.i_per_lane, info.block_particles) == (1, 256, 4, 1024)
    assert L.nbody_pass_info(2, 65536, F64, ctypes.byref(info)) == 0
    assert (info.symmetric, info.block, info.i_per_lane, info.block_particles) == (1, 128, 4, 512)
    assert L.nbody_pass_info(2, 1 << 20, F32, ctypes.byref(info)) == 0
    assert (info.symmetric, info.block_particles) == (1, 1024)
    assert L.nbody_pass_info(2, 1 << 20, 3, ctypes.byref(info)) == 0 and info.symmetric == 0
    assert L.nbody_pass_info(1, 1000, TILEC, ctypes.byref(info)) == 0 and info.symmetric == 0
    # the symmetric passes start at 12288 particles
    for op, prec in ((1, TILEC), (2, TILEC), (2, F64), (2, F32)):
        assert L.nbody_pass_info(op, 12287, prec, ctypes.byref(info)) == 0 and info.symmetric == 0
        assert L.nbody_pass_info(op, 12288, prec, ctypes.byref(info)) == 0 and info.symmetric == 1
        assert info.block_particles == 256
    assert L.nbody_pass_info(0, 1000, TILEC, ctypes.byref(info)) == NB_EINVAL
    assert L.nbody_pass_info(1, 0, TILEC, ctypes.byref(info)) == NB_EINVAL
    assert L.nbody_pass_info(1, 1000, 17, ctypes.byref(info)) == NB_EUNSUPPORTED
    assert L.nbody_pass_info(1, 1000, TILEC, None) == NB_EINVAL


def test_plain_c_consumer(Lv, tmp_path):
    """The headers compile as strict C99 and as C++, and a C program linked
    against libnbody.so (no Python, no torch) gets the same answers from the
    host-only entry points and the argument validation."""
    import os
    import shutil
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("no host C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    inc = os.path.join(root, "include")
    libdir = os.path.dirname(_lib.LIB_PATH)
    exe = str(tmp_path / "abi_consumer")
    cc = ["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-I", inc,
          os.path.join(root, "tests", "c", "abi_consumer.c"), "-L", libdir, "-lnbody",
          "-Wl,-rpath," + libdir, "-Wl,-rpath-link,/opt/rocm/lib", "-o", exe]
    r = subprocess.run(cc, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run(["g++", "-std=c++11", "-Wall", "-Werror", "-fsyntax-only", "-x", "c++",
                        "-I", inc, "-"], input='#include "diffusion3d.h"\n#include "nbody.h"\n',
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout, r.stderr)


def test_workspace_overlap_rejected(L):
    """A workspace that overlaps any buffer of the call is rejected
    (NB_EINVAL) before any HIP call, as is a potential overlapping the
    masses: the kernels would race on them. These calls stop in the
    validation, so they run with or without a GPU."""
    MiB = 1 << 20
    xi, xj, mj, acc, pot, ws = (P(k * 64 * MiB) for k in range(1, 7))
    args = dict(ni=4096, nj=4096, xi=xi, xj=xj, mj=mj, acc=acc, prec=TILEC)
    need = 16 * 4 * 4096 * 8  # 16 source ranges x 4 FP64 partials per sink
    for target in (xi, xj, mj, acc):
        assert _accel(L, ws=P(target.value - 256), wsb=need, **args) == NB_EINVAL
    assert _accel(L, pot=pot, ws=P(pot.value - 256), wsb=need, **args) == NB_EINVAL
    assert _accel(L, pot=P(mj.value + 64), **args) == NB_EINVAL  # potential over the masses
    # the symmetric pass of a set on itself: partials per block
    n = 20000
    wsn = L.nbody_workspace_size(1, n, TILEC)
    x, v, m, a = (P(k * 64 * MiB) for k in range(1, 5))
    for target in (x, v, m, a):
        st = L.nbody_step(n, x, v, m, a, 0.01, 1.0, 0.01, 1, TILEC, 0, None, 0,
                          P(target.value - 256), wsn, None)
        assert st == NB_EINVAL
    ck = P(5 * 64 * MiB)
    st = L.nbody_step(n, x, v, m, a, 0.01, 1.0, 0.01, 2, TILEC, 0, ck, 1, P(ck.value + 256), wsn, None)
    assert st == NB_EINVAL
    wsa = L.nbody_workspace_size(2, n, TILEC)
    lx, lv, lm = (P(k * 64 * MiB) for k in range(6, 9))
    for target in (x, lx, lv, lm):
        st = L.nbody_step_adjoint(n, x, v, m, a, lx, lv, lm, 0.01, 1.0, 0.01, 1, TILEC, 0, None, 0,
                                  0, P(target.value - 256), wsa, None)
        assert st == NB_EINVAL
    wsd = L.nbody_workspace_size(3, n, TILEC)
    out = P(9 * 64 * MiB)
    assert L.nbody_diag(n, x, v, m, 0.01, 1.0, TILEC, out, P(out.value - 256), wsd, None) == NB_EINVAL
    assert L.nbody_diag(n, x, v, m, 0.01, 1.0, TILEC, out, P(v.value + 256), wsd, None) == NB_EINVAL


def test_explicit_pass_shapes_validated(L):
    """Explicit launch shapes of the symmetric passes and of the one-sided
    adjoint: shapes the library is not built for, a symmetric shape for
    separate sets or for a policy without that pass, and a split of the
    symmetric pass are refused (NB_EUNSUPPORTED) before any device call;
    the workspace query answers per shape."""
    MiB = 1 << 20
    x, m, acc = P(64 * MiB), P(128 * MiB), P(192 * MiB)
    xj = P(256 * MiB)

    def ex(n, launch, prec=TILEC, src=None):
        ln = nb_launch(*launch)
        return L.nbody_accel_ex(n, x, n, src or x, m, 0.01, 1.0, prec, acc, None,
                                ctypes.byref(ln), None, 0, None)
    assert ex(20000, (4, 256, 1, 1), src=xj) == NB_EUNSUPPORTED   # separate sets
    assert ex(20000, (4, 192, 0, 1)) == NB_EUNSUPPORTED           # not whole waves
    assert ex(20000, (1, 256, 0, 1)) == NB_EUNSUPPORTED           # force: 2 or 4 per lane
    assert ex(20000, (4, 2048, 0, 1)) == NB_EUNSUPPORTED          # at most 16 waves
    assert ex(20000, (4, 256, 2, 1)) == NB_EUNSUPPORTED           # no split
    assert ex(20000, (4, 256, 0, 1), prec=3) == NB_EUNSUPPORTED   # Kahan: no symmetric pass
    assert ex(1000, (0, 0, 0, 1)) == NB_EUNSUPPORTED              # library picks one-sided there

    def adj(launch, prec=TILEC, n=20000):
        ln = nb_launch(*launch)
        lx, lv, lm, v = P(320 * MiB), P(384 * MiB), P(448 * MiB), P(512 * MiB)
        return L.nbody_step_adjoint_ex(n, x, v, m, acc, lx, lv, lm, 0.01, 1.0, 0.01, 1, prec, 0,
                                       None, 0, 0, ctypes.byref(ln), None, 0, None)
    assert adj((2, 256, 0, 1), prec=3) == NB_EUNSUPPORTED         # Kahan: one-sided only
    assert adj((2, 1024, 0, 1), prec=F64) == NB_EUNSUPPORTED      # FP64: up to 8 waves
    assert adj((3, 256, 0, 1)) == NB_EUNSUPPORTED                 # adjoint: 1, 2 or 4 per lane
    assert adj((4, 1024, 0, 1)) == NB_EUNSUPPORTED                # 4 per lane: up to 8 waves
    assert adj((1, 128, 0, 1)) == NB_EUNSUPPORTED                 # 1 per lane: 4 or 8 waves
    assert adj((1, 1024, 1, 0)) == NB_EUNSUPPORTED                # one-sided: up to 512 lanes
    assert adj((4, 256, 1, 0)) == NB_EUNSUPPORTED
    # the workspace a shape asks for: symmetric partials (every one up to
    # 4 GiB), or one-sided FP64 split partials
    q = L.nbody_pass_workspace_size
    ln = nb_launch(2, 256, 0, 1)   # blocks of 512
    assert q(0, 20000, 20000, TILEC, 1, 0, ctypes.byref(ln)) == 40 * 3 * 20000 * 4
    assert q(0, 20000, 20000, TILEC, 1, 1, ctypes.byref(ln)) == 40 * 4 * 20000 * 4
    assert q(0, 20000, 20000, F32, 1, 0, ctypes.byref(ln)) == 40 * 3 * 20000 * 4
    assert q(0, 20000, 20000, F64, 1, 0, ctypes.byref(ln)) == 40 * 3 * 20000 * 8
    assert q(0, 20000, 20000, TILEC, 0, 0, ctypes.byref(ln)) == 0  # separate sets: refused
    assert q(2, 20000, 20000, TILEC, 1, 0, ctypes.byref(ln)) == 40 * 7 * 20000 * 4
    assert q(2, 20000, 20000, F32, 1, 0, ctypes.byref(ln)) == 40 * 7 * 20000 * 4
    assert q(2, 20000, 20000, F64, 1, 0, ctypes.byref(ln)) == 40 * 7 * 20000 * 8
    ln = nb_launch(1, 256, 5, 0)
    assert q(2, 20000, 20000, F64, 1, 0, ctypes.byref(ln)) == 5 * 7 * 20000 * 8
    assert q(0, 20000, 700, TILEC, 0, 0, ctypes.byref(ln)) == 5 * 4 * 20000 * 8
    assert q(2, 20000, 20001, TILEC, 1, 0, None) == 0
    assert q(1, 20000, 20000, TILEC, 1, 0, None) == 0              # op: ACCEL or ADJOINT
    # the library's own shapes agree with nbody_workspace_size
    assert q(2, 1 << 20, 1 << 20, TILEC, 1, 0, None) == L.nbody_workspace_size(2, 1 << 20, TILEC)
    assert q(0, 1 << 20, 1 << 20, TILEC, 1, 0, None) == L.nbody_workspace_size(1, 1 << 20, TILEC)
