"""The library driven from a plain C program (tests/c/abi_gpu_consumer.c):
HIP runtime calls for device memory and the C ABI for the rest, no Python
and no torch in that process. Its force pass is checked against the oracle,
and its force, leapfrog (replayed as a HIP graph) and diagnostics against the
same calls made through the Python binding: bitwise equal, since every pass
sums in a fixed order."""

import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

import oracle
import paper_2411_18889_amd as nb
from nbody_inputs import plummer_sphere
from paper_2411_18889_amd import _lib
from tests.gpu_util import host, rel, to_dev

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    libdir = os.path.dirname(_lib.LIB_PATH)
    exe = str(tmp_path / "abi_gpu_consumer")
    cmd = ["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-isystem", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "abi_gpu_consumer.c"), "-L", libdir, "-lnbody",
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath," + libdir, "-Wl,-rpath,/opt/rocm/lib",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@pytest.mark.parametrize("n", [1000, 20000])
def test_c_program_matches_binding_and_oracle(tmp_path, n):
    exe = _build(tmp_path)
    S, eps, dt = 5, 2.0 ** -7, 2.0 ** -8
    x, v, m = plummer_sphere(n, 500 + n % 13)
    m = (m * np.random.default_rng(n).uniform(0.5, 1.5, size=n)).astype(np.float32)
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as fh:
        fh.write(np.array([n, S], dtype=np.int64).tobytes())
        fh.write(np.array([eps, dt], dtype=np.float64).tobytes())
        fh.write(np.ascontiguousarray(x).tobytes())
        fh.write(np.ascontiguousarray(v).tobytes())
        fh.write(m.tobytes())
    print("C consumer: n=%d" % n, flush=True)
    r = subprocess.run([exe, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = np.fromfile(out, dtype=np.float64)
    assert raw.size == 4 * 3 * n + 13
    a0, xs, vs, acs = (raw[k * 3 * n:(k + 1) * 3 * n].reshape(3, n) for k in range(4))
    dg = raw[12 * n:]
    # the force pass against the oracle
    assert rel(a0, oracle.accel(x, m.astype(np.float64), eps)) <= 1e-5
    # and the same calls through the binding, bitwise
    xd, vd, md = to_dev(x, v, m, "mix_tilec")
    assert np.array_equal(host(nb.accel(xd, md, eps, prec="mix_tilec")), a0)
    acc = nb.accel(xd, md, eps, prec="mix_tilec")
    nb.step(xd, vd, md, acc, eps, dt, S, prec="mix_tilec", acc_valid=True)
    assert np.array_equal(host(xd), xs) and np.array_equal(host(vd), vs)
    assert np.array_equal(host(acc), acs)
    assert np.array_equal(host(nb.diag(xd, vd, md, eps, prec="mix_tilec")), dg)
    torch.cuda.synchronize()
