"""The oracle's pins catch plausible mistakes.

Each mutant is a copy of oracle/nbody_oracle.c with one planted slip (a sign,
an exponent, an index, a dropped term, a swapped sub-step), built on the CPU
into a temporary library. The oracle pin tests are then run against that
library (NBODY_ORACLE_LIB) in a child process, and at least one of them must
fail. The original source must pass the same run.
"""

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nbody_oracle.c")
PIN_TESTS = ["tests/test_oracle_force.py", "tests/test_oracle_kdk.py",
             "tests/test_oracle_adjoint.py", "tests/test_oracle_diffusion.py"]

MUTANTS = {
    "force_sign": ("const double dx = xj[j] - px;", "const double dx = px - xj[j];"),
    "force_index": ("const double dy = xj[nj + j] - py;", "const double dy = xj[j] - py;"),
    "force_exponent": ("const double s32 = s * r; /*", "const double s32 = s; /*"),
    "force_mass_dropped": ("ax += mj[j] * dx / s32;", "ax += dx / s32;"),
    "force_softening_dropped": ("const double s = dx * dx + dy * dy + dz * dz + eps2;\n            const double r",
                                "const double s = dx * dx + dy * dy + dz * dz;\n            const double r"),
    "force_G_dropped": ("acc[ni + i] = G * ay;", "acc[ni + i] = ay;"),
    "self_not_skipped": ("if (j == self)\n                continue;", ""),
    "potential_sign": ("pot[i] = -G * phi;", "pot[i] = G * phi;"),
    "kdk_full_kick": ("const double h = 0.5 * dt;\n    const size_t n3 = 3 * (size_t)n;\n    accel_self",
                      "const double h = dt;\n    const size_t n3 = 3 * (size_t)n;\n    accel_self"),
    "kdk_drift_before_kick": ("            v[k] = v[k] + h * acc[k];\n        for (size_t k = 0; k < n3; k++)\n            x[k] = x[k] + dt * v[k];",
                              "            x[k] = x[k] + dt * v[k];\n        for (size_t k = 0; k < n3; k++)\n            v[k] = v[k] + h * acc[k];"),
    "diag_pe_mass": ("pe += m[i] * row[i];", "pe += row[i];"),
    "diag_L_sign": ("l[1] += m[i] * (rz * vx - rx * vz);", "l[1] += m[i] * (rx * vz - rz * vx);"),
    "T_factor": ("out[1] += c * (w[1] / s32 - 3.0 * d[1] * dw / s52);",
                 "out[1] += c * (w[1] / s32 - 2.0 * d[1] * dw / s52);"),
    "vjp_diag_sign": ("jt[1] = G * (off[1] - diag[1]);", "jt[1] = G * (off[1] + diag[1]);"),
    "vjp_mass_transposed": ("add_T_times(d, s32, s52, m[k], li, off);", "add_T_times(d, s32, s52, m[i], li, off);"),
    "vjp_mass_grad_sign": ("g += (li[0] * d[0] + li[1] * d[1] + li[2] * d[2]) / s32;",
                           "g -= (li[0] * d[0] + li[1] * d[1] + li[2] * d[2]) / s32;"),
    "adjoint_wrong_point": ("oracle_vjp(n, x0, m, lamv, eps, G, jt, gt);", "oracle_vjp(n, x1, m, lamv, eps, G, jt, gt);"),
    "adjoint_drift_weight": ("lamv[k] += dt * lamx[k];", "lamv[k] += h * lamx[k];"),
    "diffusion_axis_swap": ("const double ce = kappa * dt / (dx * dx), cw = ce;",
                            "const double ce = kappa * dt / (dy * dy), cw = ce;"),
    "diffusion_reflect": ("im = i > 0 ? i - 1 : 0;", "im = i > 0 ? i - 1 : (nx > 1 ? 1 : 0);"),
    "diffusion_centre": ("const double cc = 1.0 - (ce + cw + cn + cs + ct + cb);",
                         "const double cc = 1.0 - (ce + cw + cn + cs + ct);"),
}


def _build(src_text, out):
    cflags = ["-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
              "-fPIC", "-shared", "-w"]
    with tempfile.NamedTemporaryFile("w", suffix=".c", delete=False) as f:
        f.write(src_text)
        path = f.name
    try:
        subprocess.run(["gcc", *cflags, path, "-o", out, "-lm"], check=True)
    finally:
        os.unlink(path)


def _run_pins(lib):
    env = dict(os.environ, NBODY_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not slow", *PIN_TESTS], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    return r.returncode


@pytest.mark.slow
def test_every_mutant_is_caught(tmp_path):
    src = open(SRC).read()
    libs = {"original": str(tmp_path / "original.so")}
    _build(src, libs["original"])
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, name
        libs[name] = str(tmp_path / (name + ".so"))
        _build(src.replace(old, new), libs[name])
    with ThreadPoolExecutor(max_workers=4) as pool:
        codes = dict(zip(libs, pool.map(_run_pins, libs.values())))
    assert codes.pop("original") == 0
    survivors = [k for k, c in codes.items() if c == 0]
    assert not survivors, "mutants not caught by the pins: %s" % survivors
