"""The band plan of the symmetric passes, checked on the host: a C++ program
built from the library's own header (tests/c/band_plan_check.cpp) replays
every band, work item, partial write and fold read the library would issue
for many layouts and workspace sizes, through the same inline functions the
kernels use, and checks that every particle gets each of its slots exactly
once and in slot order (so the banded sums are bitwise those of one launch),
and that every band stays inside its workspace. No GPU needed."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_band_plan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc")
    exe = str(tmp_path / "band_plan_check")
    r = subprocess.run([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                        "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_2411_18889_amd", "csrc"),
                        os.path.join(ROOT, "tests", "c", "band_plan_check.cpp"), "-o", exe],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok"), (r.stdout, r.stderr)
