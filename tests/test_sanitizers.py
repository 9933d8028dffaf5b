"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

* The FP64 CPU oracle, every entry point, driven by tests/c/oracle_sanitized.c
  (gcc, -fsanitize=address,undefined, leak detection on).
* The library's host side -- argument validation, launch-shape and band
  planning, the host paths of every entry point -- built from the same
  sources with the sanitizers on the host pass only (hipcc -Xarch_host ...;
  GPU code is built as usual and never runs here), then driven by the C99
  ABI consumer (tests/c/abi_consumer.c) and by the band-plan replay
  (tests/c/band_plan_check.cpp), both built with clang's sanitizers so that
  one sanitizer runtime serves the whole process.

No GPU needed; a sanitizer report fails the test.
"""

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2411_18889_amd", "csrc")
INC = os.path.join(ROOT, "include")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-2000:], r.stderr[-4000:])
    return r


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_sanitized")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
          os.path.join(ROOT, "tests", "c", "oracle_sanitized.c"),
          os.path.join(ROOT, "oracle", "nbody_oracle.c"), "-o", exe, "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert r.stdout.strip() == "ok"


def test_library_host_side_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(hipcc) or not os.path.exists(clang):
        pytest.skip("no hipcc / clang")
    import ctypes
    import sys
    sys.path.insert(0, ROOT)
    from paper_2411_18889_amd import _lib
    from paper_2411_18889_amd.build import SOURCES
    # the consumer hands the library placeholder pointers in calls that must
    # stop in the validation or at the missing device: a host without a GPU
    buf = ctypes.create_string_buffer(128)
    if _lib.lib().nbody_device_info(buf, 128) != _lib.NB_ENODEV:
        pytest.skip("a GPU is present: the consumer's placeholder calls are for a host without one")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang",
             "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN_HOST, "-I", INC, "-I", CSRC]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        _run([hipcc, *flags, "-c", os.path.join(CSRC, src), "-o", obj], timeout=600)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    lib = str(tmp_path / "libnbody.so")
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
          "-Xarch_host", "-fsanitize=undefined", *objs, "-o", lib], timeout=600)
    exe = str(tmp_path / "abi_consumer")
    _run([clang, "-std=c99", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", INC, os.path.join(ROOT, "tests", "c", "abi_consumer.c"), "-L", str(tmp_path),
          "-lnbody", "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath-link,/opt/rocm/lib", "-o", exe],
         timeout=300)
    r = _run([exe], env=ENV, timeout=300)
    assert r.stdout.strip() == "ok"
    band = str(tmp_path / "band_plan_check")
    _run([hipcc, "-O1", "-g", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", *SAN_HOST,
          "-I", INC, "-I", CSRC, os.path.join(ROOT, "tests", "c", "band_plan_check.cpp"), "-o", band],
         timeout=600)
    r = _run([band], env=ENV, timeout=600)
    assert r.stdout.startswith("ok")
