"""Build libnbody.so (HIP, gfx950) in-tree.

Every translation unit is compiled by hipcc for gfx950 only, with packed FP32
instructions disabled (-Xclang -target-feature -Xclang -packed-fp32-ops; the
host pass warns that it does not know that feature, which is harmless), then
linked into paper_2411_18889_amd/libnbody.so next to this file.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnbody.so")
SOURCES = ["force.hip", "force_sym.hip", "adjoint.hip", "adjoint_sym.hip", "adjoint_sym_entry.hip",
           "integrate.hip", "diag.hip", "diffusion.hip", "nbody_api.hip", "noalloc.hip"]

# Per-file instruction-scheduler strategies of LLVM's AMDGPU backend, each
# measured against the default on MI355X (the figures are in the files'
# headers): the force-free symmetric adjoint kernels with the memory-clause
# strategy, which interleaves the sinks of a lane (5 % faster at 2^20); the
# symmetric force kernels with the iterative ILP strategy (1-1.5 % faster).
FILE_FLAGS = {"adjoint_sym_entry.hip": ["-mllvm", "-amdgpu-sched-strategy=max-memory-clause"],
              "force_sym.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]}

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

CXXFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CXXFLAGS, *FILE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the device-only feature; drop that note
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, err))
    if err.strip() and verbose:
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libnbody.so. Always rebuilds."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = min(len(SOURCES), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        objs = list(pool.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
