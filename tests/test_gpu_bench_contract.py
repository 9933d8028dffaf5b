"""bench.py's one-line JSON on small workloads: every field of the
benchmark contract is there, with consistent values (the roofline fraction
is achieved over peak; the CPU baseline is the oracle's)."""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    print("bench.py", " ".join(args), flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def _check_common(d):
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["value"] > 0 and d["ms_per_step"] > 0
    assert "workload" in d["config"]
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["bound"] in ("hbm", "mfma", "alu")
    assert abs(r["frac"] - r["achieved"] / r["peak"]) <= 1e-9 * max(1.0, r["frac"])


def test_bench_contract_nbody():
    d = _run("--workload", "adjoint-16384", "--steps", "1", "--warmup", "0", "--rollout", "2",
             "--cpu-sample", "256")
    _check_common(d)
    assert d["unit"] == "Ginteractions/s" and d["higher_is_better"] is True
    cb = d["cpu_baseline"]
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in cb, k
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1
    assert d["force_rel_err_sampled"] <= 1e-5


def test_bench_contract_diffusion():
    d = _run("--workload", "diffusion-256", "--steps", "2", "--warmup", "1", "--cpu-sample", "0")
    _check_common(d)
    assert d["roofline"]["bound"] == "hbm"
