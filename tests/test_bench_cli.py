"""bench.py runs on one GPU only and says so when asked for more."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_clock_sampler_stops_and_summarises():
    """The shader-clock sampler runs beside the timed steps: it must stop
    when the block ends and give {} where no clock file is readable."""
    sys.path.insert(0, ROOT)
    import time
    import bench
    with bench.ClockSampler(period=0.01) as c:
        time.sleep(0.05)
    assert not c._t.is_alive()
    s = c.summary()
    if s:
        assert s["sclk_mhz_min"] <= s["sclk_mhz_mean"] <= s["sclk_mhz_max"]
        assert s["samples"] >= 1
    c.samples = [2000.0, 2400.0]
    assert c.summary()["sclk_mhz_mean"] == 2200.0


def test_tuner_cli_help():
    r = subprocess.run([sys.executable, "-m", "paper_2411_18889_amd.tune", "--help"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0 and "--n" in r.stdout and "--prec" in r.stdout
