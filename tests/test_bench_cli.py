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


def test_executed_work_counts():
    """The executed-work roofline: a symmetric pass evaluates each pair of
    different blocks once (for both ends) and the pairs inside a block from
    both ends, so twice the first count plus the second is n^2; the one-sided
    kernel evaluates n^2 pairs. The adjoint walk of an R-step rollout with
    checkpoints every K steps has one pass per step plus the entry pass, of
    which the entry and the reloaded states carry no force sums."""
    sys.path.insert(0, ROOT)
    import bench
    for n, b in ((1 << 20, 1024), (262144, 1024), (12289, 256), (16448, 512)):
        info = {"symmetric": 1, "block_particles": b}
        off, one = bench.pair_evaluations(n, info)
        assert 2 * off + one == float(n) * n
        full, tail = divmod(n, b)
        assert one == full * b * b + tail * tail
        assert bench.executed_flop("force", n, info) == 27 * off + 20 * one
        assert bench.executed_flop("adjoint", n, info, True) == 72 * off + 55 * one
        assert bench.executed_flop("adjoint", n, info, False) == 58 * off + 48 * one
    one_sided = {"symmetric": 0, "block_particles": 0}
    assert bench.pair_evaluations(1000, one_sided) == (0.0, 1e6)
    assert bench.executed_flop("adjoint", 1000, one_sided, False) == 55e6
    assert bench.adjoint_schedule(10, 20) == (9, 2)
    assert bench.adjoint_schedule(200, 20) == (190, 11)
    assert bench.adjoint_schedule(3, 1) == (0, 4)
