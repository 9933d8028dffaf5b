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
    # two samples are too few for a clock-scaled fraction; five are enough
    assert bench.frac_at_clock(0.5, c.summary()) is None
    c.samples = [2000.0] * 5
    assert bench.frac_at_clock(0.5, c.summary()) == 0.5 * 2400 / 2000
    assert bench.frac_at_clock(0.5, {}) is None


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


def _write_pmc(folder, counter, rows):
    """A rocprofv3 --pmc CSV with one row per (kernel name, value)."""
    import csv
    os.makedirs(folder, exist_ok=True)
    with open(os.path.join(folder, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (k, v) in enumerate(rows):
            w.writerow([i, k, counter, v])


def test_traffic_summary_from_counter_folders(tmp_path):
    """--traffic-from: FETCH_SIZE scaled by what a 1 GiB copy reads (here half
    of it, so x2), WRITE_SIZE by what it writes (x1), the pair kernel's and
    its fold kernel's dispatches summed and divided by the R + 1 passes."""
    import bench
    gib_kib = float(1 << 20)
    _write_pmc(tmp_path / "cf", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", gib_kib / 2)])
    _write_pmc(tmp_path / "cw", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", gib_kib)])
    k = "void nb::asym::adjoint_sym_kernel<4, 4, false>(nb::asym::ASymArgs)"
    f = "void nb::(anonymous namespace)::adjoint_sym_finish_kernel<false>(nb::ASymFinishArgs)"
    other = "void nb::(anonymous namespace)::pe_pairs_kernel<double, float>(double const*)"
    # R = 3: 4 passes of 2 bands each
    _write_pmc(tmp_path / "f", "FETCH_SIZE", [(k, 100.0)] * 8 + [(f, 50.0)] * 8 + [(other, 1e6)])
    _write_pmc(tmp_path / "w", "WRITE_SIZE", [(k, 30.0)] * 8 + [(f, 10.0)] * 8 + [(other, 1e6)])
    out = tmp_path / "traffic.json"
    args = bench.parse(["--rollout", "3", "--traffic-out", str(out), "--traffic-from",
                        str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                        str(tmp_path / "cw")])
    bench.traffic_summary(args)
    import json
    rec = json.loads(out.read_text())["adjoint_sym_kernel@scale-2^20"]
    assert rec["passes"] == 4 and rec["pair_kernel_dispatches"] == 8
    assert rec["fetch_bytes_per_pass"] == (8 * 100 + 8 * 50) * 1024 * 2.0 / 4
    assert rec["write_bytes_per_pass"] == (8 * 30 + 8 * 10) * 1024 * 1.0 / 4
    assert rec["bytes_per_launch"] == rec["fetch_bytes_per_pass"] + rec["write_bytes_per_pass"]
    assert rec["source_sha256"] == bench.kernel_source_hash("adjoint_sym_kernel")


def test_checkpoint_interval_rule():
    """rollout(..., ckpt_every="auto") and bench.py --ckpt-every auto: the
    smallest interval whose nsteps // K + 1 slots of 9 n values fit."""
    from paper_2411_18889_amd.autograd import checkpoint_interval
    n, e = 1 << 20, 8
    slot = 9 * n * e
    assert checkpoint_interval(10, n, e, 11 * slot) == 1       # every step fits
    assert checkpoint_interval(10, n, e, 11 * slot - 1) == 2   # 6 slots
    assert checkpoint_interval(10, n, e, 3 * slot) == 4        # 3 slots (10 // 4 + 1)
    assert checkpoint_interval(10, n, e, 2 * slot) == 6        # 2 slots (10 // 6 + 1)
    assert checkpoint_interval(10, n, e, 0) == 10              # none fits: one interval
    assert checkpoint_interval(0, n, e, slot) == 1
