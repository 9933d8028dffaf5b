"""Per-workload report of the MI355X results: throughput, accuracy against
the FP64 oracle, energy drift, the adjoint's cost and gradient error, pass
times across N and the oracle's own CPU rate -- every figure of the result
tables, regenerated from committed code on one GPU.

    python tests/workload_report.py [--only NAME ...] [--skip-scan] [--skip-shard]
                                    [--skip-cpu]

Prints markdown on stdout (progress on stderr). Test infrastructure: it uses
the oracle (oracle/) for the reference values, as the GPU tests do.

Per workload and precision:
  * force pass: best of 5 `nbody_accel` calls of the set on itself, resident
    inputs, HIP events; Ginteractions/s = N^2 / time; % of the 157.3 TFLOP/s
    FP32 (78.6 FP64) vector peak from executed flop (pair evaluations x
    executed flop per evaluation) and, in brackets, by the paper's
    convention of 20 flop per interaction;
  * e_glob, per-particle p99 and max against the oracle on the same values:
    every sink up to 65536 particles, else 4096 seeded sinks plus the 128
    nearest the centre and (subcluster) the 128 nearest the subcluster's
    centre;
  * dE = (E_S - E_0) / |E_0| over the workload's steps (FP64 diagnostics),
    beside the same for an FP64 trajectory on the GPU (the subcluster and
    2^20 workloads) or for the oracle's own trajectory (1024: all steps;
    65536: the stored oracle energies);
  * adjoint-16384: forward rollout and backward times, gradient error
    against the stored oracle gradient.
"""

from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from nbody_inputs import WORKLOADS, make_state, plummer_sphere  # noqa: E402

FP32_PEAK, FP64_PEAK = 157.3e12, 78.6e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def timed(fn, reps=5):
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def errors(a, ref):
    e = float(np.linalg.norm(a - ref) / np.linalg.norm(ref))
    pe = np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)
    return e, float(np.quantile(pe, 0.99)), float(pe.max())


def sample(name, xs):
    from tests.gpu_util import cluster_centres, sample_indices
    n = xs.shape[1]
    if n <= 65536:
        return np.arange(n)
    return sample_indices(xs, 4096, 128, seed=7, centres=cluster_centres(name, xs))


def force_row(name, prec, x, v, m, w):
    import torch
    import paper_2411_18889_amd as nb
    from tests.gpu_util import host, to_dev
    bench = _bench()
    n = x.shape[1]
    xd, vd, md = to_dev(x, v, m, prec)
    info = nb.pass_info(1, n, prec)
    ms = timed(lambda: nb.accel(xd, md, w.eps, prec=prec))
    flop = bench.executed_flop("force", n, info)
    peak = FP64_PEAK if prec == "f64" else FP32_PEAK
    a = host(nb.accel(xd, md, w.eps, prec=prec))
    xs, ms_ = host(xd), host(md)
    idx = sample(name, xs)
    ref = oracle.accel_sampled(xs, ms_, w.eps, idx) if idx.size < n else oracle.accel(xs, ms_, w.eps)
    e, p99, mx = errors(a[:, idx], ref)
    # the workload's trajectory in this precision, FP64 diagnostics
    acc = torch.empty_like(xd)
    E0 = nb.diag_dict(nb.diag(xd, vd, md, w.eps, prec=prec))["E"]
    t0 = time.time()
    nb.step(xd, vd, md, acc, w.eps, w.dt, w.steps, prec=prec)
    torch.cuda.synchronize()
    t_steps = time.time() - t0
    E1 = nb.diag_dict(nb.diag(xd, vd, md, w.eps, prec=prec))["E"]
    return {"prec": prec, "pass": "symmetric %d" % info["block_particles"] if info["symmetric"]
            else "one-sided %dx%d/%d" % (info["i_per_lane"], info["block"], info["split"]),
            "ms": ms, "gint": n * n / ms / 1e6, "frac": flop / (ms * 1e-3) / peak,
            "frac_conv": 20.0 * n * n / (ms * 1e-3) / peak,
            "e": e, "p99": p99, "max": mx, "dE": (E1 - E0) / abs(E0), "steps_s": t_steps,
            "x_end": host(xd)}


def workload_rows(name):
    import torch
    import paper_2411_18889_amd as nb
    from tests.gpu_util import host, to_dev
    w = WORKLOADS[name]
    x, v, m = make_state(name)
    n = x.shape[1]
    rows = [force_row(name, p, x, v, m, w) for p in w.precisions]
    ref = ""
    if name == "fp64-1024":
        xo, vo, _ = oracle.kdk(x, v, m, w.eps, w.dt, w.steps)
        D0, D1 = oracle.diag(x, v, m, w.eps), oracle.diag(xo, vo, m, w.eps)
        ref = "oracle %.6e; positions after %d steps within %.2g of the oracle's" % (
            (D1["E"] - D0["E"]) / abs(D0["E"]), w.steps,
            np.linalg.norm(rows[0]["x_end"] - xo) / np.linalg.norm(xo))
    elif name == "fp32-65536":
        e = np.loadtxt(os.path.join(ROOT, "tests", "golden", "energy_65536.txt"))
        ref = "oracle %.3e (stored FP64 run from the same FP32 state)" % ((e[-1, 1] - e[0, 1]) / abs(e[0, 1]))
    elif name in ("subcluster-262144", "scale-2^20"):
        xd, vd, md = to_dev(x, v, m, "f64")
        acc = torch.empty_like(xd)
        E0 = nb.diag_dict(nb.diag(xd, vd, md, w.eps, prec="f64"))["E"]
        nb.step(xd, vd, md, acc, w.eps, w.dt, w.steps, prec="f64")
        E1 = nb.diag_dict(nb.diag(xd, vd, md, w.eps, prec="f64"))["E"]
        xs = host(xd)
        idx = sample(name, xs)[:512]
        e64 = float(np.linalg.norm(host(acc)[:, idx] - oracle.accel_sampled(xs, host(md), w.eps, idx))
                    / np.linalg.norm(oracle.accel_sampled(xs, host(md), w.eps, idx)))
        x64 = xs
        ref = "GPU FP64 trajectory %.4e (its force at step %d within %.1g of the oracle, 512 sinks)" % (
            (E1 - E0) / abs(E0), w.steps, e64)
        for r in rows:
            r["dx"] = float(np.linalg.norm(r["x_end"] - x64) / np.linalg.norm(x64 - x))
    return w, n, rows, ref


def adjoint_row():
    import torch
    import paper_2411_18889_amd as nb
    from tests.gpu_util import host, rel, to_dev
    w = WORKLOADS["adjoint-16384"]
    g = np.load(os.path.join(ROOT, "tests", "golden", "adjoint_16384.npz"))
    x, v, m = make_state(w)
    best = None
    for _ in range(3):
        xd, vd, md = to_dev(x, v, m, "mix_tilec")
        for t in (xd, vd, md):
            t.requires_grad_(True)
        y = torch.tensor(g["y"], device=xd.device)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        xs, _ = nb.rollout(xd, vd, md, w.eps, w.dt, w.steps, ckpt_every=w.ckpt_every, prec="mix_tilec")
        loss = ((xs - y) ** 2).sum() / x.shape[1]
        e[1].record()
        loss.backward()
        e[2].record()
        torch.cuda.synchronize()
        f, b = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
        if best is None or f + b < best[0] + best[1]:
            errs = [rel(host(t.grad), g["g" + k]) for k, t in (("x", xd), ("v", vd), ("m", md))]
            best = (f, b, errs)
    return best


def timed_batch(fn, inner, groups=3):
    """Best over `groups` of the mean time of `inner` back-to-back calls
    between one pair of HIP events (ms per call): launch gaps amortised."""
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(groups):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(inner):
            fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / inner)
    return best


def pass_scan():
    """Force and adjoint-step times across N, library shapes."""
    import torch
    import paper_2411_18889_amd as nb
    bench = _bench()
    out = []
    for n in (1024, 4096, 16384, 65536, 262144, 1 << 20, 1 << 21):
        x, v, m = plummer_sphere(n, 3)
        row = {"n": n}
        inner = 50 if n <= 16384 else (10 if n <= 65536 else (3 if n <= 262144 else 1))
        for prec in ("mix_tilec", "f32", "f64"):
            if prec == "f64" and n > (1 << 20):
                continue
            log("scan n=%d %s" % (n, prec))
            pdt, mdt = nb.pos_dtype(prec), nb.mass_dtype(prec)
            X = torch.tensor(x, dtype=pdt, device="cuda")
            V = torch.tensor(v, dtype=pdt, device="cuda")
            M = torch.tensor(m, dtype=mdt, device="cuda")
            eps = 2.0 ** -9
            ws = torch.empty(max(1, nb.workspace_size(0, n, prec)), dtype=torch.uint8, device="cuda")
            out_a = torch.empty_like(X)
            ms = timed_batch(lambda: nb.accel(X, M, eps, prec=prec, out=out_a, workspace=ws), inner)
            info = nb.pass_info(1, n, prec)
            peak = FP64_PEAK if prec == "f64" else FP32_PEAK
            row["force_" + prec] = (ms, bench.executed_flop("force", n, info) / (ms * 1e-3) / peak)
            if prec == "mix_tilec":
                ms = timed_batch(lambda: nb.accel(X, M, eps, prec=prec, potential=True, out=out_a,
                                                  workspace=ws), inner)
                row["pot"] = (ms, None)
            if prec in ("mix_tilec", "f64"):
                # one reverse step (reverse drift + a fused pass with the force
                # sums) on resident state; the calls walk the same state back
                acc = nb.accel(X, M, eps, prec=prec)
                st = (X.clone(), V.clone(), acc, torch.zeros_like(X), torch.ones_like(X),
                      torch.zeros(n, dtype=torch.float64, device="cuda"))
                wsa = torch.empty(max(1, nb.workspace_size(2, n, prec)), dtype=torch.uint8,
                                  device="cuda")
                ms = timed_batch(lambda: nb.step_adjoint(st[0], st[1], M, st[2], st[3], st[4], st[5],
                                                         eps, 2.0 ** -16, 1, prec=prec, workspace=wsa),
                                 inner)
                ainfo = nb.pass_info(2, n, prec)
                row["adj_" + prec] = (ms, bench.executed_flop("adjoint", n, ainfo, True) / (ms * 1e-3) / peak)
                if prec == "mix_tilec":
                    # the entry pass of a walk (no force sums), the kind every
                    # pass of a walk over per-step checkpoints is
                    ms = timed_batch(lambda: nb.step_adjoint(st[0], st[1], M, st[2], st[3], st[4], st[5],
                                                             eps, 2.0 ** -16, 0, prec=prec,
                                                             entry_half=True, workspace=wsa), inner)
                    row["adj0"] = (ms, bench.executed_flop("adjoint", n, ainfo, False) / (ms * 1e-3) / peak)
        out.append(row)
    return out


def shard_rows(G=8):
    """One GPU's share of the scale-2^20 force pass sharded by sinks over G
    GPUs: `nbody_accel` of the first N/G particles against all N (the
    one-sided kernel, separate sink and source sets), beside the full
    symmetric pass of the set on itself; sampled error of the shard against
    the oracle (256 seeded sinks)."""
    import torch
    import paper_2411_18889_amd as nb
    from tests.gpu_util import host, to_dev
    w = WORKLOADS["scale-2^20"]
    x, v, m = make_state("scale-2^20")
    n = x.shape[1]
    ni = n // G
    out = []
    for prec in ("mix_tilec", "f32", "f64"):
        log("shard %s" % prec)
        xd, _, md = to_dev(x, v, m, prec)
        xi = xd[:, :ni].contiguous()
        ai = torch.empty_like(xi)
        L = nb._lib.lib()
        wsi = torch.empty(max(1, int(L.nbody_pass_workspace_size(0, ni, n, nb._lib.PREC[prec], 0, 0,
                                                                     None))),
                          dtype=torch.uint8, device="cuda")
        ws = torch.empty(max(1, nb.workspace_size(0, n, prec)), dtype=torch.uint8, device="cuda")
        ms = timed(lambda: nb.accel(xi, md, w.eps, prec=prec, xj=xd, out=ai, workspace=wsi))
        full = timed(lambda: nb.accel(xd, md, w.eps, prec=prec, workspace=ws), reps=3)
        a = host(nb.accel(xi, md, w.eps, prec=prec, xj=xd))
        idx = np.sort(np.random.default_rng(11).choice(ni, 256, replace=False))
        xs = host(xd)
        ref = oracle.accel_sampled(xs, host(md), w.eps, idx)
        e = float(np.linalg.norm(a[:, idx] - ref) / np.linalg.norm(ref))
        peak = FP64_PEAK if prec == "f64" else FP32_PEAK
        out.append({"prec": prec, "ni": ni, "n": n, "ms": ms, "full": full,
                    "gint": ni * float(n) / ms / 1e6,
                    "frac": 20.0 * ni * float(n) / (ms * 1e-3) / peak, "e": e})
    return out


def cpu_table():
    out = []
    k0 = oracle.num_threads()
    for n, sinks in ((1024, None), (16384, None), (65536, None), (262144, 512), (1 << 20, 256)):
        x, _, m = plummer_sphere(n, 3)
        row = {"n": n}
        for threads in (1, k0):
            oracle.set_num_threads(threads)
            s = sinks if sinks else (n if threads > 1 or n <= 16384 else 1024)
            idx = np.arange(s) * (n // s)
            t0 = time.time()
            oracle.accel_sampled(x, m, 2.0 ** -9, idx)
            row[threads] = (s * float(n) / (time.time() - t0) / 1e9, s)
        out.append(row)
    oracle.set_num_threads(k0)
    return out, k0


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--only", nargs="*", default=list(WORKLOADS))
    ap.add_argument("--skip-scan", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-shard", action="store_true")
    args = ap.parse_args()
    import paper_2411_18889_amd as nb
    print("Device: %s. Command: `python tests/workload_report.py%s`\n"
          % (nb.device_info(), "".join(" " + a for a in sys.argv[1:])))
    print("| workload | N | precision | pass | force pass | Ginteractions/s | % peak executed (20-flop convention) "
          "| e_glob | p99 | max | dE over the steps | reference dE | positions vs FP64 run |")
    print("|---|---:|---|---|---:|---:|---|---|---|---|---|---|---|")
    bench = _bench()

    def clock_line(clk):
        c = clk.summary()
        return ("\nMean shader clock while these were measured: %.0f MHz (%.0f-%.0f; the peaks assume "
                "2400)" % (c["sclk_mhz_mean"], c["sclk_mhz_min"], c["sclk_mhz_max"])) if c else ""

    with bench.ClockSampler() as clk:
        for name in args.only:
            if name == "adjoint-16384":
                continue
            log("workload", name)
            w, n, rows, ref = workload_rows(name)
            for r in rows:
                print("| %s | %d | %s | %s | %.4g ms | %.0f | %.1f %% (%.1f %%) | %.2g | %.2g | %.2g | %.4e | %s | %s |"
                      % (name, n, r["prec"], r["pass"], r["ms"], r["gint"], 100 * r["frac"],
                         100 * r["frac_conv"], r["e"], r["p99"], r["max"], r["dE"], ref,
                         "%.2g of the distance travelled" % r["dx"] if "dx" in r else "—"))
    print(clock_line(clk))
    if "adjoint-16384" in args.only:
        log("workload adjoint-16384")
        f, b, errs = adjoint_row()
        print("\nadjoint-16384 (200 steps, checkpoints every 20, mix_tilec): forward rollout %.1f ms, "
              "backward %.1f ms, backward / forward %.2f; gradient rel err against the oracle "
              "x0 %.2g, v0 %.2g, m %.2g" % (f, b, b / f, *errs))
    if not args.skip_scan:
        print("\nPass times across N (Plummer, eps = 2^-9; force = `nbody_accel` of the set on itself, "
              "adjoint step = one reverse step of `nbody_step_adjoint` (a pass with the force sums), "
              "adjoint entry pass = the entry pass of a walk (no force sums; every pass of a walk over "
              "per-step checkpoints is of this kind), resident inputs and workspace; "
              "best of 3 batches of 50 (up to 16384), 10, 3, then 1 back-to-back calls; "
              "ms per call, % of the FP32 (FP64) vector peak from executed flop)\n")
        print("| N | force tile-compensated | force + potential tile-compensated | adjoint step tile-compensated "
              "| adjoint entry pass tile-compensated | force FP32 | force FP64 | adjoint step FP64 |")
        print("|---:|---|---|---|---|---|---|---|")
        with bench.ClockSampler() as clk:
            scan = pass_scan()
        for r in scan:
            def cell(k):
                if k not in r:
                    return "—"
                ms, frac = r[k]
                g = "%.4g ms (%.0f G/s" % (ms, r["n"] ** 2 / ms / 1e6)
                return g + (", %.0f %%)" % (100 * frac) if frac is not None else ")")
            print("| %d | %s | %s | %s | %s | %s | %s | %s |" % (
                r["n"], cell("force_mix_tilec"), cell("pot"), cell("adj_mix_tilec"), cell("adj0"),
                cell("force_f32"), cell("force_f64"), cell("adj_f64")))
        print(clock_line(clk))
    if not args.skip_shard:
        print("\nOne GPU's share of the scale-2^20 force pass sharded by sinks over 8 GPUs "
              "(`nbody_accel` of N/8 sinks against all N sources, one-sided kernel; best of 5) "
              "beside the full symmetric pass on one GPU (best of 3)\n")
        print("| precision | sinks x sources | shard pass | Ginteractions/s | % peak (20-flop) "
              "| full pass, one GPU | full / 8 | e_glob (256 sinks) |")
        print("|---|---|---:|---:|---:|---:|---:|---:|")
        with bench.ClockSampler() as clk:
            shards = shard_rows()
        for r in shards:
            print("| %s | %d x %d | %.4g ms | %.0f | %.1f %% | %.4g ms | %.4g ms | %.2g |" % (
                r["prec"], r["ni"], r["n"], r["ms"], r["gint"], 100 * r["frac"], r["full"],
                r["full"] / 8, r["e"]))
        print(clock_line(clk))
    if not args.skip_cpu:
        rows, k0 = cpu_table()
        print("\nFP64 oracle (`oracle_accel`) on the host: Ginteractions/s (sampled sinks x all N)\n")
        print("| N | 1 thread | %d threads |" % k0)
        print("|---:|---|---|")
        for r in rows:
            print("| %d | %.3g (%d sinks) | %.3g (%d sinks) |" % (r["n"], r[1][0], r[1][1], r[k0][0], r[k0][1]))


if __name__ == "__main__":
    main()
