"""Throughput of the N-body hot path on one MI355X.

One step = one forward + adjoint pass over a rollout of R KDK steps of the
scale-2^20 workload (N = 1,048,576 equal-mass Plummer sphere, eps = 2^-10,
dt = 2^-11, FP32 pair arithmetic with tile-compensated FP64 sums, FP64
positions and drift; R = 10 by default):
  * FP64 energy / momentum diagnostics of the initial state;
  * the forward rollout: a(x_0), then R KDK steps (R+1 force evaluations),
    with the state (x, v, a) checkpointed every K steps -- by default every
    step, when the checkpoints fit in a quarter of the free HBM (0.8 GB at
    2^20 for R = 10);
  * FP64 diagnostics of the final state;
  * the adjoint walk back over the R steps from the final state (R+1 fused
    adjoint pair passes; a state the forward pass checkpointed is reloaded,
    any other is walked back, its force recomputed in the pass).
Inputs are resident in HBM before timing starts. `value` counts pair
interactions of the force and adjoint kernels, N^2 per pass, per second of
the whole step. Per-kernel device times come from the library's own HIP
events around each launch over the timed steps (nbody_profile_*).

Printed: one JSON line (the last line of stdout).
"""

from __future__ import annotations

import argparse
import json
import ctypes
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3e12      # MI355X published FP32 vector peak
PEAK_CLOCK_MHZ = 2400.0          # the shader clock the published peaks assume

# The paper's convention: flop per interaction (i, j), counted from the pair
# body of its listing -- 3 sub + 3 FMA + 3 mul + 3 FMA with FMA = 2, plus 2
# for the reciprocal square root -- and the same count for the fused adjoint
# body; N^2 interactions per pass.
FLOP_PER_INTERACTION_FORCE = 20
FLOP_PER_INTERACTION_ADJOINT = 55

# Executed flop per pair evaluation, counted from the kernels' pair bodies
# (FMA = 2, reciprocal square root = 2). A one-sided evaluation serves one
# sink; an off-diagonal evaluation of the symmetric passes serves both ends
# of the pair (the diagonal block items evaluate every pair from both ends,
# one-sided).
#   force, one-sided: 3 sub, 3 FMA (s), 3 mul (r^3 m_j), 3 FMA (sum) = 20
#   force, symmetric: + 1 mul (r^3 m_i) + 3 FMA (source side) = 27
#   adjoint, one-sided with the force sums: 55 (without them: 48)
#   adjoint, symmetric with the force sums: 72 (without them: 58): the one-
#     sided body + d.lam_i (5) - 2 for d.u from the two dots - 1 for the
#     factor -3 that comes with the masses + the source side (1 mul + 7 FMA
#     with the force sums, 4 FMA without)
EXEC_FLOP = {("force", False): 20, ("force", True): 27,
             ("adjoint", False, True): 55, ("adjoint", False, False): 48,
             ("adjoint", True, True): 72, ("adjoint", True, False): 58}


def pair_evaluations(n, info):
    """(off-diagonal, one-sided) pair evaluations of one pass over n
    particles in the pass `info` (nbody_pass_info): the symmetric passes
    evaluate each pair of different blocks once and the pairs inside a block
    from both ends; the one-sided kernel evaluates all n^2."""
    n = int(n)
    if not info["symmetric"]:
        return 0.0, float(n) * n
    b = int(info["block_particles"])
    full, tail = divmod(n, b)
    diag = float(full) * b * b + float(tail) * tail
    return (float(n) * n - diag) / 2.0, diag


def executed_flop(kind, n, info, force_sums=True):
    """Executed flop of one pass (kind "force" or "adjoint")."""
    off, one = pair_evaluations(n, info)
    if kind == "force":
        return off * EXEC_FLOP[("force", True)] + one * EXEC_FLOP[("force", False)]
    sym_f = EXEC_FLOP[("adjoint", True, force_sums)]
    # the one-sided adjoint kernel always carries the force sums; the
    # diagonal items of the symmetric one only when asked for
    one_f = EXEC_FLOP[("adjoint", False, force_sums if info["symmetric"] else True)]
    return off * sym_f + one * one_f


def checkpoint_interval(arg, R, n, pos_bytes):
    """The rollout's checkpoint interval: `arg` if it is an integer, else
    (auto) the smallest K >= 1 whose R // K + 1 slots of 9 n position-type
    values fit in a quarter of the free device memory (the rule of
    rollout(..., ckpt_every="auto"))."""
    if str(arg) != "auto":
        return max(1, int(arg))
    import torch
    from paper_2411_18889_amd.autograd import checkpoint_interval as fit
    free, _ = torch.cuda.mem_get_info()
    return fit(R, n, pos_bytes, free // 4)


def adjoint_schedule(R, K):
    """(passes with the force sums, passes without) of the reverse walk of an
    R-step rollout checkpointed every K steps, started with the entry-half
    update at step R: the entry pass and the passes at reloaded (checkpoint)
    states need no force sums, every walked-back state does."""
    anchors = sum(1 for s in range(R) if s % K == 0)
    return R - anchors, 1 + anchors


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="scale-2^20")
    ap.add_argument("--rollout", type=int, default=10, help="KDK steps per forward+adjoint pass")
    ap.add_argument("--ckpt-every", default="auto",
                    help="checkpoint interval of the rollout: an integer >= 1, or 'auto' (the "
                         "default): every step when the checkpoints (72 bytes per particle per "
                         "stored step in the mixed policies) fit in a quarter of the free device "
                         "memory, so that the reverse walk reloads every state the forward pass "
                         "computed instead of recomputing its force; else the smallest interval "
                         "that fits")
    ap.add_argument("--prec", default="mix_tilec")
    ap.add_argument("--cpu-sample", type=int, default=32768,
                    help="sinks in the CPU-oracle baseline sample (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run one plain device-to-device copy of this many MiB (to "
                         "calibrate the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                         "COPY_WRITE_DIR"),
                    help="no GPU: turn four rocprofv3 --pmc output folders (FETCH_SIZE and "
                         "WRITE_SIZE of a run of this benchmark with --rollout R, and of "
                         "--copy-probe-mib 1024) into profiles/hbm_traffic.json")
    ap.add_argument("--traffic-out", default=os.path.join(ROOT, "profiles", "hbm_traffic.json"),
                    help="the summary --traffic-from writes (entries of other workloads kept)")
    return ap.parse_args(argv)


CSRC = os.path.join(ROOT, "paper_2411_18889_amd", "csrc")
KERNEL_SOURCES = {"force_kernel": ["common.h", "force.hip"],
                  "force_sym_kernel": ["common.h", "force_sym.hip"],
                  "adjoint_kernel": ["common.h", "adjoint.hip"],
                  "adjoint_sym_kernel": ["common.h", "adjoint_sym.hip", "adjoint_sym_pairs.h",
                                         "adjoint_sym_entry.hip"],
                  "diffusion_kernel4": ["common.h", "diffusion.hip"]}


def gpu_clocks():
    """Current shader clock (MHz) and power cap (W) of the first AMD GPU from
    sysfs, best effort: {} when the files are not readable."""
    import glob
    out = {}
    for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
        try:
            with open(dev + "/vendor") as fh:
                if fh.read().strip() != "0x1002":
                    continue
            with open(dev + "/pp_dpm_sclk") as fh:
                cur = [ln for ln in fh.read().splitlines() if ln.strip().endswith("*")]
            if cur:
                out["sclk_mhz"] = float(cur[0].split(":")[1].strip().rstrip("*").strip().lower().rstrip("mhz"))
            caps = glob.glob(dev + "/hwmon/hwmon*/power1_cap")
            if caps:
                with open(caps[0]) as fh:
                    out["power_cap_w"] = int(fh.read().strip()) / 1e6
        except (OSError, ValueError, IndexError):
            continue
        if out:
            break
    return out


class ClockSampler:
    """Samples the shader clock (sysfs pp_dpm_sclk, current level) every
    `period` seconds on a host thread while the timed steps run; the peak
    figures assume 2.4 GHz, and the clock under a sustained load sits below
    it when the power cap binds."""

    def __init__(self, period=0.1):
        import threading
        self.period, self.samples = period, []
        self._stop = threading.Event()
        self._t = threading.Thread(target=self._run, daemon=True)

    def _run(self):
        while not self._stop.is_set():
            c = gpu_clocks().get("sclk_mhz")
            if c:
                self.samples.append(c)
            self._stop.wait(self.period)

    def __enter__(self):
        self._t.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        self._t.join()

    def summary(self):
        if not self.samples:
            return {}
        v = self.samples
        return {"sclk_mhz_mean": sum(v) / len(v), "sclk_mhz_min": min(v), "sclk_mhz_max": max(v),
                "samples": len(v), "source": "sysfs pp_dpm_sclk, every %.1f s" % self.period}


# the clock-scaled fractions need the clock under load: at least this many
# samples (half a second of timed work at the default period); a short timed
# region may catch only the ramp from idle
MIN_CLOCK_SAMPLES = 5


def frac_at_clock(frac, clk):
    """`frac` against the peak scaled to the mean measured shader clock, or
    None when the sampler has too few samples for a clock under load."""
    if not clk or clk.get("samples", 0) < MIN_CLOCK_SAMPLES:
        return None
    return frac * PEAK_CLOCK_MHZ / clk["sclk_mhz_mean"]


def kernel_source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def hbm_traffic(kernel, workload):
    """Scaled FETCH_SIZE + WRITE_SIZE bytes per launch of `kernel` on
    `workload`, from the committed counter summary, or None when there is none
    or the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)["%s@%s" % (kernel, workload)]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash(kernel):
        return None
    return rec["bytes_per_launch"]


HBM_PEAK = 8.0e12                # MI355X HBM3E bandwidth, bytes/s
DIFF_BYTES_PER_POINT = 8         # algorithmic: read f once, write fn once (FP32)
DIFF_FLOP_PER_POINT = 13         # 7 multiplications + 6 additions per point


def bench_diffusion(args):
    """The 3-D diffusion stencil on an n^3 FP32 grid (workload diffusion-<n>):
    one step = one explicit update of every point (ping-pong buffers)."""
    import numpy as np
    import torch

    import paper_2411_18889_amd as nb
    from paper_2411_18889_amd import _lib

    n = int(args.workload.split("-")[1])
    dev = torch.device("cuda:0")
    print("device:", nb.device_info(), flush=True)
    rng = np.random.Generator(np.random.PCG64(7))
    f0 = rng.uniform(0.0, 1.0, size=(n, n, n)).astype(np.float32)
    prm = dict(dx=1.0, dy=1.0, dz=1.0, dt=0.1, kappa=1.0)
    a = torch.tensor(f0, device=dev)
    b = torch.empty_like(a)
    for _ in range(max(1, args.warmup)):
        nb.api.diffusion3d_step(a, out=b, **prm)
    torch.cuda.synchronize()
    steps = max(1, args.steps) * 50
    L = _lib.lib()
    prof = _lib.nb_profile_t()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    _lib.check(L.nbody_profile_begin(), "nbody_profile_begin")
    e0.record(stream)
    src, dst = a, b
    for _ in range(steps):
        nb.api.diffusion3d_step(src, out=dst, **prm)
        src, dst = dst, src
    e1.record(stream)
    torch.cuda.synchronize()
    _lib.check(L.nbody_profile_end(ctypes.byref(prof)), "nbody_profile_end")
    ms = e0.elapsed_time(e1) / steps
    k_ms = prof.ms[2] / max(1, prof.calls[2])
    pts = float(n) ** 3
    cpu = None
    if args.cpu_sample > 0:
        import oracle
        tc = time.time()
        oracle.diffusion3d(f0.astype(np.float64), **prm)
        tcpu = time.time() - tc
        cpu = {"value": pts / tcpu / 1e9, "unit": "Gpoints/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": "one full FP64 step of the %d^3 grid (%.2f s)" % (n, tcpu)}
    out = {
        "metric": "3-D diffusion stencil throughput (points updated per second)",
        "value": pts / (ms * 1e-3) / 1e9,
        "unit": "Gpoints/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded uniform field",
        "config": {"workload": args.workload, "grid": [n, n, n], **prm},
        "roofline": {"kernel": "diffusion_kernel4", "bound": "hbm",
                     "achieved": DIFF_BYTES_PER_POINT * pts / (k_ms * 1e-3) / 1e9,
                     "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": DIFF_BYTES_PER_POINT * pts / (k_ms * 1e-3) / HBM_PEAK,
                     "traffic": hbm_traffic("diffusion_kernel4", args.workload),
                     "bytes_per_point": DIFF_BYTES_PER_POINT, "avg_launch_ms": k_ms},
        "gflops": DIFF_FLOP_PER_POINT * pts / (ms * 1e-3) / 1e9,
        "paper_convention_GBps": 32 * pts / (ms * 1e-3) / 1e9,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# kernel families whose HBM traffic is summarised: the pair kernel and its
# fold (finishing) kernel, per pass
TRAFFIC_KERNELS = {"force_sym_kernel": ("force_sym_kernel", "force_sym_finish_kernel"),
                   "adjoint_sym_kernel": ("adjoint_sym_kernel", "adjoint_sym_finish_kernel"),
                   "force_kernel": ("force_kernel", "force_reduce_kernel"),
                   "adjoint_kernel": ("adjoint_kernel", "adjoint_reduce_kernel"),
                   "diffusion_kernel4": ("diffusion_kernel4",)}


def _kernel_base(name):
    """The bare function name of a (demangled) kernel name: 'void
    nb::(anonymous namespace)::adjoint_sym_kernel<8, 2, true>(...)' ->
    'adjoint_sym_kernel'."""
    import re
    name = re.sub(r"^void\s+", "", name.strip()).replace("(anonymous namespace)::", "")
    head = re.split(r"[<(]", name, maxsplit=1)[0]
    return head.split("::")[-1].strip()


def _pmc_rows(folder, counter):
    """(kernel name, value) of every dispatch in a rocprofv3 --pmc CSV output
    folder for one counter."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") == counter:
                    rows.append((r["Kernel_Name"], float(r["Counter_Value"])))
    if not rows:
        raise SystemExit("no %s rows under %s" % (counter, folder))
    return rows


def traffic_summary(args):
    """profiles/hbm_traffic.json from FETCH_SIZE / WRITE_SIZE runs (KiB per
    dispatch), each scaled by what the same counter reads for a plain copy of
    known size; bytes per pass = the pair kernel's and its fold kernel's
    dispatches of the run over the passes of the run (R + 1 of each kind)."""
    fetch_dir, write_dir, cfetch_dir, cwrite_dir = args.traffic_from
    copy_bytes = 1 << 30
    def copy_kib(folder, counter):
        vals = [v for k, v in _pmc_rows(folder, counter) if "copy" in k.lower() or "elementwise" in k]
        return max(vals)
    f_factor = copy_bytes / (copy_kib(cfetch_dir, "FETCH_SIZE") * 1024.0)   # bytes read per KiB counted
    w_factor = copy_bytes / (copy_kib(cwrite_dir, "WRITE_SIZE") * 1024.0)
    fetch, write = _pmc_rows(fetch_dir, "FETCH_SIZE"), _pmc_rows(write_dir, "WRITE_SIZE")
    passes = args.rollout + 1
    out = {"_note": "HBM-side bytes per pass = (FETCH_SIZE KiB x 1024 x %.3f + WRITE_SIZE KiB x "
                    "1024 x %.3f) summed over the pair kernel's and its fold kernel's dispatches "
                    "of the profiled benchmark step, over the passes of that step (each entry's "
                    "'passes': R + 1 for a step with --rollout R; the stencil: per dispatch); "
                    "factors from a plain 1 GiB device copy (the bytes it moves over the "
                    "counters' reading); regenerate when the kernel's sources change"
                    % (f_factor, w_factor),
           "commands": ["cd /tmp && export TMPDIR=/tmp; from the repository root, one counter C "
                        "per run, C in FETCH_SIZE WRITE_SIZE, each run into a folder of its own "
                        "(the folders of each entry are in its 'counter_folders'):",
                        "rocprofv3 --pmc C -d <folder> -o bench --output-format csv -- "
                        "python3 bench.py --steps 1 --warmup 0 --rollout R --cpu-sample 0",
                        "rocprofv3 --pmc C -d <folder> -o diff --output-format csv -- "
                        "python3 bench.py --workload diffusion-512 --steps 1 --warmup 1 --cpu-sample 0",
                        "rocprofv3 --pmc C -d <folder> -o copy --output-format csv -- "
                        "python3 bench.py --copy-probe-mib 1024",
                        "python3 bench.py [--workload W] --rollout R --traffic-from <FETCH_SIZE folder> "
                        "<WRITE_SIZE folder> <copy FETCH_SIZE folder> <copy WRITE_SIZE folder>"]}
    for fam, names in TRAFFIC_KERNELS.items():
        fk = sum(v for k, v in fetch if _kernel_base(k) in names)
        wk = sum(v for k, v in write if _kernel_base(k) in names)
        nd = sum(1 for k, _ in fetch if _kernel_base(k) == fam)
        if nd == 0:
            continue
        if fam == "diffusion_kernel4":
            passes = nd
        out["%s@%s" % (fam, args.workload)] = {
            "source_sha256": kernel_source_hash(fam),
            "bytes_per_launch": (fk * 1024.0 * f_factor + wk * 1024.0 * w_factor) / passes,
            "fetch_bytes_per_pass": fk * 1024.0 * f_factor / passes,
            "write_bytes_per_pass": wk * 1024.0 * w_factor / passes,
            "pair_kernel_dispatches": nd, "passes": passes,
            "counter_folders": list(args.traffic_from),
            **({} if fam == "diffusion_kernel4" else {"rollout": args.rollout})}
    path = args.traffic_out
    old = {}
    if os.path.exists(path):
        with open(path) as fh:
            old = json.load(fh)
    for k, v in old.items():  # keep the entries of other workloads
        if "@" in k and k not in out and not k.endswith("@" + args.workload):
            out[k] = v
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: v for k, v in out.items() if "@" in k}, indent=1))


def copy_probe(mib):
    import torch
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.traffic_from:
        traffic_summary(args)
        return
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return
    if args.workload.startswith("diffusion-"):
        bench_diffusion(args)
        return

    import numpy as np
    import torch

    import paper_2411_18889_amd as nb
    from nbody_inputs import WORKLOADS, make_state, random_unit_vectors
    from paper_2411_18889_amd import _lib

    w = WORKLOADS[args.workload]
    prec, R = args.prec, args.rollout
    dev = torch.device("cuda:0")
    print("device:", nb.device_info(), flush=True)
    t0 = time.time()
    x0, v0, m0 = make_state(w)
    n = x0.shape[1]
    pdt, mdt = nb.pos_dtype(prec), nb.mass_dtype(prec)
    K = checkpoint_interval(args.ckpt_every, R, n, torch.tensor([], dtype=pdt).element_size())
    X0 = torch.tensor(x0, dtype=pdt, device=dev)
    V0 = torch.tensor(v0, dtype=pdt, device=dev)
    M = torch.tensor(m0, dtype=mdt, device=dev)
    lam0 = torch.tensor(random_unit_vectors((3, n), 99), dtype=pdt, device=dev)
    x, v, acc = torch.empty_like(X0), torch.empty_like(X0), torch.empty_like(X0)
    lx, lv = torch.empty_like(X0), torch.empty_like(X0)
    lm = torch.empty(n, dtype=torch.float64, device=dev)
    ckpt = torch.empty((R // K + 1, 9 * n), dtype=pdt, device=dev)
    d0, d1 = (torch.empty(13, dtype=torch.float64, device=dev) for _ in range(2))
    print("inputs ready: N=%d (%.1f s)" % (n, time.time() - t0), flush=True)

    L = _lib.lib()
    prof = _lib.nb_profile_t()

    stream = torch.cuda.current_stream()
    pass_events = []

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    step_events = []

    def one_step():
        s0 = ev()
        x.copy_(X0)
        v.copy_(V0)
        nb.diag(x, v, M, w.eps, prec=prec, out=d0)
        e0 = ev()
        nb.step(x, v, M, acc, w.eps, w.dt, R, prec=prec, ckpt=ckpt, ckpt_every=K)
        e1 = ev()
        nb.diag(x, v, M, w.eps, prec=prec, out=d1)
        lx.copy_(lam0)
        lv.zero_()
        lm.zero_()
        e2 = ev()
        nb.step_adjoint(x, v, M, acc, lx, lv, lm, w.eps, w.dt, R, prec=prec, entry_half=True,
                        ckpt=ckpt, ckpt_every=K, step_end=R)
        e3 = ev()
        pass_events.append((e0, e1, e2, e3))
        step_events.append((s0, e3))

    for i in range(args.warmup):
        one_step()
        torch.cuda.synchronize()
        print("warmup step %d done" % i, flush=True)

    pass_events.clear()
    step_events.clear()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    _lib.check(L.nbody_profile_begin(), "nbody_profile_begin")
    with ClockSampler() as clocks:
        ev0.record(stream)
        wall0 = time.time()
        for i in range(args.steps):
            one_step()
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.time() - wall0
    _lib.check(L.nbody_profile_end(ctypes.byref(prof)), "nbody_profile_end")
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    print("timed %d steps: %.1f ms/step (wall %.1f s)" % (args.steps, ms_step, wall), flush=True)

    step_ms = sorted(a.elapsed_time(b) for a, b in step_events)
    passes_fwd, passes_adj = R + 1, R + 1
    interactions = float(n) * n * (passes_fwd + passes_adj)
    value = interactions / (ms_step * 1e-3) / 1e9

    f_ms = prof.ms[0] / max(1, prof.calls[0])
    a_ms = prof.ms[1] / max(1, prof.calls[1])
    kinds = ["force", "adjoint", "update", "diag", "copy"]
    per_kind = {k: {"ms_per_step": prof.ms[i] / args.steps, "calls": int(prof.calls[i])}
                for i, k in enumerate(kinds)}
    fwd_ms = sum(a.elapsed_time(b) for a, b, _, _ in pass_events) / len(pass_events)
    adj_ms = sum(c.elapsed_time(d) for _, _, c, d in pass_events) / len(pass_events)
    # the passes the library runs here (the symmetric kernels evaluate each
    # pair of different blocks once, for both ends)
    fpass, apass = nb.pass_info(1, n, prec), nb.pass_info(2, n, prec)
    fk = "force_sym_kernel" if fpass["symmetric"] else "force_kernel"
    ak = "adjoint_sym_kernel" if apass["symmetric"] else "adjoint_kernel"
    # executed work per launch: the force pass is the same every time; the
    # adjoint passes of one walk carry the force sums or not (entry and
    # reloaded states), averaged over the walk
    nF, nNoF = adjoint_schedule(R, K)
    f_flop = executed_flop("force", n, fpass)
    a_flop = (nF * executed_flop("adjoint", n, apass, True)
              + nNoF * executed_flop("adjoint", n, apass, False)) / (nF + nNoF)
    f_off, f_one = pair_evaluations(n, fpass)
    a_off, a_one = pair_evaluations(n, apass)
    peak_tf = FP32_VECTOR_PEAK / 1e12

    def roofline(kernel, info, flop, ms, conv_flop, off, one, what, partials=0.0):
        tf = flop / (ms * 1e-3) / 1e12
        conv_tf = conv_flop * float(n) * n / (ms * 1e-3) / 1e12
        r = {"kernel": kernel + what, "bound": "alu", "achieved": tf, "peak": peak_tf,
             "unit": "TFLOP/s", "frac": tf / peak_tf,
             "traffic": hbm_traffic(kernel, w.name),
             "executed_flop_per_launch": flop,
             "pair_evaluations_per_launch": off + one,
             "pair_evaluations_both_ends": off, "pair_evaluations_one_sided": one,
             "shape": info, "avg_launch_ms": ms,
             "ginteractions_per_s": float(n) * n / (ms * 1e-3) / 1e9,
             "paper_convention": {"flop_per_interaction": conv_flop,
                                  "interactions_per_launch": float(n) * n,
                                  "achieved": conv_tf, "frac": conv_tf / peak_tf}}
        if info["symmetric"]:
            # the FP32 partials per particle, quantity and block that the pass
            # writes and its fold kernels read back: the price of a fixed-
            # order reduction without atomics (the workspace holds one band
            # of them at a time)
            r["partials_bytes_per_launch"] = partials
            if r["traffic"] is not None:
                r["traffic_rate_tb_s"] = r["traffic"] / (ms * 1e-3) / 1e12
        return r

    def partials(info, nq):  # FP32 partials of one symmetric pass
        if not info["symmetric"]:
            return 0.0
        b = int(info["block_particles"])
        return float((n + b - 1) // b) * nq * n * 4

    # the paper-style count of the adjoint: 55 flop per interaction for a
    # pass that also sums the force, 48 (the one-sided count without the
    # force sums) for one that reloads it, averaged over the walk
    conv_adj = (nF * FLOP_PER_INTERACTION_ADJOINT
                + nNoF * EXEC_FLOP[("adjoint", False, False)]) / (nF + nNoF)
    roof_adj = roofline(ak, apass, a_flop, a_ms, conv_adj, a_off, a_one,
                        " (fused J^T lam + G^T lam; the force sums in %d of %d passes)"
                        % (nF, nF + nNoF),
                        (nF * partials(apass, 7) + nNoF * partials(apass, 4)) / (nF + nNoF))
    roof_adj["passes_with_force_sums"], roof_adj["passes_without"] = nF, nNoF
    force_roof = roofline(fk, fpass, f_flop, f_ms, FLOP_PER_INTERACTION_FORCE, f_off, f_one, "",
                          partials(fpass, 3))
    dom = "adjoint" if prof.ms[1] >= prof.ms[0] else "force"
    roof = roof_adj if dom == "adjoint" else force_roof

    clk = clocks.summary()
    for r in (roof_adj, force_roof):
        # the same achieved rate against the peak scaled to the measured clock
        f = frac_at_clock(r["frac"], clk)
        if f is not None:
            r["frac_at_measured_sclk"] = f
    if clk and clk["samples"] < MIN_CLOCK_SAMPLES:
        clk["note"] = ("fewer than %d samples: too short a timed region for the clock under load"
                       % MIN_CLOCK_SAMPLES)

    D0 = nb.diag_dict(d0)
    D1 = nb.diag_dict(d1)
    dE = (D1["E"] - D0["E"]) / abs(D0["E"])

    cpu = None
    rel_err = None
    if args.cpu_sample > 0:
        import oracle
        # forward force of the initial state on the GPU, then the same sinks
        # one by one on the host cores
        xs = torch.tensor(x0, dtype=pdt, device=dev)
        a_gpu = nb.accel(xs, M, w.eps, prec=prec).cpu().numpy()
        xh, mh = xs.cpu().numpy().astype(np.float64), M.cpu().numpy().astype(np.float64)
        rng = np.random.default_rng(1234)
        idx = np.sort(rng.choice(n, size=min(args.cpu_sample, n), replace=False))
        tc = time.time()
        ref = oracle.accel_sampled(xh, mh, w.eps, idx)
        tcpu = time.time() - tc
        rel_err = float(np.linalg.norm(a_gpu[:, idx] - ref) / np.linalg.norm(ref))
        # the same oracle on one thread, over the first eighth of the sinks
        k0 = oracle.num_threads()
        idx1 = idx[: max(1, min(1024, len(idx) // 8))]
        oracle.set_num_threads(1)
        tc = time.time()
        oracle.accel_sampled(xh, mh, w.eps, idx1)
        t1 = time.time() - tc
        oracle.set_num_threads(k0)
        cpu = {"value": len(idx) * float(n) / tcpu / 1e9, "unit": "Ginteractions/s",
               "cores": k0, "kind": "oracle",
               "sample": "%d seeded sinks x all %d sources, FP64 force (%.1f s)"
                         % (len(idx), n, tcpu),
               "one_thread_value": len(idx1) * float(n) / t1 / 1e9,
               "one_thread_sample": "%d of the same sinks (%.1f s)" % (len(idx1), t1)}
        print("cpu oracle: %.3f Ginteractions/s on %d threads; GPU force rel err %.3g"
              % (cpu["value"], cpu["cores"], rel_err), flush=True)

    out = {
        "metric": "Ginteractions/s & % FP32 vector peak; adjoint/forward time at rel err ≤1e-5",
        "value": value,
        "unit": "Ginteractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "step_ms_best": step_ms[0],
        "step_ms_median": step_ms[len(step_ms) // 2],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec.startswith("mix") else prec,
        "precision": ("f32 pair arithmetic, f64 sums and state" if prec.startswith("mix")
                      else prec + " throughout"),
        "data": "synthetic: seeded Plummer sphere",
        "config": {"workload": w.name, "n": n, "eps": w.eps, "dt": w.dt, "rollout_steps": R,
                   "ckpt_every": K, "precision": prec,
                   "step": "diag + forward rollout (R+1 force passes) + diag + adjoint walk "
                           "(R+1 fused passes)"},
        "roofline": roof,
        ("force_kernel" if dom == "adjoint" else "adjoint_kernel"):
            force_roof if dom == "adjoint" else roof_adj,
        "forward_pass_ms": fwd_ms,
        "adjoint_pass_ms": adj_ms,
        "adjoint_over_forward": adj_ms / fwd_ms,
        "adjoint_over_forward_kernel": a_ms / f_ms,
        "force_rel_err_sampled": rel_err,
        "energy_drift": dE,
        "gpu_clocks_timed_region": clk,
        "gpu_clocks_after_run": gpu_clocks(),
        "per_kind": per_kind,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
