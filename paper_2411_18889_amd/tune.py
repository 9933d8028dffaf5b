"""Launch-shape autotuner for the pair passes.

The paper picks the number of threads per block by a parameter survey on
each machine (section "N-body simulation", NTHREADS); this tool does the same
for every pair pass of the library, in the launch parameters of each:

* the force pass (``--op force``): the one-sided kernel's sinks per lane,
  workgroup size (= j-tile length) and j-split, through ``nbody_accel_ex``,
  and, for a policy that has it, the symmetric (third-law) pass's waves per
  workgroup and sinks per lane;
* the fused adjoint pass (``--op adjoint``): the same two families through
  ``nbody_step_adjoint_ex``, timed on one step of the reverse walk (a pass
  that also sums a(x), as every walked-back step does) or, with
  ``--adjoint-pass entry``, on the entry pass (no force sums, as every pass
  of a walk over per-step checkpoints).

For every (N, precision) it times each shape on a seeded Plummer sphere with
the workspace the library asks for that shape, checks that each shape
returns the same result as the library's own choice (shapes differ by
rounding only: to 1e-5 relative for the force, 1e-4 for the adjoint's
position adjoint, 1e-3 for it in the plain FP32 policy, 1e-12 in FP64),
and reports the fastest. The symmetric family is swept for the policies
that have it (tile-compensated, plain FP32, FP64).

    python -m paper_2411_18889_amd.tune --op force adjoint --n 65536 1048576

Prints one JSON line per (op, N, precision): the best shape, its time, the
library's current choice and its time, and the five fastest shapes.
"""

from __future__ import annotations

import argparse
import itertools
import json
import os
import sys

# shapes the library is built for (nb_launch in include/nbody.h)
SYM_PRECS = ("mix_tilec", "f32", "f64")  # the policies with symmetric passes
SYM_FORCE = [(2, 128), (2, 256), (2, 512), (2, 1024), (4, 128), (4, 256), (4, 512), (4, 1024),
             (8, 128), (8, 256), (8, 512)]
SYM_ADJOINT = [(2, 128), (2, 256), (2, 512), (2, 1024), (1, 256), (1, 512), (4, 128), (4, 256),
               (4, 512)]


def _time(fn, reps, reset=None):
    import torch
    if reset:
        reset()
    fn()
    torch.cuda.synchronize()
    total = 0.0
    for _ in range(reps):
        if reset:
            reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        total += e0.elapsed_time(e1)
    return total / reps


def _warm_up(fn, seconds=0.3, reset=None):
    import time
    import torch
    t0 = time.time()
    while time.time() - t0 < seconds:
        if reset:
            reset()
        fn()
        torch.cuda.synchronize()


def candidate_shapes(op, n, prec, sym_pass):
    """The shapes a full sweep times: one-sided (sinks per lane, block,
    split) and, where the policy has it, symmetric (sinks per lane, block)."""
    shapes = []
    splits = sorted({1, 2, 4, 8, 16, 32} | {max(1, min(256, (4096 * 64) // max(1, n)))})
    ipls, blocks = ((1, 2, 4), (64, 128, 256, 512, 1024)) if op == "force" else \
        ((1, 2), (64, 128, 256, 512))
    for ipl, block, split in itertools.product(ipls, blocks, splits):
        if split > 1 and n // split < block:
            continue
        waves = -(-n // (ipl * block)) * (block // 64) * split
        if split > 1 and waves > 131072:  # past ~128 waves per SIMD a split only adds partials
            continue
        shapes.append({"i_per_lane": ipl, "block": block, "split": split, "symmetric": 0})
    if sym_pass:
        for ipl, block in (SYM_FORCE if op == "force" else SYM_ADJOINT):
            if op != "force" and prec == "f64" and block > 512:
                continue  # the FP64 adjoint: up to 8 waves (16 would spill)
            if block * ipl <= n:
                shapes.append({"i_per_lane": ipl, "block": block, "split": 0, "symmetric": 1})
    return shapes


def tune(n, prec, op="force", eps=2.0 ** -8, shapes=None, reps=None, seed=5, one_sided=True,
         adjoint_pass="walk"):
    """Times every shape (or `shapes`, a list of nb_launch dicts or of
    (i_per_lane, block, split) one-sided triples) of the `op` pass at n.
    one_sided=False leaves the one-sided family out of the default sweep.
    adjoint_pass: "walk" (a walked-back step, the pass with the force sums)
    or "entry" (the entry pass, without them, as every pass of a walk over
    a state checkpointed at every step)."""
    import numpy as np
    import torch

    from . import api
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from nbody_inputs import plummer_sphere

    x, v, m = plummer_sphere(n, seed)
    dev = torch.device("cuda:0")
    pdt = api.pos_dtype(prec)
    X = torch.tensor(x, dtype=pdt, device=dev)
    V = torch.tensor(v, dtype=pdt, device=dev)
    M = torch.tensor(m, dtype=api.mass_dtype(prec), device=dev)
    sym_pass = prec in SYM_PRECS
    if reps is None:
        reps = max(2, min(200, int(2e11 // (n * n))))
    if shapes is None:
        shapes = candidate_shapes(op, n, prec, sym_pass)
        if not one_sided:
            shapes = [s for s in shapes if s["symmetric"]]
    shapes = [s if isinstance(s, dict) else
              {"i_per_lane": s[0], "block": s[1], "split": s[2], "symmetric": 0} for s in shapes]

    if op == "force":
        def run(launch):
            return api.accel(X, M, eps, prec=prec, launch=launch)
        reset = None
        compare = run
    else:
        acc0 = api.accel(X, M, eps, prec=prec)
        lam = torch.tensor(np.random.default_rng(seed + 1).normal(size=(3, n)), dtype=pdt, device=dev)
        st = {}

        def reset():
            st["x"], st["v"], st["a"] = X.clone(), V.clone(), acc0.clone()
            st["lx"], st["lv"] = torch.zeros_like(lam), lam.clone()
            st["lm"] = torch.zeros(n, dtype=torch.float64, device=dev)

        def run(launch):
            if adjoint_pass == "walk":  # one walked-back step: reverse drift + a pass with the force sums
                api.step_adjoint(st["x"], st["v"], M, st["a"], st["lx"], st["lv"], st["lm"], eps,
                                 2.0 ** -16, 1, prec=prec, launch=launch)
            else:  # the entry pass: J^T lam and G^T lam at x, no force sums
                api.step_adjoint(st["x"], st["v"], M, st["a"], st["lx"], st["lv"], st["lm"], eps,
                                 2.0 ** -16, 0, prec=prec, launch=launch, entry_half=True)

        def compare(launch):
            reset()
            run(launch)
            return st["lx"].clone()

    # shapes differ by the rounding of the FP32 pair arithmetic: within the
    # accuracy bars of the results (1e-5 for accelerations; 1e-4 for the
    # gradient terms, whose pair sums cancel more; 1e-3 for them with plain
    # FP32 running sums, whose order differs most between shapes)
    tol = 1e-12 if prec == "f64" else (1e-5 if op == "force" else (1e-3 if prec == "f32" else 1e-4))
    base = compare(None)
    lib_call = lambda: run(None)
    _warm_up(lib_call, reset=reset)
    t_lib = _time(lib_call, reps, reset)
    best = None
    rows = []
    for launch in shapes:
        r = compare(launch)
        err = float(torch.linalg.norm(r - base) / torch.linalg.norm(base))
        if err > tol:
            raise RuntimeError("shape %s disagrees with the default by %.3g" % (launch, err))
        ms = _time(lambda: run(launch), reps, reset)
        rows.append((ms, launch))
        if best is None or ms < best[0]:
            best = (ms, launch)
    t_lib = min(t_lib, _time(lib_call, reps, reset))
    rows.sort(key=lambda r: r[0])
    info = api.pass_info(1 if op == "force" else 2, n, prec)
    return {"op": op if op == "force" else "adjoint-" + adjoint_pass, "n": n, "prec": prec,
            "best": best[1], "best_ms": best[0],
            "best_gpairs_per_s": n * n / best[0] / 1e6, "library_ms": t_lib,
            "library_shape": {k: info[k] for k in ("symmetric", "block", "i_per_lane", "split")},
            "library_gpairs_per_s": n * n / t_lib / 1e6,
            "checked": len(rows),
            "top5": [{"ms": ms, **ln} for ms, ln in rows[:5]]}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, nargs="+", default=[16384, 65536, 262144, 1048576])
    ap.add_argument("--prec", nargs="+", default=["mix_tilec"])
    ap.add_argument("--op", nargs="+", default=["force"], choices=["force", "adjoint"])
    ap.add_argument("--symmetric-only", action="store_true",
                    help="sweep the symmetric pass's shapes only")
    ap.add_argument("--adjoint-pass", default="walk", choices=["walk", "entry"],
                    help="the adjoint pass timed: a walked-back step (with the force sums) or "
                         "the entry pass (without them)")
    args = ap.parse_args(argv)
    for op in args.op:
        for prec in args.prec:
            for n in args.n:
                print(json.dumps(tune(n, prec, op=op, one_sided=not args.symmetric_only,
                                      adjoint_pass=args.adjoint_pass)), flush=True)


if __name__ == "__main__":
    main()
