"""Writes the stored expected values of the full-size GPU tests.

Calls only the FP64 CPU oracle (oracle/) and the seeded input generator
(nbody_inputs/); nothing here comes from the GPU library.

  adjoint_16384.npz  (workload adjoint-16384: N = 16384, eps = 2^-7,
                      dt = 2^-8, 200 KDK steps)
      y        target positions: end state of an FP64 run of 200 steps from
               the initial state perturbed by N(0, 1e-3) (seed 44)
      loss     L = (1/N) sum_i |x_200,i - y_i|^2 from the unperturbed state
      gx, gv, gm   dL/dx_0, dL/dv_0, dL/dm from the oracle's reverse-mode
               walk over the stored FP64 trajectory (float32 storage)
      fd_x, fd_v, fd_m   central differences (L(p + h u) - L(p - h u)) / 2h,
               h = 1e-6, FP64 forward runs, along the directions
               direction(block, k) (two per block; for the masses the step is
               m * u, relative)
  energy_65536.txt   (workload fp32-65536) E(t) of the FP64 oracle run of
               100 steps from the FP32-rounded initial state, every step

Run from the repository root: python tests/golden/make_goldens.py [adjoint|energy]
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from nbody_inputs import WORKLOADS, make_state, perturb_state, random_unit_vectors  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
H = 1e-6
DIRECTION_SEEDS = {"x": 1001, "v": 1002, "m": 1003}


def direction(block, k, n):
    """The k-th seeded unit direction for block 'x', 'v' or 'm' of n particles."""
    shape = (n,) if block == "m" else (3, n)
    return random_unit_vectors(shape, DIRECTION_SEEDS[block] + 10 * k)


def _loss(x0, v0, m, w, y):
    x, _, _ = oracle.kdk(x0, v0, m, w.eps, w.dt, w.steps)
    return float(np.sum((x - y) ** 2) / x0.shape[1])


def adjoint_golden():
    w = WORKLOADS["adjoint-16384"]
    x0, v0, m = make_state(w)
    n = x0.shape[1]
    t = time.time()
    xp, vp = perturb_state(x0, v0, w.perturb_seed, w.perturb_sigma)
    y, _, _ = oracle.kdk(xp, vp, m, w.eps, w.dt, w.steps)
    print("targets %.0f s" % (time.time() - t), flush=True)
    xs, _, _, tx, _ = oracle.kdk(x0, v0, m, w.eps, w.dt, w.steps, trajectory=True)
    loss = float(np.sum((xs - y) ** 2) / n)
    print("forward %.0f s, loss %.6e" % (time.time() - t, loss), flush=True)
    gx, gv, gm = oracle.adjoint(tx, m, w.eps, w.dt, 2.0 / n * (xs - y), np.zeros_like(x0))
    del tx
    print("adjoint %.0f s" % (time.time() - t), flush=True)
    out = dict(y=y, loss=np.array(loss), gx=gx.astype(np.float32), gv=gv.astype(np.float32),
               gm=gm.astype(np.float32))
    for name in "xvm":
        fd = []
        for u in (direction(name, k, n) for k in range(2)):
            args_p = [x0, v0, m]
            args_m = [x0, v0, m]
            i = "xvm".index(name)
            # the mass direction is relative (m * u), so it keeps its scale
            step = u * m if name == "m" else u
            args_p[i] = args_p[i] + H * step
            args_m[i] = args_m[i] - H * step
            fd.append((_loss(*args_p, w, y) - _loss(*args_m, w, y)) / (2 * H))
            print("fd %s %.0f s: %.9e" % (name, time.time() - t, fd[-1]), flush=True)
        out["fd_" + name] = np.array(fd)
    np.savez_compressed(os.path.join(HERE, "adjoint_16384.npz"), **out)
    print("wrote adjoint_16384.npz", flush=True)


def energy_golden():
    w = WORKLOADS["fp32-65536"]
    x0, v0, m = make_state(w)
    x = x0.astype(np.float32).astype(np.float64)
    v = v0.astype(np.float32).astype(np.float64)
    m = m.astype(np.float32).astype(np.float64)
    lines = ["# FP64 oracle energy of workload fp32-65536 (N = 65536, eps = 2^-8, dt = 2^-9),",
             "# from the FP32-rounded initial state, every 5 steps; columns: step E KE PE",
             "# written by tests/golden/make_goldens.py energy (calls only oracle/)"]
    t = time.time()
    _, _, _, tx, tv = oracle.kdk(x, v, m, w.eps, w.dt, w.steps, trajectory=True)
    print("trajectory %.0f s" % (time.time() - t), flush=True)
    for s in range(0, w.steps + 1, 5):
        d = oracle.diag(tx[s], tv[s], m, w.eps)
        lines.append("%d %.17e %.17e %.17e" % (s, d["E"], d["KE"], d["PE"]))
        print("step %d %.0f s E %.12e" % (s, time.time() - t, d["E"]), flush=True)
    open(os.path.join(HERE, "energy_65536.txt"), "w").write("\n".join(lines) + "\n")
    print("wrote energy_65536.txt", flush=True)


if __name__ == "__main__":
    what = sys.argv[1:] or ["adjoint", "energy"]
    if "adjoint" in what:
        adjoint_golden()
    if "energy" in what:
        energy_golden()
