"""Full-size workload checks against values the FP64 oracle stored ahead of
time (tests/golden/make_goldens.py, which calls only oracle/ and the input
generator)."""

import os

import numpy as np
import pytest
import torch

import paper_2411_18889_amd as nb
from nbody_inputs import WORKLOADS, make_state
from tests.gpu_util import DEV, host, rel, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_adjoint_workload_gradient():
    """adjoint-16384: 200 KDK steps with checkpoints every 20, FP32 pair
    arithmetic in forward and adjoint (mix_tilec); gradients of the mean
    squared distance to the targets w.r.t. x_0, v_0 and m within 1e-4 of the
    oracle's FP64 reverse-mode gradient, and directional derivatives within
    1e-4 of FP64 central differences (h = 1e-6)."""
    w = WORKLOADS["adjoint-16384"]
    g = np.load(os.path.join(GOLDEN, "adjoint_16384.npz"))
    x, v, m = make_state(w)
    xd, vd, md = to_dev(x, v, m, "mix_tilec")
    for t in (xd, vd, md):
        t.requires_grad_(True)
    y = torch.tensor(g["y"], device=DEV)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    xs, vs = nb.rollout(xd, vd, md, w.eps, w.dt, w.steps, ckpt_every=w.ckpt_every, prec="mix_tilec")
    loss = ((xs - y) ** 2).sum() / x.shape[1]
    e[1].record()
    loss.backward()
    e[2].record()
    torch.cuda.synchronize()
    ratio = e[1].elapsed_time(e[2]) / e[0].elapsed_time(e[1])
    errs = {k: rel(host(t.grad), g["g" + k]) for k, t in (("x", xd), ("v", vd), ("m", md))}
    print("adjoint-16384: loss %.9e (oracle %.9e), grad rel err %s, backward/forward %.2f"
          % (float(loss), float(g["loss"]), errs, ratio))
    assert float(loss) == pytest.approx(float(g["loss"]), rel=1e-6)
    assert max(errs.values()) <= 1e-4
    from tests.golden.make_goldens import direction
    for k, t in (("x", xd), ("v", vd), ("m", md)):
        grad = host(t.grad)
        for q, fd in enumerate(g["fd_" + k]):
            u = direction(k, q, x.shape[1])
            step = u * host(md) if k == "m" else u
            assert float(np.sum(grad * step)) == pytest.approx(float(fd), rel=1e-4), k


def test_fp32_workload_energy_drift():
    """fp32-65536: 100 KDK steps in FP32; the GPU's energy drift follows the
    FP64 oracle's (same FP32-rounded initial state) to within 1e-5 of |E|."""
    w = WORKLOADS["fp32-65536"]
    ref = np.loadtxt(os.path.join(GOLDEN, "energy_65536.txt"))
    x, v, m = make_state(w)
    xd, vd, md = to_dev(x, v, m, "f32")
    acc = torch.empty_like(xd)
    E = [nb.diag_dict(nb.diag(xd, vd, md, w.eps, prec="f32"))["E"]]
    steps = [0]
    for k in range(0, w.steps, 5):
        nb.step(xd, vd, md, acc, w.eps, w.dt, 5, prec="f32", acc_valid=k > 0)
        E.append(nb.diag_dict(nb.diag(xd, vd, md, w.eps, prec="f32"))["E"])
        steps.append(k + 5)
    E = np.array(E)
    assert np.array_equal(ref[:, 0].astype(int), np.array(steps))
    E0 = ref[0, 1]
    assert E[0] == pytest.approx(E0, rel=1e-12)
    d_gpu = (E - E[0]) / abs(E0)
    d_ref = (ref[:, 1] - E0) / abs(E0)
    print("fp32-65536 energy drift: GPU %.3e, oracle %.3e at step 100; max |difference| %.3e"
          % (d_gpu[-1], d_ref[-1], np.abs(d_gpu - d_ref).max()))
    assert np.abs(d_gpu - d_ref).max() <= 1e-5
