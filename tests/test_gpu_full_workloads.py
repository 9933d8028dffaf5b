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


def _f64_force_parity(xd, md, eps, name, seed):
    """Sampled sinks of the FP64 force pass against the oracle: <= 1e-12."""
    import oracle
    from tests.gpu_util import cluster_centres, sample_indices
    a = host(nb.accel(xd, md, eps, prec="f64"))
    xs, ms = host(xd), host(md)
    idx = sample_indices(xs, 256, 32, seed=seed, centres=cluster_centres(name, xs))
    e = rel(a[:, idx], oracle.accel_sampled(xs, ms, eps, idx))
    return e


@pytest.mark.parametrize("name", ["subcluster-262144", "scale-2^20"])
def test_workload_energy_drift_per_variant(name):
    """The workloads' trajectories as the workload descriptions ask: 20 steps
    (subcluster, every mixed variant) or 10 steps (2^20, tile-compensated)
    against an FP64 trajectory run on the GPU, whose force pass first passes
    the sampled <= 1e-12 parity check against the oracle at the initial and
    at the final state. Per variant: the energy drift dE = (E_S - E_0)/|E_0|
    (FP64 diagnostics) differs from the FP64 trajectory's by less than the
    work a force error of 1e-5 could do over the run, and the final positions
    differ by less than 1e-5 of the distance travelled."""
    w = WORKLOADS[name]
    x, v, m = make_state(name)
    S = w.steps
    # the FP64 reference trajectory, parity-checked at both ends
    xd, vd, md = to_dev(x, v, m, "f64")
    e0 = _f64_force_parity(xd, md, w.eps, name, seed=61)
    D0 = nb.diag_dict(nb.diag(xd, vd, md, w.eps, prec="f64"))
    acc = torch.empty_like(xd)
    nb.step(xd, vd, md, acc, w.eps, w.dt, S, prec="f64")
    D1 = nb.diag_dict(nb.diag(xd, vd, md, w.eps, prec="f64"))
    e1 = _f64_force_parity(xd, md, w.eps, name, seed=62)
    print("%s FP64 reference: force parity %.3g (step 0), %.3g (step %d)" % (name, e0, e1, S))
    assert e0 <= 1e-12 and e1 <= 1e-12
    dE_ref = (D1["E"] - D0["E"]) / abs(D0["E"])
    x_ref = host(xd)
    travelled = np.linalg.norm(x_ref - x)
    del xd, vd, acc
    # the bound on the energy difference a 1e-5 force error allows
    import oracle
    idx = np.arange(0, x.shape[1], max(1, x.shape[1] // 8192))
    a0 = oracle.accel_sampled(x, m, w.eps, idx)
    power = float((m[idx] * np.linalg.norm(v[:, idx], axis=0) * np.linalg.norm(a0, axis=0)).sum()
                  * (x.shape[1] / idx.size))
    bound = 2.0 * 1e-5 * S * w.dt * power / abs(D0["E"])
    for prec in w.precisions:
        xd, vd, md = to_dev(x, v, m, prec)
        acc = torch.empty_like(xd)
        E0 = nb.diag_dict(nb.diag(xd, vd, md, w.eps, prec=prec))["E"]
        nb.step(xd, vd, md, acc, w.eps, w.dt, S, prec=prec)
        E1 = nb.diag_dict(nb.diag(xd, vd, md, w.eps, prec=prec))["E"]
        assert E0 == pytest.approx(D0["E"], rel=1e-13)
        dE = (E1 - E0) / abs(E0)
        dx = np.linalg.norm(host(xd) - x_ref)
        print("%s %s: dE %.4e (FP64 trajectory %.4e, difference %.3g, bound %.3g); "
              "|x - x_fp64| %.3g of the distance travelled"
              % (name, prec, dE, dE_ref, abs(dE - dE_ref), bound, dx / travelled))
        assert abs(dE - dE_ref) <= bound
        assert dx <= 1e-5 * travelled
        del xd, vd, acc
