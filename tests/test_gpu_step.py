"""GPU parity of the KDK leapfrog, checkpoints and FP64 diagnostics."""

import numpy as np
import pytest
import torch

import oracle
import paper_2411_18889_amd as nb
from nbody_inputs import WORKLOADS, make_state, plummer_sphere
from tests.gpu_util import DEV, host, rel, sample_indices, to_dev

pytestmark = pytest.mark.gpu


def test_fp64_workload_ten_steps():
    """fp64-1024: 10 KDK steps in FP64 against the oracle, <= 1e-12."""
    w = WORKLOADS["fp64-1024"]
    x, v, m = make_state(w)
    xd, vd, md = to_dev(x, v, m, "f64")
    acc = torch.empty_like(xd)
    nb.step(xd, vd, md, acc, w.eps, w.dt, w.steps, prec="f64")
    xo, vo, ao = oracle.kdk(x, v, m, w.eps, w.dt, w.steps)
    assert rel(host(xd), xo) <= 1e-12
    assert rel(host(vd), vo) <= 1e-12
    assert rel(host(acc), ao) <= 1e-12


@pytest.mark.parametrize("n", (1, 2, 65, 300))
@pytest.mark.parametrize("prec", ("f64", "mix_tilec", "f32"))
def test_steps_small(n, prec):
    x, v, m = plummer_sphere(n, 40 + n)
    eps, dt, S = 2.0 ** -5, 2.0 ** -7, 5
    xd, vd, md = to_dev(x, v, m, prec)
    x0, v0, m0 = host(xd), host(vd), host(md)
    acc = torch.empty_like(xd)
    nb.step(xd, vd, md, acc, eps, dt, S, prec=prec)
    xo, vo, ao = oracle.kdk(x0, v0, m0, eps, dt, S)
    tol = 1e-12 if prec == "f64" else 1e-5
    assert rel(host(xd), xo) <= tol
    assert rel(host(vd), vo) <= max(tol, 1e-6 if prec != "f64" else tol)
    if n > 1:
        assert rel(host(acc), ao) <= tol * 10


def test_fp32_workload_step_one():
    """fp32-65536, step 1: the GPU's acceleration at its own FP32 state x_1,
    against the oracle at the same (promoted) state, on sampled sinks."""
    w = WORKLOADS["fp32-65536"]
    x, v, m = make_state(w)
    xd, vd, md = to_dev(x, v, m, "f32")
    acc = torch.empty_like(xd)
    nb.step(xd, vd, md, acc, w.eps, w.dt, 1, prec="f32")
    xs, ms = host(xd), host(md)
    idx = sample_indices(xs, 2048, 128, seed=3)
    e = rel(host(acc)[:, idx], oracle.accel_sampled(xs, ms, w.eps, idx))
    print("fp32-65536 step 1 e_glob %.3g" % e)
    assert e <= 1e-5


@pytest.mark.parametrize("prec", ("f64", "mix_tilec"))
def test_reversibility(prec):
    x, v, m = plummer_sphere(2048, 51)
    eps, dt, S = 2.0 ** -7, 2.0 ** -8, 10
    xd, vd, md = to_dev(x, v, m, prec)
    x0, v0 = xd.clone(), vd.clone()
    acc = torch.empty_like(xd)
    nb.step(xd, vd, md, acc, eps, dt, S, prec=prec)
    vd.neg_()
    nb.step(xd, vd, md, acc, eps, dt, S, prec=prec, acc_valid=True)
    vd.neg_()
    tol = 1e-12 if prec == "f64" else 1e-6
    assert float((xd - x0).abs().max()) <= tol
    assert float((vd - v0).abs().max()) <= tol


def test_checkpoints_hold_the_intermediate_states():
    x, v, m = plummer_sphere(700, 52)
    eps, dt, S, K = 2.0 ** -6, 2.0 ** -7, 7, 3
    xd, vd, md = to_dev(x, v, m, "f64")
    n = xd.shape[1]
    ckpt = torch.full((S // K + 1, 9 * n), float("nan"), dtype=torch.float64, device=DEV)
    acc = torch.empty_like(xd)
    nb.step(xd, vd, md, acc, eps, dt, S, prec="f64", ckpt=ckpt, ckpt_every=K)
    for slot in range(S // K + 1):
        k = slot * K
        xo, vo, ao = oracle.kdk(x, v, m, eps, dt, k)
        c = host(ckpt[slot]).reshape(3, 3, n)
        assert rel(c[0], xo) <= 1e-12 and rel(c[1], vo) <= 1e-12 and rel(c[2], ao) <= 1e-12


@pytest.mark.parametrize("prec", ("f64", "f32", "mix_tilec"))
def test_diag_matches_oracle(prec):
    x, v, m = plummer_sphere(3000, 53)
    eps = 2.0 ** -7
    xd, vd, md = to_dev(x, v, m, prec)
    d = nb.diag_dict(nb.diag(xd, vd, md, eps, prec=prec))
    o = oracle.diag(host(xd), host(vd), host(md), eps)
    for k in ("KE", "PE", "E", "M"):
        assert d[k] == pytest.approx(o[k], rel=1e-12), k
    for k in ("Px", "Py", "Pz", "Lx", "Ly", "Lz", "COMx", "COMy", "COMz"):
        assert abs(d[k] - o[k]) <= 1e-13, k


def test_energy_drift_fp32_vs_fp64_short():
    """A short FP32 run drifts in energy by no more than a small multiple of
    the FP64 run's drift plus the FP32 rounding floor."""
    x, v, m = plummer_sphere(8192, 54)
    eps, dt, S = 2.0 ** -8, 2.0 ** -9, 20
    drift = {}
    for prec in ("f64", "f32", "mix_tilec"):
        xd, vd, md = to_dev(x, v, m, prec)
        E0 = nb.diag_dict(nb.diag(xd, vd, md, eps, prec=prec))["E"]
        acc = torch.empty_like(xd)
        nb.step(xd, vd, md, acc, eps, dt, S, prec=prec)
        E1 = nb.diag_dict(nb.diag(xd, vd, md, eps, prec=prec))["E"]
        drift[prec] = abs(E1 - E0) / abs(E0)
    print("energy drift over 20 steps:", drift)
    assert drift["mix_tilec"] <= 10 * drift["f64"] + 1e-6
    assert drift["f32"] <= 10 * drift["f64"] + 1e-5


def test_resume_from_saved_state_is_bitwise(tmp_path):
    """5 steps, save (x, v, a) with torch.save, reload, 5 more steps: bitwise
    the same state as 10 steps in one call (the kernels are deterministic and
    the saved acceleration is reused, not recomputed)."""
    x, v, m = plummer_sphere(3000, 55)
    eps, dt = 2.0 ** -7, 2.0 ** -8
    for prec in ("mix_tilec", "f32", "f64"):
        xa, va, ma = to_dev(x, v, m, prec)
        xb, vb, mb = to_dev(x, v, m, prec)
        aa, ab = torch.empty_like(xa), torch.empty_like(xb)
        nb.step(xa, va, ma, aa, eps, dt, 10, prec=prec)
        nb.step(xb, vb, mb, ab, eps, dt, 5, prec=prec)
        path = tmp_path / ("state_%s.pt" % prec)
        torch.save({"x": xb.cpu(), "v": vb.cpu(), "a": ab.cpu(), "step": 5}, path)
        st = torch.load(path, weights_only=True)
        xc, vc, ac = (st[k].to(DEV) for k in ("x", "v", "a"))
        nb.step(xc, vc, mb, ac, eps, dt, 5, prec=prec, acc_valid=True)
        assert torch.equal(xc, xa) and torch.equal(vc, va) and torch.equal(ac, aa), prec
