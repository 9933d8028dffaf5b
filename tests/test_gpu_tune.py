"""The launch-shape tuner (the paper's per-machine NTHREADS survey,
generalised to every pair pass): on a small set of shapes it times each one,
checks each against the library's own result, and reports the fastest; and
every explicit shape of the symmetric passes and of the one-sided adjoint
gives the oracle's result."""

import numpy as np
import pytest
import torch

import oracle
import paper_2411_18889_amd as nb
from nbody_inputs import plummer_sphere
from paper_2411_18889_amd import tune
from tests.gpu_util import DEV, host, rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ("mix_tilec", "f64"))
def test_tuner_reports_the_fastest_checked_shape(prec):
    shapes = [(1, 256, 1), (2, 128, 4), (1, 64, 16)]
    r = tune.tune(4096, prec, shapes=shapes, reps=3)
    assert r["n"] == 4096 and r["prec"] == prec
    best = (r["best"]["i_per_lane"], r["best"]["block"], r["best"]["split"])
    assert best in shapes
    assert r["best_ms"] > 0 and r["library_ms"] > 0
    assert r["best_ms"] == min(row["ms"] for row in r["top5"])
    assert len(r["top5"]) == len(shapes)


@pytest.mark.parametrize("op", ("force", "adjoint"))
def test_tuner_sweeps_symmetric_and_one_sided(op):
    n = 20000
    shapes = [{"i_per_lane": 2, "block": 256, "split": 0, "symmetric": 1},
              {"i_per_lane": 2, "block": 512, "split": 0, "symmetric": 1},
              {"i_per_lane": 1, "block": 256, "split": 4, "symmetric": 0}]
    r = tune.tune(n, "mix_tilec", op=op, shapes=shapes, reps=2)
    assert r["op"] == (op if op == "force" else "adjoint-walk")
    assert r["checked"] == 3 and r["best"] in shapes
    assert r["library_shape"]["symmetric"] == 1
    assert r["best_ms"] == min(row["ms"] for row in r["top5"])


def test_candidate_shapes_cover_the_library_choice():
    for op, code in (("force", 1), ("adjoint", 2)):
        for n in (20000, 1 << 20):
            info = nb.pass_info(code, n, "mix_tilec")
            lib = {"i_per_lane": info["i_per_lane"], "block": info["block"], "split": 0,
                   "symmetric": 1}
            assert lib in tune.candidate_shapes(op, n, "mix_tilec", True)


@pytest.mark.parametrize("ipl,block", tune.SYM_FORCE)
@pytest.mark.parametrize("prec", ("mix_tilec", "f32", "f64"))
def test_symmetric_force_shapes_against_oracle(prec, ipl, block):
    n = 20000 + 37
    x, v, m = plummer_sphere(n, 900)
    xd, _, md = to_dev(x, v, m, prec)
    eps = 2.0 ** -8
    a, pot = nb.accel(xd, md, eps, prec=prec, potential=True,
                      launch={"i_per_lane": ipl, "block": block, "symmetric": 1})
    ra, rp = oracle.accel(host(xd), host(md), eps, potential=True)
    tol = 1e-12 if prec == "f64" else 1e-5
    assert rel(host(a), ra) <= tol and rel(host(pot), rp) <= tol


ADJ_SHAPES = [{"i_per_lane": ipl, "block": block, "split": 0, "symmetric": 1}
              for ipl, block in tune.SYM_ADJOINT] + \
             [{"i_per_lane": ipl, "block": block, "split": split, "symmetric": 0}
              for ipl, block, split in ((1, 64, 1), (2, 128, 3), (1, 512, 8), (2, 256, 1))]


@pytest.mark.parametrize("launch", ADJ_SHAPES, ids=lambda l: "%s-%d-%d-%d" % (
    "sym" if l["symmetric"] else "one", l["i_per_lane"], l["block"], l["split"]))
def test_adjoint_shapes_against_oracle(launch):
    """The entry pass (J^T lam and G^T lam at x, no force sums) and one
    walked-back step (a pass that also sums a(x)) in each shape: against
    the oracle's transposed Jacobians and accelerations."""
    n, prec, eps = 20000 + 37, "mix_tilec", 2.0 ** -8
    x, v, m = plummer_sphere(n, 901)
    xd, vd, md = to_dev(x, v, m, prec)
    lam = torch.tensor(np.random.default_rng(902).normal(size=(3, n)), device=DEV)
    acc = nb.accel(xd, md, eps, prec=prec)
    lx = torch.zeros_like(lam)
    lm = torch.zeros(n, dtype=torch.float64, device=DEV)
    dt = 2.0 ** -9
    nb.step_adjoint(xd, vd, md, acc, lx, lam.clone(), lm, eps, dt, 0, prec=prec, entry_half=True,
                    launch=launch)
    jt, gt = oracle.vjp(host(xd), host(md), host(lam), eps)
    c = 0.5 * dt
    assert rel(host(lx) / c, jt) <= 1e-4 and rel(host(lm) / c, gt) <= 1e-4
    # one walked-back step: the pass also leaves a(x) of the walked-back state
    h = 0.5 * dt
    xw = host(xd) - dt * (host(vd) - h * host(acc))
    nb.step_adjoint(xd, vd, md, acc, torch.zeros_like(lam), lam.clone(),
                    torch.zeros(n, dtype=torch.float64, device=DEV), eps, dt, 1, prec=prec,
                    launch=launch)
    assert rel(host(acc), oracle.accel(xw, host(md), eps)) <= 1e-5
