"""The fused epilogues are bitwise the separate launches they replace.

The force pass's finishing kernel applies the leapfrog's closing half-kick
and, inside a multi-step call, the next step's kick and drift; the adjoint
pass's finishing kernel applies the next step's reverse drift. A call that
checkpoints every step (no fusion: the state has to be stored between the
kick and the drift) and a chain of single-step adjoint calls (each starts
with its own reverse-drift launch) must give bitwise the same state as the
fused calls -- for the one-sided kernel with a split source range (its
reduction kernel is the finishing kernel) and for the symmetric pass."""

import numpy as np
import pytest
import torch

import paper_2411_18889_amd as nb
from nbody_inputs import plummer_sphere
from tests.gpu_util import DEV, to_dev

pytestmark = pytest.mark.gpu

# (n, policy, which pass): 5000 one-sided with a split source range;
# 20000 the symmetric pass; f64 and f32 run the symmetric force and adjoint
# too
CASES = [(5000, "mix_tilec"), (20000, "mix_tilec"), (20000, "f64"), (20000, "f32"),
         (3000, "mix_kahan")]


@pytest.mark.parametrize("n,prec", CASES)
def test_fused_kick_drift_is_bitwise(n, prec):
    S = 5
    x, v, m = plummer_sphere(n, 810 + n % 13)
    eps, dt = 2.0 ** -7, 2.0 ** -8
    info = nb.pass_info(1, n, prec)
    assert info["symmetric"] == 1 or info["split"] > 1  # a pass with a finishing kernel
    out = []
    for every in (None, 1):
        xd, vd, md = to_dev(x, v, m, prec)
        acc = torch.empty_like(xd)
        ckpt = None if every is None else torch.empty((S + 1, 9 * n), dtype=xd.dtype, device=DEV)
        nb.step(xd, vd, md, acc, eps, dt, S, prec=prec, ckpt=ckpt, ckpt_every=every or 0)
        out.append((xd, vd, acc))
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("n,prec", [(5000, "mix_tilec"), (20000, "mix_tilec"), (3000, "f64"),
                                    (20000, "f64"), (20000, "f32")])
def test_fused_reverse_drift_is_bitwise(n, prec):
    S = 4
    x, v, m = plummer_sphere(n, 820 + n % 7)
    eps, dt = 2.0 ** -7, 2.0 ** -8
    info = nb.pass_info(2, n, prec)
    assert info["symmetric"] == 1 or info["split"] > 1
    rng = np.random.default_rng(n)
    lam_x, lam_v = rng.normal(size=(3, n)), rng.normal(size=(3, n))
    res = []
    for chained in (False, True):
        xd, vd, md = to_dev(x, v, m, prec)
        acc = torch.empty_like(xd)
        nb.step(xd, vd, md, acc, eps, dt, S, prec=prec)
        lx = torch.tensor(lam_x, dtype=xd.dtype, device=DEV)
        lv = torch.tensor(lam_v, dtype=xd.dtype, device=DEV)
        lm = torch.zeros(n, dtype=torch.float64, device=DEV)
        if chained:  # S calls of one step: no reverse drift is fused
            for k in range(S):
                nb.step_adjoint(xd, vd, md, acc, lx, lv, lm, eps, dt, 1, prec=prec,
                                entry_half=(k == 0), exit_full=(k < S - 1))
        else:
            nb.step_adjoint(xd, vd, md, acc, lx, lv, lm, eps, dt, S, prec=prec, entry_half=True)
        res.append((xd, vd, acc, lx, lv, lm))
    for a, b in zip(*res):
        assert torch.equal(a, b)
