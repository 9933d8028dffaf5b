"""GPU parity of the symmetric (third-law) force pass, which the library
uses for one set acting on itself with the tile-compensated and the plain
FP32 policies from 12288 particles on: blocks of 256 or 512 particles below
81920, 1024 below 2^18, 2048 from there, a work item per block pair, FP32
partials per block added in a fixed order.

Checked against the FP64 oracle (all sinks up to 20000, sampled sinks above),
against the one-sided kernel on every sink at any size, and by the third law
itself, which the j-side sums carry: sum_i m_i a_i = 0."""

import numpy as np
import pytest
import torch

import oracle
import paper_2411_18889_amd as nb
from nbody_inputs import plummer_sphere
from tests.gpu_util import DEV, host, per_particle, rel, sample_indices, to_dev

pytestmark = pytest.mark.gpu

PREC = "mix_tilec"
TOL = 1e-5
TOLS = {"f32": 1e-5, "f64": 1e-12}

# blocks of 256 (12288 .. 24575), 512, 1024 and 2048 (eight sinks per lane,
# from 2^18); ragged last blocks and tiles
SYM_NS = (12288, 12289, 14000, 16384, 16385, 20000, 24576 + 7, 32768, 32769, 32768 + 255, 40000, 65535, 65536,
          65536 + 1000, 81920 + 5, 131072 + 77, 262144 + 1, 262144 + 2047)


def _classic(xd, md, eps):
    # the one-sided kernel in an explicit launch shape
    return nb.accel(xd, md, eps, prec=PREC, launch={"i_per_lane": 2, "block": 256, "split": 4})


@pytest.mark.parametrize("n", SYM_NS)
def test_sym_matches_oracle_and_one_sided(n):
    x, v, m = plummer_sphere(n, 200 + n % 97)
    m = m * np.random.default_rng(n).uniform(0.5, 1.5, size=n)  # unequal masses
    eps = 2.0 ** -8
    xd, _, md = to_dev(x, v, m, PREC)
    a = host(nb.accel(xd, md, eps, prec=PREC))
    xs, ms = host(xd), host(md)
    if n <= 40000:
        ref = oracle.accel(xs, ms, eps)
        e = rel(a, ref)
    else:
        idx = sample_indices(xs, 1024, 64, seed=n)
        ref = oracle.accel_sampled(xs, ms, eps, idx)
        e = rel(a[:, idx], ref)
    print("n=%d sym e_glob %.3g" % (n, e))
    assert e <= TOL
    # every sink, against the one-sided kernel (itself parity-tested)
    c = host(_classic(xd, md, eps))
    assert rel(a, c) <= TOL
    med, p99, mx = per_particle(a, c)
    assert p99 <= 1e-5, (med, p99, mx)


@pytest.mark.parametrize("prec,n", [(p, n) for p in ("f32", "f64")
                                    for n in (12288, 12289, 20000, 40000, 65535, 65536 + 1000,
                                              262144 + 2047)])
def test_sym_f32_f64_policies(prec, n):
    """The plain FP32 policy (FP32 state, every sum FP32) and the FP64 one
    (FP64 pair arithmetic, FP64 source-side sums through the lanes, FP64
    partials) run the same symmetric pass from 12288 particles: against the
    oracle on the same state (every sink up to 40000, sampled above; 1e-5
    and 1e-12), against the one-sided kernel on every sink, bitwise
    reproducible, and with the potential (which leaves the accelerations
    bitwise unchanged)."""
    tol = TOLS[prec]
    x, v, m = plummer_sphere(n, 270 + n % 83)
    m = m * np.random.default_rng(n + 2).uniform(0.5, 1.5, size=n)
    eps = 2.0 ** -8
    xd, _, md = to_dev(x, v, m, prec)
    assert nb.pass_info(1, n, prec)["symmetric"] == 1
    a1 = nb.accel(xd, md, eps, prec=prec)
    a, pot = nb.accel(xd, md, eps, prec=prec, potential=True)
    assert torch.equal(a, a1)
    ah, ph = host(a), host(pot)
    xs, ms = host(xd), host(md)
    if n <= 40000:
        ra, rp = oracle.accel(xs, ms, eps, potential=True)
        ea, ep = rel(ah, ra), rel(ph, rp)
    else:
        idx = sample_indices(xs, 1024, 64, seed=n)
        ra, rp = oracle.accel_sampled(xs, ms, eps, idx, potential=True)
        ea, ep = rel(ah[:, idx], ra), rel(ph[idx], rp)
    print("n=%d %s symmetric e_glob %.3g, potential %.3g" % (n, prec, ea, ep))
    assert ea <= tol and ep <= tol
    c = host(nb.accel(xd, md, eps, prec=prec, launch={"i_per_lane": 2, "block": 256, "split": 4}))
    assert rel(ah, c) <= tol
    assert torch.equal(nb.accel(xd, md, eps, prec=prec), a1)


def test_sym_third_law_and_determinism():
    n = 65536
    x, v, m = plummer_sphere(n, 211)
    xd, _, md = to_dev(x, v, m, PREC)
    a1 = nb.accel(xd, md, 2.0 ** -8, prec=PREC)
    a2 = nb.accel(xd, md, 2.0 ** -8, prec=PREC)
    assert torch.equal(a1, a2)  # fixed-order sums: bitwise reproducible
    a = host(a1)
    mm = host(md)
    tot = np.abs((a * mm).sum(axis=1))
    scale = (np.abs(a) * mm).sum()
    assert np.all(tot <= 1e-6 * scale), (tot, scale)


@pytest.mark.parametrize("prec", ("mix_tilec", "f64"))
def test_sym_step_matches_oracle(prec):
    """The leapfrog at n = 32768 (symmetric force with the closing half-kick
    in its finishing kernel) against the oracle's FP64 steps."""
    n, S = 32768, 3
    x, v, m = plummer_sphere(n, 230)
    eps, dt = 2.0 ** -7, 2.0 ** -8
    xd, vd, md = to_dev(x, v, m, prec)
    acc = torch.empty_like(xd)
    nb.step(xd, vd, md, acc, eps, dt, S, prec=prec)
    xo, vo, ao = oracle.kdk(x, v, host(md), eps, dt, S)
    f64 = prec == "f64"
    assert rel(host(xd), xo) <= (1e-14 if f64 else 1e-9)
    assert rel(host(vd) - v, vo - v) <= (1e-12 if f64 else 1e-5)
    assert rel(host(acc), ao) <= (1e-12 if f64 else TOL)


@pytest.mark.parametrize("n", (1_200_000, (1 << 21) + 3))
def test_sym_large_blocks(n):
    """Blocks of 2048 (4 waves x 8 sinks) with a ragged last block, and at
    2^21 + 3 (25.8 GB of partials, folded in bands of the workspace):
    sampled sinks against the oracle, every sink against the one-sided
    kernel, and the third law."""
    x, v, m = plummer_sphere(n, 240 + n % 5)
    eps = 2.0 ** -10
    xd, _, md = to_dev(x, v, m, PREC)
    a = nb.accel(xd, md, eps, prec=PREC)
    ah = host(a)
    xs, ms = host(xd), host(md)
    idx = sample_indices(xs, 256, 32, seed=n)
    e = rel(ah[:, idx], oracle.accel_sampled(xs, ms, eps, idx))
    print("n=%d sym e_glob (sampled) %.3g" % (n, e))
    assert e <= TOL
    c = _classic(xd, md, eps)
    assert float((a - c).norm() / c.norm()) <= TOL
    del c
    tot = np.abs((ah * ms).sum(axis=1))
    assert np.all(tot <= 1e-6 * (np.abs(ah) * ms).sum())


@pytest.mark.parametrize("n", (16384, 24576 + 7, 65536 + 1000, 1_600_000))
def test_sym_potential(n):
    """The potential from the symmetric pass (a fourth partial per particle
    and block, the j = i term removed after the sum): against the oracle
    (every sink up to 40000, sampled above) and the one-sided kernel on every
    sink. Its accelerations are bitwise those of the pass without the
    potential (the same blocks; the fourth partial is summed on its own)."""
    x, v, m = plummer_sphere(n, 260 + n % 89)
    m = m * np.random.default_rng(n + 1).uniform(0.5, 1.5, size=n)  # unequal masses
    eps = 2.0 ** -9
    xd, _, md = to_dev(x, v, m, PREC)
    a, pot = nb.accel(xd, md, eps, prec=PREC, potential=True)
    a0 = nb.accel(xd, md, eps, prec=PREC)
    assert torch.equal(a, a0)
    del a0
    ph = host(pot)
    xs, ms = host(xd), host(md)
    if n <= 40000:
        ra, rp = oracle.accel(xs, ms, eps, potential=True)
        ea, ep = rel(host(a), ra), rel(ph, rp)
    else:
        idx = sample_indices(xs, 256 if n > 500000 else 1024, 32, seed=n)
        ra, rp = oracle.accel_sampled(xs, ms, eps, idx, potential=True)
        ea, ep = rel(host(a)[:, idx], ra), rel(ph[idx], rp)
    print("n=%d sym potential e_glob %.3g (acc %.3g)" % (n, ep, ea))
    assert ea <= TOL and ep <= TOL
    c, cp = nb.accel(xd, md, eps, prec=PREC, potential=True,
                     launch={"i_per_lane": 2, "block": 256, "split": 1})
    assert float((pot - cp).norm() / cp.norm()) <= TOL
    assert float((pot - cp).abs().max() / cp.abs().max()) <= 1e-5
    assert bool((pot < 0).all())


@pytest.mark.parametrize("n", (1000, 20000))
def test_degenerate_coincident_and_massless(n):
    """Coincident particles (d = 0 between distinct i, j: no force between
    them, eps > 0 keeps s finite) and massless test particles (feel the
    others, pull on nothing), through the one-sided kernel (n = 1000) and the
    symmetric pass (n = 20000), force and gradient."""
    x, v, m = plummer_sphere(n, 250)
    x[:, 10:20] = x[:, 5:6]                   # eleven particles at one point
    x[:, n - 7:] = x[:, n - 8:n - 7]          # eight at another, in the last block
    m = m.copy()
    m[::97] = 0.0                             # test particles
    eps = 2.0 ** -7
    xd, vd, md = to_dev(x, v, m, PREC)
    a = host(nb.accel(xd, md, eps, prec=PREC))
    assert np.all(np.isfinite(a))
    ref = oracle.accel(host(xd), host(md), eps)
    assert rel(a, ref) <= TOL
    # a massless particle moved far away changes no other particle's force
    x2 = x.copy()
    x2[:, 0] = x2[:, 0] + 50.0 if m[0] == 0 else x2[:, 0]
    a2 = host(nb.accel(to_dev(x2, v, m, PREC)[0], md, eps, prec=PREC))
    assert rel(a2[:, 1:], a[:, 1:]) <= 1e-6
    # gradient of a short rollout stays finite and matches the oracle
    S = 2
    y = x + 0.01
    xg, vg, mg = to_dev(x, v, m, PREC)
    for t in (xg, vg, mg):
        t.requires_grad_(True)
    xs, _ = nb.rollout(xg, vg, mg, eps, 2.0 ** -8, S, ckpt_every=1, prec=PREC)
    ((xs - torch.tensor(y, device=DEV)) ** 2).sum().backward()
    _, _, _, tx, _ = oracle.kdk(host(xd), host(vd), host(md), eps, 2.0 ** -8, S, trajectory=True)
    xo = tx[-1]
    go = oracle.adjoint(tx, host(md), eps, 2.0 ** -8, 2.0 * (xo - y), np.zeros_like(v))
    for g, r in zip((xg.grad, vg.grad, mg.grad), go):
        gh = host(g)
        assert np.all(np.isfinite(gh))
        assert rel(gh, r) <= 1e-4
