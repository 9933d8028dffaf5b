"""GPU parity of the pair-force kernel (Eq. (1)) against the FP64 oracle.

Every comparison feeds both sides the same values: the oracle gets the
device arrays promoted to FP64 exactly (for the mixed policies, the FP64
positions; their rounding to FP32 inside the kernel is part of the measured
error). Bars: global relative error <= 1e-12 (FP64) and <= 1e-5 (FP32 pair
arithmetic).
"""

import numpy as np
import pytest
import torch

import oracle
import paper_2411_18889_amd as nb
from nbody_inputs import make_state, plummer_sphere
from tests.gpu_util import (DEV, PRECS, TOL, cluster_centres, host, per_particle, rel,
                            sample_indices, to_dev)

pytestmark = pytest.mark.gpu

EDGE_NS = (1, 2, 3, 7, 63, 64, 65, 255, 256, 257, 511, 1000, 1041)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", EDGE_NS)
def test_force_tile_edges(prec, n):
    x, v, m = plummer_sphere(n, 100 + n)
    eps = 2.0 ** -6
    xd, _, md = to_dev(x, v, m, prec)
    a, pot = nb.accel(xd, md, eps, prec=prec, potential=True)
    ref, rpot = oracle.accel(host(xd), host(md), eps, potential=True)
    if n == 1:
        assert np.all(host(a) == 0) and np.all(host(pot) == 0)
        return
    assert rel(host(a), ref) <= TOL[prec]
    assert rel(host(pot), rpot) <= TOL[prec]


@pytest.mark.parametrize("prec", ("f64", "mix_tilec", "f32"))
def test_force_separate_sink_and_source_sets(prec):
    xs, vs, ms = plummer_sphere(777, 5)
    xt, _, _ = plummer_sphere(300, 6)
    eps = 2.0 ** -5
    xsd, _, msd = to_dev(xs, vs, ms, prec)
    xtd = torch.tensor(xt, dtype=nb.pos_dtype(prec), device=DEV)
    a, pot = nb.accel(xtd, msd, eps, prec=prec, xj=xsd, potential=True)
    ref, rpot = oracle.accel(host(xtd), host(msd), eps, xj=host(xsd), potential=True)
    assert rel(host(a), ref) <= TOL[prec]
    assert rel(host(pot), rpot) <= TOL[prec]


def test_two_body_closed_form_f64():
    # |d|^2 + eps^2 = 9 + 16 = 25: a_1 = G m_2 d / 125 exactly as in the golden case
    x = torch.tensor([[1.0, 2.0], [-1.0, 1.0], [5.0, 7.0]], device=DEV, dtype=torch.float64)
    m = torch.tensor([0.25, 0.5], device=DEV, dtype=torch.float64)
    a, pot = nb.accel(x, m, 4.0, G=2.0, prec="f64", potential=True)
    np.testing.assert_allclose(host(a)[:, 0], [1 / 125, 2 / 125, 2 / 125], rtol=1e-15)
    np.testing.assert_allclose(host(a)[:, 1], [-1 / 250, -2 / 250, -2 / 250], rtol=1e-15)
    np.testing.assert_allclose(host(pot), [-1 / 5, -1 / 10], rtol=1e-15)


@pytest.mark.parametrize("prec", ("f64", "mix_tilec", "mix_kahan", "f32"))
def test_launch_shape_invariance_and_determinism(prec):
    n = 3000
    x, v, m = plummer_sphere(n, 9)
    eps = 2.0 ** -6
    xd, _, md = to_dev(x, v, m, prec)
    ref = oracle.accel(host(xd), host(md), eps)
    base = nb.accel(xd, md, eps, prec=prec)
    again = nb.accel(xd, md, eps, prec=prec)
    assert torch.equal(base, again)  # no atomics: bitwise reproducible
    for ipl in (1, 2, 4):
        for block in (64, 128, 256, 512, 1024):
            for split in (1, 3, 8):
                a = nb.accel(xd, md, eps, prec=prec,
                             launch={"i_per_lane": ipl, "block": block, "split": split})
                assert rel(host(a), ref) <= TOL[prec], (ipl, block, split)


@pytest.mark.parametrize("prec", ("f64", "mix_tilec"))
def test_newton_third_law_on_gpu(prec):
    x, v, m = plummer_sphere(4096, 3)
    xd, _, md = to_dev(x, v, m, prec)
    a = host(nb.accel(xd, md, 2.0 ** -7, prec=prec))
    mm = host(md)
    tot = np.abs((a * mm).sum(axis=1))
    scale = (np.abs(a) * mm).sum()
    assert np.all(tot <= (1e-14 if prec == "f64" else 1e-6) * scale)


def test_fp64_workload_full():
    """fp64-1024: N=1024, eps=1/64, FP64 throughout, global error <= 1e-12."""
    x, v, m = make_state("fp64-1024")
    xd, _, md = to_dev(x, v, m, "f64")
    a = host(nb.accel(xd, md, 2.0 ** -6, prec="f64"))
    assert rel(a, oracle.accel(x, m, 2.0 ** -6)) <= 1e-12


# the compensated forms: besides the global error, the 99th percentile of
# the per-particle relative error is held to the FP32 bar as well
COMPENSATED = ("mix_tilec", "mix_kahan", "mix_acc64")


@pytest.mark.parametrize("name,prec,count", [
    ("fp32-65536", "f32", 2048),
    ("subcluster-262144", "mix_tilec", 2048),
    ("subcluster-262144", "mix_kahan", 2048),
    ("subcluster-262144", "mix_acc64", 2048),
    ("subcluster-262144", "mix_acc32", 2048),
    ("scale-2^20", "mix_tilec", 512),
])
def test_full_size_sampled(name, prec, count):
    """Full-size workloads in the launch shape the library picks, checked on
    sampled sinks -- seeded random ones, the 128 nearest the centre of mass
    and, in the subcluster workload, the 128 nearest the subcluster's centre
    -- against the oracle's one-by-one sums on the FP64 state (the kernel's
    own rounding of positions is part of the error). Global error <= 1e-5
    for every FP32 form; p99 of the per-particle error <= 1e-5 as well for
    the compensated ones."""
    from nbody_inputs import WORKLOADS
    w = WORKLOADS[name]
    x, v, m = make_state(name)
    xd, _, md = to_dev(x, v, m, prec)
    a = host(nb.accel(xd, md, w.eps, prec=prec))
    xs, ms = host(xd), host(md)
    idx = sample_indices(xs, count, 128, seed=7, centres=cluster_centres(name, xs))
    ref = oracle.accel_sampled(xs, ms, w.eps, idx)
    e = rel(a[:, idx], ref)
    med, p99, mx = per_particle(a[:, idx], ref)
    print("%s %s: e_glob %.3g  per-particle median %.3g p99 %.3g max %.3g"
          % (name, prec, e, med, p99, mx))
    assert e <= TOL[prec]
    if prec in COMPENSATED:
        assert p99 <= 1e-5, (med, p99, mx)


@pytest.mark.parametrize("prec", COMPENSATED)
def test_subcluster_core_sinks(prec):
    """The 512 sinks nearest the subcluster's centre (offset 3 from the
    origin, scale 0.1: the closest pairs of the workload, where the rounding
    of positions to FP32 weighs most): per-particle p99 <= 1e-5 and global
    error <= 1e-5 against the oracle on the FP64 state."""
    name = "subcluster-262144"
    x, v, m = make_state(name)
    xd, _, md = to_dev(x, v, m, prec)
    a = host(nb.accel(xd, md, 2.0 ** -9, prec=prec))
    xs, ms = host(xd), host(md)
    c = cluster_centres(name, xs)[0]
    idx = np.sort(np.argsort(np.linalg.norm(xs - c[:, None], axis=0))[:512])
    ref = oracle.accel_sampled(xs, ms, 2.0 ** -9, idx)
    e = rel(a[:, idx], ref)
    med, p99, mx = per_particle(a[:, idx], ref)
    print("%s core sinks: e_glob %.3g median %.3g p99 %.3g max %.3g" % (prec, e, med, p99, mx))
    assert e <= 1e-5 and p99 <= 1e-5


MAX_N = 1 << 30  # the largest particle count the library accepts


@pytest.mark.parametrize("prec", ["mix_tilec", "f64"])
def test_max_size_sink_set(prec):
    """2^30 sinks, the largest count the ABI accepts, against 1000 sources
    (several tiles and a ragged tail), with the potential: the sink indexing
    at the top of its range. Sampled sinks, the first and the last ones
    among them, against the oracle. Positions are seeded Plummer draws made
    on the device (2^30 of them would take minutes on the host)."""
    from nbody_inputs import plummer_positions_device
    pdt, mdt = nb.pos_dtype(prec), nb.mass_dtype(prec)
    xi = plummer_positions_device(MAX_N, 401, DEV).to(pdt)
    xj = plummer_positions_device(1000, 402, DEV).to(pdt)
    mj = torch.full((1000,), 1.0 / 1000, dtype=mdt, device=DEV)
    eps = 2.0 ** -10
    a, pot = nb.accel(xi, mj, eps, prec=prec, xj=xj, potential=True)
    rng = np.random.default_rng(403)
    idx = np.unique(np.concatenate([np.arange(64), rng.integers(0, MAX_N, 2048),
                                    np.arange(MAX_N - 300, MAX_N)]))
    it = torch.tensor(idx, device=DEV)
    ah, ph, xs = host(a[:, it]), host(pot[it]), host(xi[:, it])
    del a, pot, xi
    torch.cuda.empty_cache()
    ref, rpot = oracle.accel(xs, host(mj), eps, xj=host(xj), potential=True)
    e, ep = rel(ah, ref), rel(ph, rpot)
    print("%s: 2^30 sinks x 1000 sources, sampled e_glob %.3g, potential %.3g" % (prec, e, ep))
    assert e <= TOL[prec] and ep <= TOL[prec]


def test_max_size_source_set():
    """16 sinks against 2^30 sources: the source range split into 256 ranges
    of 2^22 with FP64 partials, and the workspace that
    nbody_workspace_size(NB_OP_ACCEL, 2^30) reports; every sink against the
    oracle, with the potential."""
    from nbody_inputs import plummer_positions_device
    prec = "mix_tilec"
    xj = plummer_positions_device(MAX_N, 404, DEV)
    mj = torch.full((MAX_N,), 2.0 ** -30, dtype=torch.float32, device=DEV)
    xi = plummer_positions_device(16, 405, DEV)
    eps = 2.0 ** -10
    a, pot = nb.accel(xi, mj, eps, prec=prec, xj=xj, potential=True)
    ah, ph = host(a), host(pot)
    xjh = xj.cpu().numpy()
    del xj, mj
    torch.cuda.empty_cache()
    ref, rpot = oracle.accel(host(xi), np.full(MAX_N, 2.0 ** -30), eps, xj=xjh, potential=True)
    e, ep = rel(ah, ref), rel(ph, rpot)
    print("16 sinks x 2^30 sources: e_glob %.3g, potential %.3g" % (e, ep))
    assert e <= TOL[prec] and ep <= TOL[prec]


@pytest.mark.parametrize("prec", ["mix_tilec", "f32", "f64"])
def test_one_shard_of_eight(prec):
    """One GPU's share of the scale-2^20 force pass sharded by sinks over
    eight GPUs: the last N/8 particles as sinks against all N as sources
    (separate sets, the one-sided kernel). 512 seeded sinks of the shard
    against the oracle, and the whole shard against the same rows of the
    pass of the set on itself (the symmetric kernel: another order of the
    same sums)."""
    x, v, m = make_state("scale-2^20")
    n = x.shape[1]
    ni = n // 8
    eps = 2.0 ** -10
    xd, _, md = to_dev(x, v, m, prec)
    xi = xd[:, n - ni:].contiguous()
    a = host(nb.accel(xi, md, eps, prec=prec, xj=xd))
    full = host(nb.accel(xd, md, eps, prec=prec))[:, n - ni:]
    idx = np.sort(np.random.default_rng(31).choice(ni, 512, replace=False))
    ref = oracle.accel_sampled(host(xd), host(md), eps, idx + (n - ni))
    e, e_full = rel(a[:, idx], ref), rel(a, full)
    print("%s: shard %d x %d sampled e_glob %.3g, against the full pass %.3g" % (prec, ni, n, e, e_full))
    assert e <= TOL[prec] and e_full <= TOL[prec]
