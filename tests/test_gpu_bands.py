"""The symmetric passes in bands: with a workspace smaller than every partial
of a pass, the block-pair triangle runs in bands of rows, each folded into
per-particle running sums in slot order, so the results are bitwise those of
the pass in one band -- for the force (three policies, with and without the
potential, inside the leapfrog with its fused kick and drift) and for the
fused adjoint (with and without the force sums, with its fused reverse
drift), from the least workspace the library accepts up to one that holds
every partial. At 2^20 (the benchmark's configuration) the default workspace
against every partial; at 2^22, beyond the sizes a single band of partials
could serve, sampled rows against the oracle."""

import numpy as np
import pytest
import torch

import oracle
import paper_2411_18889_amd as nb
from nbody_inputs import plummer_sphere
from paper_2411_18889_amd._lib import NB_EWORKSPACE, NBodyError
from tests.gpu_util import DEV, host, rel, sample_indices, to_dev

pytestmark = pytest.mark.gpu


def _align(b):
    return (b + 255) // 256 * 256


def _sizes(n, prec, op, nq):
    """(every partial at once, the least workspace accepted) of the symmetric
    pass: FP32 partials (FP64 for f64), running sums in FP64 (FP32 for f32);
    the least is the running sums plus the first block row's partials (its
    slot of every particle and its other slots of its own particles)."""
    info = nb.pass_info(op, n, prec)
    assert info["symmetric"] == 1
    b = info["block_particles"]
    nblk = -(-n // b)
    elem = 8 if prec == "f64" else 4
    fin = 4 if (prec == "f32" and op != 2) else 8  # the adjoint folds in FP64
    full = nblk * nq * n * elem
    least = _align(nq * n * fin) + nq * elem * (n + (nblk - 1) * min(n, b))
    return full, min(full, least)


def _ws(nbytes):
    return torch.empty(nbytes, dtype=torch.uint8, device=DEV)


@pytest.mark.parametrize("prec", ("mix_tilec", "f32", "f64"))
@pytest.mark.parametrize("n", (12289, 40000, 65536 + 1000, 262144 + 999))
def test_force_bands_bitwise(prec, n):
    x, v, m = plummer_sphere(n, 700 + n % 11)
    m = m * np.random.default_rng(n).uniform(0.5, 1.5, size=n)
    eps = 2.0 ** -8
    xd, _, md = to_dev(x, v, m, prec)
    for pot in (False, True):
        full, least = _sizes(n, prec, 1, 4 if pot else 3)
        print("%s n=%d pot=%s: every partial %d B, least %d B" % (prec, n, pot, full, least),
              flush=True)
        ref = nb.accel(xd, md, eps, prec=prec, potential=pot, workspace=_ws(full))
        for w in (least, least + (full - least) // 7, least + (full - least) // 2, full - 1):
            got = nb.accel(xd, md, eps, prec=prec, potential=pot, workspace=_ws(w))
            if pot:
                assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), w
            else:
                assert torch.equal(got, ref), w
        with pytest.raises(NBodyError) as ei:
            nb.accel(xd, md, eps, prec=prec, potential=pot, workspace=_ws(least - 1))
        assert ei.value.status == NB_EWORKSPACE
    a = host(ref[0])
    idx = sample_indices(host(xd), 256, 32, seed=n)
    e = rel(a[:, idx], oracle.accel_sampled(host(xd), host(md), eps, idx))
    assert e <= (1e-12 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("prec", ("mix_tilec", "f64"))
def test_step_bands_bitwise(prec):
    """Three leapfrog steps: the fold kernels apply the closing half-kick and
    the next step's kick and drift to each band's particles once no later
    band reads them."""
    n, S = 40000 + 123, 3
    x, v, m = plummer_sphere(n, 733)
    eps, dt = 2.0 ** -8, 2.0 ** -9
    full, least = _sizes(n, prec, 1, 3)
    out = []
    for w in (full, least, (least + full) // 3):
        xd, vd, md = to_dev(x, v, m, prec)
        acc = torch.empty_like(xd)
        nb.step(xd, vd, md, acc, eps, dt, S, prec=prec, workspace=_ws(w))
        out.append((xd, vd, acc))
    for r in out[1:]:
        for a, b in zip(r, out[0]):
            assert torch.equal(a, b)
    xo, vo, ao = oracle.kdk(x, v, host(md), eps, dt, S)
    assert rel(host(out[0][2]), ao) <= (1e-12 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("prec,n", (("mix_tilec", 40000 + 77), ("mix_tilec", 262144 + 77),
                                    ("f64", 40000 + 77), ("f32", 40000 + 77)))
def test_adjoint_bands_bitwise(prec, n):
    """A three-step reverse walk (entry pass without the force sums, walked-
    back passes with them, reverse drifts fused into the folds), with two
    sinks per lane (40077) and four (262221, blocks of 1024; FP64 at 40077,
    blocks of 512)."""
    S = 3
    x, v, m = plummer_sphere(n, 744)
    eps, dt = 2.0 ** -8, 2.0 ** -9
    lam = np.random.default_rng(5).normal(size=(3, n))
    full, least = _sizes(n, prec, 2, 7)
    res = []
    for w in (full, least, (least + 2 * full) // 3):
        xd, vd, md = to_dev(x, v, m, prec)
        acc = torch.empty_like(xd)
        nb.step(xd, vd, md, acc, eps, dt, S, prec=prec)
        lx = torch.tensor(lam, dtype=nb.pos_dtype(prec), device=DEV)
        lv = torch.zeros_like(lx)
        lm = torch.zeros(n, dtype=torch.float64, device=DEV)
        nb.step_adjoint(xd, vd, md, acc, lx, lv, lm, eps, dt, S, prec=prec, entry_half=True,
                        workspace=_ws(w))
        res.append((xd, vd, acc, lx, lv, lm))
    for r in res[1:]:
        for a, b in zip(r, res[0]):
            assert torch.equal(a, b)
    with pytest.raises(NBodyError):
        xd, vd, md = to_dev(x, v, m, prec)
        nb.step_adjoint(xd, vd, md, torch.zeros_like(xd), torch.zeros_like(xd),
                        torch.zeros_like(xd), torch.zeros(n, dtype=torch.float64, device=DEV),
                        eps, dt, 1, prec=prec, workspace=_ws(least - 1))


def test_full_size_default_workspace_bitwise():
    """scale-2^20 as the benchmark runs it: the force pass and an adjoint
    pass with the workspace the library asks for (FP64 running sums and
    bands of 4 GiB) against the same passes with every partial at once (12.9
    and 30 GB): bitwise equal. Times printed."""
    from nbody_inputs import make_state
    prec, eps = "mix_tilec", 2.0 ** -10
    x, v, m = make_state("scale-2^20")
    n = x.shape[1]
    xd, vd, md = to_dev(x, v, m, prec)
    wdef = nb.workspace_size(1, n, prec)
    full, _ = _sizes(n, prec, 1, 3)
    assert wdef < full
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    a_def = nb.accel(xd, md, eps, prec=prec, workspace=_ws(wdef))
    ev[1].record()
    torch.cuda.synchronize()
    ws_full = _ws(full)
    ev[2].record()
    a_full = nb.accel(xd, md, eps, prec=prec, workspace=ws_full)
    ev[3].record()
    torch.cuda.synchronize()
    del ws_full
    print("2^20 force: banded %.1f ms, one band %.1f ms" % (ev[0].elapsed_time(ev[1]),
                                                           ev[2].elapsed_time(ev[3])))
    assert torch.equal(a_def, a_full)
    # one walked-back adjoint pass (force sums) from the same state
    full7, _ = _sizes(n, prec, 2, 7)
    wdef7 = nb.workspace_size(2, n, prec)
    lam = torch.tensor(np.random.default_rng(9).normal(size=(3, n)), device=DEV)
    res = []
    for w in (wdef7, full7):
        xs, vs, accs = xd.clone(), vd.clone(), a_full.clone()
        lx, lv = torch.zeros_like(lam), lam.clone()
        lm = torch.zeros(n, dtype=torch.float64, device=DEV)
        ws = _ws(w)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        nb.step_adjoint(xs, vs, md, accs, lx, lv, lm, eps, 2.0 ** -11, 1, prec=prec, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        print("2^20 adjoint step, workspace %d B: %.1f ms" % (w, e0.elapsed_time(e1)))
        del ws
        res.append((xs, vs, accs, lx, lv, lm))
    for a, b in zip(*res):
        assert torch.equal(a, b)


def test_beyond_one_band_of_partials():
    """2^22 particles: the force pass (blocks of 2048, 103 GB of partials in
    all) and a fused adjoint pass (blocks of 1024, 481 GB in all) in bands of
    4 GiB; sampled rows against the oracle, and the third law on the force."""
    from nbody_inputs import plummer_positions_device
    prec, n, eps = "mix_tilec", 1 << 22, 2.0 ** -11
    xd = plummer_positions_device(n, 751, DEV)
    md = torch.full((n,), 1.0 / n, dtype=torch.float32, device=DEV)
    assert nb.pass_info(1, n, prec)["symmetric"] == 1 and nb.pass_info(2, n, prec)["symmetric"] == 1
    print("2^22 force pass", flush=True)
    a = nb.accel(xd, md, eps, prec=prec)
    xh, mh = host(xd), host(md)
    idx = sample_indices(xh, 256, 32, seed=752)
    ah = host(a)
    e = rel(ah[:, idx], oracle.accel_sampled(xh, mh, eps, idx))
    print("2^22 force: sampled e_glob %.3g" % e, flush=True)
    assert e <= 1e-5
    tot = np.abs((ah * mh).sum(axis=1))
    assert np.all(tot <= 1e-6 * (np.abs(ah) * mh).sum())
    # the entry pass of a reverse walk: J^T lam and G^T lam at x
    print("2^22 adjoint pass", flush=True)
    lam = torch.tensor(np.random.default_rng(753).normal(size=(3, n)), device=DEV)
    lx = torch.zeros_like(lam)
    lm = torch.zeros(n, dtype=torch.float64, device=DEV)
    vd = torch.zeros_like(xd)
    dt = 2.0 ** -12
    nb.step_adjoint(xd, vd, md, a, lx, lam, lm, eps, dt, 0, prec=prec, entry_half=True)
    c = 0.5 * dt
    jt, gt = oracle.vjp_sampled(xh, mh, host(lam), eps, idx)
    ex, em = rel(host(lx)[:, idx] / c, jt), rel(host(lm)[idx] / c, gt)
    print("2^22 adjoint: J^T lam rel err %.3g, G^T lam %.3g" % (ex, em))
    assert ex <= 1e-4 and em <= 1e-4


def test_fp64_adjoint_many_bands():
    """2^21 particles in FP64: the symmetric adjoint's FP64 partials (blocks
    of 1024, 240 GB in all) run as dozens of bands of the 4 GiB default
    workspace; the entry pass's sampled rows against the oracle at the FP64
    bar."""
    from nbody_inputs import plummer_positions_device
    prec, n, eps = "f64", 1 << 21, 2.0 ** -11
    xd = plummer_positions_device(n, 761, DEV).to(torch.float64)
    md = torch.full((n,), 1.0 / n, dtype=torch.float64, device=DEV)
    info = nb.pass_info(2, n, prec)
    assert info["symmetric"] == 1 and info["block_particles"] == 1024
    lam = torch.tensor(np.random.default_rng(762).normal(size=(3, n)), device=DEV)
    lx = torch.zeros_like(lam)
    lm = torch.zeros(n, dtype=torch.float64, device=DEV)
    vd, acc = torch.zeros_like(xd), torch.zeros_like(xd)
    dt = 2.0 ** -12
    print("2^21 FP64 adjoint pass", flush=True)
    nb.step_adjoint(xd, vd, md, acc, lx, lam, lm, eps, dt, 0, prec=prec, entry_half=True)
    c = 0.5 * dt
    xh, mh = host(xd), host(md)
    idx = sample_indices(xh, 256, 32, seed=763)
    jt, gt = oracle.vjp_sampled(xh, mh, host(lam), eps, idx)
    ex, em = rel(host(lx)[:, idx] / c, jt), rel(host(lm)[idx] / c, gt)
    print("2^21 FP64 adjoint: J^T lam rel err %.3g, G^T lam %.3g" % (ex, em))
    assert ex <= 1e-12 and em <= 1e-12
