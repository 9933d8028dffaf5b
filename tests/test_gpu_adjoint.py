"""GPU parity of the hand-written adjoint (fused adjoint pair kernel and the
reverse KDK walk with checkpoints) against the oracle's FP64 reverse-mode
gradient, which stores the whole trajectory and shares nothing with the
GPU's reconstruction schedule."""

import numpy as np
import pytest
import torch

import oracle
import paper_2411_18889_amd as nb
from nbody_inputs import plummer_sphere
from tests.gpu_util import DEV, host, rel, to_dev


pytestmark = pytest.mark.gpu


def _problem(n, seed):
    x, v, m = plummer_sphere(n, seed)
    m = m * np.random.default_rng(seed).uniform(0.5, 1.5, size=n)
    y = x + 0.05 * np.random.default_rng(seed + 1).normal(size=x.shape)
    return x, v, m, y


def _oracle_grads(x, v, m, y, eps, dt, S):
    n = x.shape[1]
    xs, _, _, tx, _ = oracle.kdk(x, v, m, eps, dt, S, trajectory=True)
    return oracle.adjoint(tx, m, eps, dt, 2.0 / n * (xs - y), np.zeros_like(v))


def _gpu_grads(x, v, m, y, eps, dt, S, K, prec):
    xd, vd, md = to_dev(x, v, m, prec)
    xd.requires_grad_(True)
    vd.requires_grad_(True)
    md.requires_grad_(True)
    xs, vs = nb.rollout(xd, vd, md, eps, dt, S, ckpt_every=K, prec=prec)
    yd = torch.tensor(y, dtype=xs.dtype, device=DEV)
    loss = ((xs - yd) ** 2).sum() / x.shape[1]
    loss.backward()
    return host(xd.grad), host(vd.grad), host(md.grad), (host(xd), host(vd), host(md))


@pytest.mark.parametrize("n,S,K", [(64, 6, 2), (300, 12, 5), (1000, 9, 20), (12288 + 5, 3, 2),
                                   (40000 + 77, 2, 1)])
def test_adjoint_f64_matches_oracle(n, S, K):
    """Up to 1000 particles the one-sided kernel; from 12288 the symmetric
    pass (FP64 partials; 40077: four waves of two sinks per lane, blocks of
    512)."""
    x, v, m, y = _problem(n, 60 + n)
    eps, dt = 2.0 ** -5, 2.0 ** -7
    gx, gv, gm, _ = _gpu_grads(x, v, m, y, eps, dt, S, K, "f64")
    ox, ov, om = _oracle_grads(x, v, m, y, eps, dt, S)
    assert rel(gx, ox) <= 1e-10
    assert rel(gv, ov) <= 1e-10
    assert rel(gm, om) <= 1e-10


def test_gradcheck_f64_rollout():
    """torch.autograd.gradcheck of the FP64 rollout: the hand-written adjoint
    against central differences of the GPU's own forward."""
    n, S = 8, 3
    x, v, m, _ = _problem(n, 83)
    xd, vd, md = to_dev(x, v, m, "f64")
    for t in (xd, vd, md):
        t.requires_grad_(True)

    def f(a, b, c):
        xs, vs = nb.rollout(a, b, c, 2.0 ** -3, 2.0 ** -5, S, ckpt_every=2, prec="f64")
        return xs, vs

    assert torch.autograd.gradcheck(f, (xd, vd, md), eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("prec", ("mix_tilec", "mix_acc64", "mix_kahan", "mix_acc32", "f32"))
def test_adjoint_fp32_pairs_matches_oracle(prec):
    n, S, K = 2048, 40, 20
    x, v, m, y = _problem(n, 70)
    eps, dt = 2.0 ** -7, 2.0 ** -8
    gx, gv, gm, (x0, v0, m0) = _gpu_grads(x, v, m, y, eps, dt, S, K, prec)
    ox, ov, om = _oracle_grads(x0, v0, m0, y, eps, dt, S)
    errs = (rel(gx, ox), rel(gv, ov), rel(gm, om))
    print(prec, "gradient rel err x0 %.3g v0 %.3g m %.3g" % errs)
    assert max(errs) <= 1e-4


@pytest.mark.parametrize("n,prec", [(12288 + 5, "mix_tilec"), (16384 + 300, "mix_tilec"),
                                    (32768, "mix_tilec"), (32768 + 300, "mix_tilec"),
                                    (12288 + 5, "f32"), (32768 + 300, "f32")])
def test_adjoint_symmetric_pass_matches_oracle(n, prec):
    """From 12288 particles on, the tile-compensated (and the plain FP32)
    policy walks back with the symmetric (third-law) adjoint pass: blocks of
    n/64, ragged last blocks. Checked against the oracle's gradient and
    (tile-compensated) against the one-sided kernel of the FP64-summed
    policy on every particle."""
    S, K = 3, 2
    x, v, m, y = _problem(n, 90 + n % 7)
    eps, dt = 2.0 ** -7, 2.0 ** -8
    gx, gv, gm, (x0, v0, m0) = _gpu_grads(x, v, m, y, eps, dt, S, K, prec)
    ox, ov, om = _oracle_grads(x0, v0, m0, y, eps, dt, S)
    errs = (rel(gx, ox), rel(gv, ov), rel(gm, om))
    print("n=%d %s symmetric adjoint gradient rel err x0 %.3g v0 %.3g m %.3g"
          % ((n, prec) + errs))
    assert max(errs) <= 1e-4
    if prec != "mix_tilec":
        return
    cx, cv, cm, _ = _gpu_grads(x, v, m, y, eps, dt, S, K, "mix_acc64")
    assert rel(gx, cx) <= 1e-5 and rel(gv, cv) <= 1e-5 and rel(gm, cm) <= 1e-4


@pytest.mark.parametrize("n", (163840 + 3, 600_000, 1 << 20, (1 << 21) + 3))
def test_adjoint_symmetric_large_blocks(n):
    """Blocks of 1024 (4 waves x 4 sinks) from 163840 + 3 and at 600,000 (a
    ragged last block), 2^20 and 2^21 + 3, whose partials (30 and 120 GB in
    all) are folded in bands of the default workspace: one step forward and
    back, against the one-sided kernel with the FP64-summed policy on every
    particle."""
    S, K = 1, 1
    x, v, m, y = _problem(n, 95)
    eps, dt = 2.0 ** -10, 2.0 ** -11
    gx, gv, gm, _ = _gpu_grads(x, v, m, y, eps, dt, S, K, "mix_tilec")
    cx, cv, cm, _ = _gpu_grads(x, v, m, y, eps, dt, S, K, "mix_acc64")
    errs = (rel(gx, cx), rel(gv, cv), rel(gm, cm))
    print("n=%d symmetric vs one-sided adjoint: x0 %.3g v0 %.3g m %.3g" % ((n,) + errs))
    assert errs[0] <= 1e-5 and errs[1] <= 1e-5 and errs[2] <= 1e-4


def test_checkpoint_interval_invariance():
    n, S = 512, 12
    x, v, m, y = _problem(n, 80)
    eps, dt = 2.0 ** -6, 2.0 ** -7
    res = [_gpu_grads(x, v, m, y, eps, dt, S, K, "f64")[:3] for K in (1, 4, 5, 12, 100)]
    for r in res[1:]:
        for a, b in zip(r, res[0]):
            assert rel(a, b) <= 1e-12


def test_auto_checkpoint_interval_is_every_step_when_it_fits():
    """ckpt_every="auto" at a size whose per-step checkpoints fit: bitwise
    the gradients of ckpt_every=1 (symmetric passes, tile-compensated)."""
    n, S = 20000, 4
    x, v, m, y = _problem(n, 81)
    eps, dt = 2.0 ** -7, 2.0 ** -8
    a = _gpu_grads(x, v, m, y, eps, dt, S, "auto", "mix_tilec")[:3]
    b = _gpu_grads(x, v, m, y, eps, dt, S, 1, "mix_tilec")[:3]
    for p, q in zip(a, b):
        assert np.array_equal(p, q)


def test_split_calls_equal_one_call():
    """Three nbody_step_adjoint calls over consecutive spans (flags
    ENTRY_HALF / EXIT_FULL) give the same gradient as the oracle."""
    n, S = 256, 9
    x, v, m, y = _problem(n, 81)
    eps, dt = 2.0 ** -6, 2.0 ** -7
    xd, vd, md = to_dev(x, v, m, "f64")
    acc = torch.empty_like(xd)
    nb.step(xd, vd, md, acc, eps, dt, S, prec="f64")
    lx = (2.0 / n) * (xd - torch.tensor(y, device=DEV))
    lv = torch.zeros_like(vd)
    lm = torch.zeros(n, dtype=torch.float64, device=DEV)
    spans = [(3, True, True), (4, False, True), (2, False, False)]
    for ns, entry, exit_full in spans:
        nb.step_adjoint(xd, vd, md, acc, lx, lv, lm, eps, dt, ns, prec="f64",
                        entry_half=entry, exit_full=exit_full)
    ox, ov, om = _oracle_grads(x, v, m, y, eps, dt, S)
    assert rel(host(lx), ox) <= 1e-10 and rel(host(lv), ov) <= 1e-10 and rel(host(lm), om) <= 1e-10
    # and the state has been walked back to the initial one
    assert float((xd - torch.tensor(x, device=DEV)).abs().max()) <= 1e-12


@pytest.mark.parametrize("n", (4096, 40000))
def test_position_adjoint_sum_invariant_on_gpu(n):
    S = 8
    x, v, m, _ = _problem(n, 82)
    eps, dt = 2.0 ** -7, 2.0 ** -8
    xd, vd, md = to_dev(x, v, m, "mix_tilec")
    acc = torch.empty_like(xd)
    nb.step(xd, vd, md, acc, eps, dt, S, prec="mix_tilec")
    rng = np.random.default_rng(3)
    lx0 = rng.normal(size=(3, n))
    lv0 = rng.normal(size=(3, n))
    lx = torch.tensor(lx0, device=DEV)
    lv = torch.tensor(lv0, device=DEV)
    lm = torch.zeros(n, dtype=torch.float64, device=DEV)
    nb.step_adjoint(xd, vd, md, acc, lx, lv, lm, eps, dt, S, prec="mix_tilec", entry_half=True)
    # the position-adjoint updates cancel in the sum up to the FP32 rounding
    # of the pair terms: bound the residual by 1e-5 of their total size
    dlx = host(lx) - lx0
    scale = np.abs(dlx).sum(axis=1)
    assert np.all(np.abs(dlx.sum(axis=1)) <= 1e-5 * scale), (dlx.sum(axis=1), scale)
    expect_lv = lv0.sum(axis=1) + S * dt * lx0.sum(axis=1)
    assert np.all(np.abs(host(lv).sum(axis=1) - expect_lv) <= 1e-5 * S * dt * scale + 1e-9)


def test_adjoint_symmetric_pass_bitwise_reproducible():
    """The symmetric adjoint pass sums in a fixed order (no atomics): the
    same walk twice gives bitwise the same adjoints and state."""
    n, S = 40000, 2
    x, v, m, _ = _problem(n, 97)
    eps, dt = 2.0 ** -8, 2.0 ** -9
    xd, vd, md = to_dev(x, v, m, "mix_tilec")
    acc = torch.empty_like(xd)
    nb.step(xd, vd, md, acc, eps, dt, S, prec="mix_tilec")
    lam = torch.tensor(np.random.default_rng(5).normal(size=(3, n)), device=DEV)
    outs = []
    for _ in range(2):
        st = [t.clone() for t in (xd, vd, acc)]
        lx, lv = lam.clone(), torch.zeros_like(lam)
        lm = torch.zeros(n, dtype=torch.float64, device=DEV)
        nb.step_adjoint(st[0], st[1], md, st[2], lx, lv, lm, eps, dt, S, prec="mix_tilec",
                        entry_half=True)
        outs.append((lx, lv, lm, st[0], st[1]))
    assert nb.pass_info(2, n, "mix_tilec")["symmetric"] == 1
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_adjoint_symmetric_checkpoint_interval_invariance():
    """Symmetric adjoint pass: with a checkpoint every step every pass reloads
    the state and skips the force sums (the force-free kernels); with one
    every 3 steps most passes walk the state back with the force. The
    gradients agree to the reconstruction's rounding."""
    n, S = 40000, 6
    x, v, m, y = _problem(n, 98)
    eps, dt = 2.0 ** -8, 2.0 ** -9
    assert nb.pass_info(2, n, "mix_tilec")["symmetric"] == 1
    res = [_gpu_grads(x, v, m, y, eps, dt, S, K, "mix_tilec")[:3] for K in (1, 3, 100)]
    for r in res[1:]:
        for a, b in zip(r, res[0]):
            assert rel(a, b) <= 1e-7


@pytest.mark.parametrize("prec", ("mix_tilec", "f64", "f32"))
@pytest.mark.parametrize("walk", (False, True))
def test_adjoint_pass_full_size_against_oracle_rows(walk, prec):
    """scale-2^20, in the launch configuration the benchmark times (and the
    FP64 and FP32 policies' symmetric passes at the same size): one fused
    adjoint pass against the oracle's transposed Jacobians on sampled rows.
    walk = False: the entry pass (state from the caller, force sums skipped);
    walk = True: one step walked back with a tiny dt, so the pass also
    computes a(x) and steps the velocity (the force-summing kernel); the
    oracle then takes the walked-back state the call leaves."""
    from nbody_inputs import make_state
    from tests.gpu_util import sample_indices
    x, v, m = make_state("scale-2^20")
    n = x.shape[1]
    eps, G = 2.0 ** -10, 1.0
    xd, vd, md = to_dev(x, v, m, prec)
    assert nb.pass_info(2, n, prec)["symmetric"] == 1
    acc = nb.accel(xd, md, eps, prec=prec)
    lam = torch.tensor(np.random.default_rng(11).normal(size=(3, n)), dtype=nb.pos_dtype(prec),
                       device=DEV)
    lx = torch.zeros_like(lam)
    lm = torch.zeros(n, dtype=torch.float64, device=DEV)
    if walk:
        dt = 2.0 ** -24
        h = 0.5 * dt
        nb.step_adjoint(xd, vd, md, acc, lx, lam, lm, eps, dt, 1, G=G, prec=prec)
        c = h  # the last (and only) pass of a walk ending at step 0
    else:
        dt = 2.0 ** -11
        nb.step_adjoint(xd, vd, md, acc, lx, lam, lm, eps, dt, 0, G=G, prec=prec,
                        entry_half=True)
        c = 0.5 * dt
    xw = host(xd)  # the state the pass saw
    idx = sample_indices(xw, 256, 32, seed=12)
    jt, gt = oracle.vjp_sampled(xw, host(md), host(lam), eps, idx, G=G)
    ex = rel(host(lx)[:, idx] / c, jt)
    em = rel(host(lm)[idx] / c, gt)
    print("scale-2^20 %s adjoint pass (walk=%s): J^T lam rel err %.3g, G^T lam %.3g"
          % (prec, walk, ex, em))
    tol = 1e-12 if prec == "f64" else 1e-4
    assert ex <= tol and em <= tol
    if walk:  # the pass also left a(x) of the walked-back state
        ea = rel(host(acc)[:, idx], oracle.accel_sampled(xw, host(md), eps, idx))
        assert ea <= (1e-12 if prec == "f64" else 1e-5)


_SYM_ADJ = [(2, 128), (2, 256), (2, 512), (2, 1024), (1, 256), (1, 512), (4, 128), (4, 256),
            (4, 512)]


@pytest.mark.parametrize("prec,ipl,block", [("f64",) + s for s in _SYM_ADJ if s[1] <= 512] +
                         [("f32",) + s for s in _SYM_ADJ])
def test_adjoint_symmetric_pass_fp64_fp32(prec, ipl, block):
    """The symmetric adjoint pass in the FP64 and plain FP32 policies, in
    every shape the library has for them (20037 particles: ragged last
    blocks; FP64 not in 16-wave workgroups): the entry pass against the
    oracle's transposed Jacobians and against the one-sided kernel, then one
    walked-back step (a pass with the force sums) against the oracle's a(x)
    of the walked-back state."""
    n, eps, dt = 20000 + 37, 2.0 ** -8, 2.0 ** -9
    x, v, m = plummer_sphere(n, 903)
    xd, vd, md = to_dev(x, v, m, prec)
    pdt = nb.pos_dtype(prec)
    lam = torch.tensor(np.random.default_rng(904).normal(size=(3, n)), dtype=pdt, device=DEV)
    acc = nb.accel(xd, md, eps, prec=prec)
    sym = {"i_per_lane": ipl, "block": block, "split": 0, "symmetric": 1}
    one = {"i_per_lane": 1, "block": 256, "split": 8, "symmetric": 0}
    out = []
    for launch in (sym, one):
        lx = torch.zeros_like(lam)
        lm = torch.zeros(n, dtype=torch.float64, device=DEV)
        nb.step_adjoint(xd, vd, md, acc, lx, lam.clone(), lm, eps, dt, 0, prec=prec,
                        entry_half=True, launch=launch)
        out.append((host(lx), host(lm)))
    jt, gt = oracle.vjp(host(xd), host(md), host(lam), eps)
    c = 0.5 * dt
    (sx, sm), (ox, om) = out
    errs = (rel(sx / c, jt), rel(sm / c, gt), rel(ox / c, jt), rel(om / c, gt))
    print("%s %dx%d: symmetric J^T lam %.3g, G^T lam %.3g; one-sided %.3g, %.3g"
          % ((prec, ipl, block) + errs))
    tol = 1e-12 if prec == "f64" else 1e-4
    assert max(errs[:2]) <= tol
    if prec == "f64":
        assert rel(sx, ox) <= 1e-13 and rel(sm, om) <= 1e-13
    h = 0.5 * dt
    xw = host(xd) - dt * (host(vd) - h * host(acc))
    nb.step_adjoint(xd, vd, md, acc, torch.zeros_like(lam), lam.clone(),
                    torch.zeros(n, dtype=torch.float64, device=DEV), eps, dt, 1, prec=prec,
                    launch=sym)
    assert rel(host(acc), oracle.accel(xw, host(md), eps)) <= (1e-12 if prec == "f64" else 1e-5)
