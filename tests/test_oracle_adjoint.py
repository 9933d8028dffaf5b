"""Pins of the oracle's Jacobian products and reverse-mode KDK gradient.

* J u against central differences of the force itself (oracle.accel), and
  the adjoint identity <J u, lam> = <u, J^T lam> tying the two code paths;
* G^T lam against the exact linearity of Eq. (1) in the source masses;
* translation invariance: sum_k (J^T lam)_k = 0 and J^T (m (x) e) = 0;
* the full rollout gradient against central differences of the oracle's own
  forward run, and against torch.autograd (CPU, FP64) of a separately written
  dense tensor formula.
"""

import numpy as np
import pytest

import oracle
from nbody_inputs import plummer_sphere


def _setup(n, seed):
    x, v, m = plummer_sphere(n, seed)
    rng = np.random.default_rng(seed + 100)
    m = m * rng.uniform(0.5, 1.5, size=n)  # unequal masses
    return x, v, m


def test_jvp_matches_central_differences():
    x, _, m = _setup(24, 41)
    eps = 2.0 ** -4
    u = np.random.default_rng(1).normal(size=x.shape)
    h = 1e-6
    fd = (oracle.accel(x + h * u, m, eps) - oracle.accel(x - h * u, m, eps)) / (2 * h)
    ju = oracle.jvp(x, m, u, eps)
    np.testing.assert_allclose(ju, fd, rtol=0, atol=1e-7 * np.abs(fd).max())


def test_vjp_adjoint_identity():
    x, _, m = _setup(40, 42)
    eps = 2.0 ** -5
    rng = np.random.default_rng(2)
    u, lam = rng.normal(size=x.shape), rng.normal(size=x.shape)
    jt, _ = oracle.vjp(x, m, lam, eps)
    ju = oracle.jvp(x, m, u, eps)
    lhs, rhs = np.sum(ju * lam), np.sum(u * jt)
    assert abs(lhs - rhs) <= 1e-13 * (np.abs(ju * lam).sum())


def test_mass_vjp_is_exact_linearity():
    # a(x; w) is linear in the source masses w, so <lam, a(x; w)> = <G^T lam, w>.
    x, _, m = _setup(30, 43)
    eps = 2.0 ** -5
    rng = np.random.default_rng(3)
    lam, w = rng.normal(size=x.shape), rng.normal(size=m.shape)
    _, gt = oracle.vjp(x, m, lam, eps, G=1.5)
    lhs = np.sum(lam * oracle.accel(x, w, eps, G=1.5))
    assert abs(lhs - gt @ w) <= 1e-13 * np.abs(gt * w).sum()


def test_vjp_translation_invariance():
    x, _, m = _setup(50, 44)
    eps = 2.0 ** -5
    lam = np.random.default_rng(4).normal(size=x.shape)
    jt, _ = oracle.vjp(x, m, lam, eps)
    assert np.all(np.abs(jt.sum(axis=1)) <= 1e-13 * np.abs(jt).sum())
    # lam_i = m_i e makes every pair term m_k m_i e - m_i m_k e vanish
    e = np.array([[0.3], [-1.2], [0.7]])
    jt2, _ = oracle.vjp(x, m, m * e, eps)
    jt_ref, _ = oracle.vjp(x, m, np.random.default_rng(5).normal(size=x.shape) * m, eps)
    assert np.abs(jt2).max() <= 1e-13 * np.abs(jt_ref).max()


def _loss_and_grads(x0, v0, m, eps, dt, S, y):
    n = x0.shape[1]
    x, v, _, tx, _ = oracle.kdk(x0, v0, m, eps, dt, S, trajectory=True)
    L = np.sum((x - y) ** 2) / n
    gx, gv, gm = oracle.adjoint(tx, m, eps, dt, 2.0 / n * (x - y), np.zeros_like(v))
    return L, gx, gv, gm


def _loss(x0, v0, m, eps, dt, S, y):
    x, _, _ = oracle.kdk(x0, v0, m, eps, dt, S)
    return np.sum((x - y) ** 2) / x0.shape[1]


def test_rollout_gradient_vs_central_differences():
    n, S = 16, 8
    x0, v0, m = _setup(n, 45)
    eps, dt = 2.0 ** -3, 2.0 ** -5
    rng = np.random.default_rng(5)
    y = x0 + 0.1 * rng.normal(size=x0.shape)
    L, gx, gv, gm = _loss_and_grads(x0, v0, m, eps, dt, S, y)
    h = 1e-6
    for k in range(4):
        ux, uv, um = rng.normal(size=x0.shape), rng.normal(size=v0.shape), rng.normal(size=m.shape)
        fx = (_loss(x0 + h * ux, v0, m, eps, dt, S, y) - _loss(x0 - h * ux, v0, m, eps, dt, S, y)) / (2 * h)
        fv = (_loss(x0, v0 + h * uv, m, eps, dt, S, y) - _loss(x0, v0 - h * uv, m, eps, dt, S, y)) / (2 * h)
        fm = (_loss(x0, v0, m + h * um * m, eps, dt, S, y) - _loss(x0, v0, m - h * um * m, eps, dt, S, y)) / (2 * h)
        assert np.sum(gx * ux) == pytest.approx(fx, rel=1e-6, abs=1e-10)
        assert np.sum(gv * uv) == pytest.approx(fv, rel=1e-6, abs=1e-10)
        assert np.sum(gm * um * m) == pytest.approx(fm, rel=1e-6, abs=1e-10)


def test_rollout_gradient_vs_torch_autograd():
    torch = pytest.importorskip("torch")
    n, S = 12, 5
    x0, v0, m = _setup(n, 46)
    eps, dt, G = 2.0 ** -3, 2.0 ** -5, 1.25
    y = x0 + 0.05 * np.random.default_rng(6).normal(size=x0.shape)
    x, v, _, tx, _ = oracle.kdk(x0, v0, m, eps, dt, S, G=G, trajectory=True)
    gx, gv, gm = oracle.adjoint(tx, m, eps, dt, 2.0 / n * (x - y), np.zeros_like(v), G=G)

    # dense (n, n, 3) formulation, written independently of the oracle
    X = torch.tensor(x0.T.copy(), dtype=torch.float64, requires_grad=True)
    V = torch.tensor(v0.T.copy(), dtype=torch.float64, requires_grad=True)
    Mt = torch.tensor(m, dtype=torch.float64, requires_grad=True)
    Y = torch.tensor(y.T.copy(), dtype=torch.float64)
    off = 1.0 - torch.eye(n, dtype=torch.float64)

    def acc(P):
        D = P[None, :, :] - P[:, None, :]            # D[i, j] = r_j - r_i
        s = (D * D).sum(-1) + eps * eps
        W = off * Mt[None, :] * s ** -1.5
        return G * (W[:, :, None] * D).sum(1)

    P, U = X, V
    A = acc(P)
    for _ in range(S):
        U = U + 0.5 * dt * A
        P = P + dt * U
        A = acc(P)
        U = U + 0.5 * dt * A
    L = ((P - Y) ** 2).sum() / n
    L.backward()
    np.testing.assert_allclose(gx, X.grad.numpy().T, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(gv, V.grad.numpy().T, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(gm, Mt.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_adjoint_position_sum_invariant():
    # J^T lam sums to zero over particles, so every position-adjoint update
    # leaves sum_i lamx_i unchanged: sum lamx_0 = sum lamx_S, and
    # sum lamv_0 = sum lamv_S + S dt sum lamx_S.
    n, S = 20, 6
    x0, v0, m = _setup(n, 47)
    eps, dt = 2.0 ** -4, 2.0 ** -6
    _, _, _, tx, _ = oracle.kdk(x0, v0, m, eps, dt, S, trajectory=True)
    rng = np.random.default_rng(7)
    lx, lv = rng.normal(size=x0.shape), rng.normal(size=x0.shape)
    gx, gv, _ = oracle.adjoint(tx, m, eps, dt, lx, lv)
    np.testing.assert_allclose(gx.sum(axis=1), lx.sum(axis=1), rtol=0, atol=1e-12)
    np.testing.assert_allclose(gv.sum(axis=1), lv.sum(axis=1) + S * dt * lx.sum(axis=1),
                               rtol=0, atol=1e-12)


def test_vjp_sampled_rows_are_vjp_rows():
    # the sampled form evaluates the same rows with the same arithmetic
    x, v, m = plummer_sphere(300, 41)
    lam = np.random.default_rng(2).normal(size=(3, 300))
    jt, gt = oracle.vjp(x, m, lam, 2.0 ** -5, G=1.5)
    idx = np.array([299, 0, 17, 17, 150])
    js, gs = oracle.vjp_sampled(x, m, lam, 2.0 ** -5, idx, G=1.5)
    assert np.array_equal(js, jt[:, idx]) and np.array_equal(gs, gt[idx])
