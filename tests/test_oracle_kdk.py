"""Pins of the oracle's kick-drift-kick leapfrog and its diagnostics.

Closed forms: the softened circular binary (angular frequency
w^2 = G M / (r^2 + eps^2)^(3/2)) and the unsoftened Kepler ellipse solved
from Kepler's equation; second-order convergence (halving dt divides the
error by 4); exact invariants of the scheme (time reversibility, linear and
angular momentum); the two-body energy; the Plummer sphere's virial values.
A wrong half-step weight, a drift with the old velocity or a force sign slip
breaks reversibility, the convergence order or the orbit closed forms.
"""

import numpy as np
import pytest

import oracle
from nbody_inputs import plummer_sphere


def _binary(m1, m2, r, vt):
    """Two bodies on the x axis about their centre of mass, velocities along
    y with relative speed vt."""
    M = m1 + m2
    x = np.array([[-m2 / M * r, m1 / M * r], [0.0, 0.0], [0.0, 0.0]])
    v = np.array([[0.0, 0.0], [-m2 / M * vt, m1 / M * vt], [0.0, 0.0]])
    return x, v, np.array([m1, m2])


def test_circular_binary_second_order():
    m1, m2, r, eps, G = 0.6, 0.4, 1.0, 0.1, 1.0
    M = m1 + m2
    w = np.sqrt(G * M / (r * r + eps * eps) ** 1.5)
    x0, v0, m = _binary(m1, m2, r, w * r)
    period = 2 * np.pi / w
    errs = []
    for nsteps in (128, 256, 512):
        x, v, _ = oracle.kdk(x0, v0, m, eps, period / nsteps, nsteps, G=G)
        errs.append(np.abs(x - x0).max())
    assert errs[0] < 5e-3
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.6 < e1 / e2 < 4.4


def _kepler_relative(t, a, e, GM):
    n = np.sqrt(GM / a ** 3)
    Mean = n * t
    E = Mean.copy() if np.ndim(Mean) else np.array(Mean, dtype=float)
    for _ in range(50):  # Newton on E - e sin E = Mean
        E = E - (E - e * np.sin(E) - Mean) / (1 - e * np.cos(E))
    return np.array([a * (np.cos(E) - e), a * np.sqrt(1 - e * e) * np.sin(E), 0.0])


def test_kepler_ellipse_unsoftened():
    m1 = m2 = 0.5
    a, e, G = 1.0, 0.5, 1.0
    GM = G * (m1 + m2)
    # start at periapsis: r = a (1 - e), v = sqrt(GM (1 + e) / (a (1 - e)))
    x0, v0, m = _binary(m1, m2, a * (1 - e), np.sqrt(GM * (1 + e) / (a * (1 - e))))
    T = 0.7 * 2 * np.pi * np.sqrt(a ** 3 / GM)
    rel = _kepler_relative(T, a, e, GM)
    errs = []
    for nsteps in (400, 800, 1600):
        x, _, _ = oracle.kdk(x0, v0, m, 0.0, T / nsteps, nsteps, G=G)
        errs.append(np.abs((x[:, 1] - x[:, 0]) - rel).max())
    assert errs[-1] < 1e-3
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.6 < e1 / e2 < 4.4


def test_kepler_energy_bounded_no_drift():
    m1 = m2 = 0.5
    a, e = 1.0, 0.5
    x0, v0, m = _binary(m1, m2, a * (1 - e), np.sqrt((1 + e) / (a * (1 - e))))
    period = 2 * np.pi
    per = 128
    _, _, _, tx, tv = oracle.kdk(x0, v0, m, 0.0, period / per, 10 * per, trajectory=True)
    E0 = oracle.diag(tx[0], tv[0], m, 0.0)["E"]
    dE = np.array([oracle.diag(tx[k], tv[k], m, 0.0)["E"] - E0 for k in range(0, 10 * per + 1, 8)])
    first, last = np.abs(dE[: len(dE) // 5]).max(), np.abs(dE[-len(dE) // 5:]).max()
    assert first > 0 and last < 1.5 * first and np.abs(dE).max() < 0.05 * abs(E0)


def test_time_reversibility():
    x0, v0, m = plummer_sphere(256, 21)
    eps, dt, S = 2.0 ** -6, 2.0 ** -7, 10
    x, v, _ = oracle.kdk(x0, v0, m, eps, dt, S)
    xb, vb, _ = oracle.kdk(x, -v, m, eps, dt, S)
    np.testing.assert_allclose(xb, x0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(-vb, v0, rtol=0, atol=1e-12)


def test_momenta_conserved():
    x0, v0, m = plummer_sphere(256, 22)
    # give the system a bulk velocity so P and the COM motion are non-trivial
    v0 = v0 + np.array([[0.3], [-0.1], [0.2]])
    eps, dt, S = 2.0 ** -6, 2.0 ** -7, 20
    d0 = oracle.diag(x0, v0, m, eps)
    x, v, _ = oracle.kdk(x0, v0, m, eps, dt, S)
    d1 = oracle.diag(x, v, m, eps)
    scale = (m * np.abs(v0).sum(axis=0)).sum()
    for k in ("Px", "Py", "Pz"):
        assert abs(d1[k] - d0[k]) < 1e-14 * scale
    lscale = (m * np.linalg.norm(x0, axis=0) * np.linalg.norm(v0, axis=0)).sum()
    for k in ("Lx", "Ly", "Lz"):
        assert abs(d1[k] - d0[k]) < 1e-13 * lscale
    # the centre of mass moves with the constant total momentum
    for c, k in enumerate(("COMx", "COMy", "COMz")):
        assert abs(d1[k] - (d0[k] + S * dt * d0["P" + "xyz"[c]] / d0["M"])) < 1e-13


def test_energy_error_second_order():
    x0, v0, m = plummer_sphere(128, 23)
    eps, T = 2.0 ** -4, 0.25
    E0 = oracle.diag(x0, v0, m, eps)["E"]
    errs = []
    for nsteps in (16, 32, 64):
        x, v, _ = oracle.kdk(x0, v0, m, eps, T / nsteps, nsteps)
        errs.append(abs(oracle.diag(x, v, m, eps)["E"] - E0))
    for e1, e2 in zip(errs, errs[1:]):
        assert 2.5 < e1 / e2 < 6.0


def test_free_particle_and_zero_steps():
    x0 = np.array([[0.5], [0.25], [-1.0]])
    v0 = np.array([[0.125], [-0.5], [2.0]])
    x, v, a = oracle.kdk(x0, v0, np.array([1.0]), 0.1, 2.0 ** -4, 16)
    assert np.array_equal(v, v0) and np.all(a == 0)
    np.testing.assert_allclose(x, x0 + v0, rtol=0, atol=1e-15)
    xs, _, _ = plummer_sphere(32, 24)[0], None, None
    x1, v1, _ = oracle.kdk(xs, np.zeros_like(xs), np.full(32, 1 / 32), 0.1, 0.01, 0)
    assert np.array_equal(x1, xs) and np.all(v1 == 0)


def test_two_body_energy_closed_form():
    # masses 1/4, 1/2 at distance 3 with eps = 4: PE = -G m1 m2 / 5
    x = np.array([[0.0, 3.0], [0.0, 0.0], [0.0, 0.0]])
    v = np.array([[1.0, 0.0], [0.0, -2.0], [0.0, 0.0]])
    m = np.array([0.25, 0.5])
    d = oracle.diag(x, v, m, 4.0, G=2.0)
    assert d["PE"] == pytest.approx(-2.0 * 0.25 * 0.5 / 5.0, rel=1e-15)
    assert d["KE"] == 0.5 * 0.25 * 1.0 + 0.5 * 0.5 * 4.0
    assert d["E"] == pytest.approx(d["KE"] + d["PE"], rel=1e-15)
    assert (d["Px"], d["Py"]) == (0.25, -1.0)
    # L = sum m r x v: only particle 2 has r x v = (3,0,0) x (0,-2,0) = (0,0,-6)
    assert d["Lz"] == 0.5 * -6.0
    assert d["COMx"] == pytest.approx(0.5 * 3.0 / 0.75, rel=1e-15)


def test_angular_momentum_cross_product():
    # one particle: L = m r x v = 2 (1,2,3) x (4,5,6) = 2 (-3, 6, -3)
    d = oracle.diag(np.array([[1.0], [2.0], [3.0]]), np.array([[4.0], [5.0], [6.0]]),
                    np.array([2.0]), 0.1)
    assert (d["Lx"], d["Ly"], d["Lz"]) == (-6.0, 12.0, -6.0)
    assert (d["Px"], d["Py"], d["Pz"]) == (8.0, 10.0, 12.0)
    assert d["KE"] == 0.5 * 2.0 * 77.0 and d["PE"] == 0.0


def test_rigid_rotation_angular_momentum():
    k, R, w = 12, 0.7, 1.5
    phi = 2 * np.pi * np.arange(k) / k
    x = np.stack([R * np.cos(phi), R * np.sin(phi), np.zeros(k)])
    v = np.stack([-w * x[1], w * x[0], np.zeros(k)])
    m = np.full(k, 1.0 / k)
    d = oracle.diag(x, v, m, 0.1)
    assert d["Lz"] == pytest.approx(R * R * w, rel=1e-14)
    assert abs(d["Lx"]) < 1e-16 and abs(d["Ly"]) < 1e-16


@pytest.mark.slow
def test_plummer_virial_values():
    # Untruncated Plummer sphere with G = M = a = 1: W = -3 pi / 32,
    # K = 3 pi / 64, E = -3 pi / 64 and 2K / |W| = 1. The truncation at
    # r = 10 and the softening move the sample by a few per cent at most.
    x, v, m = plummer_sphere(8192, 31)
    d = oracle.diag(x, v, m, 2.0 ** -8)
    assert d["PE"] == pytest.approx(-3 * np.pi / 32, rel=0.04)
    assert d["KE"] == pytest.approx(3 * np.pi / 64, rel=0.04)
    assert 2 * d["KE"] / abs(d["PE"]) == pytest.approx(1.0, abs=0.05)


def test_high_precision_kdk_brute_force():
    # Ten steps of the same scheme carried out at 50 significant digits: the
    # oracle's FP64 trajectory stays within rounding of it.
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    x, v, m = plummer_sphere(8, 23)
    eps, dt, S = 2.0 ** -3, 2.0 ** -6, 10
    n = x.shape[1]
    mf = [mpmath.mpf(float(q)) for q in m]
    e2 = mpmath.mpf(eps) ** 2

    def acc(X):
        out = [[mpmath.mpf(0)] * n for _ in range(3)]
        for i in range(n):
            for j in range(n):
                if j != i:
                    d = [X[c][j] - X[c][i] for c in range(3)]
                    w = mf[j] / (d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + e2) ** mpmath.mpf(1.5)
                    for c in range(3):
                        out[c][i] += w * d[c]
        return out

    X = [[mpmath.mpf(float(q)) for q in row] for row in x]
    V = [[mpmath.mpf(float(q)) for q in row] for row in v]
    h, dtm = mpmath.mpf(dt) / 2, mpmath.mpf(dt)
    A = acc(X)
    for _ in range(S):
        V = [[V[c][i] + h * A[c][i] for i in range(n)] for c in range(3)]
        X = [[X[c][i] + dtm * V[c][i] for i in range(n)] for c in range(3)]
        A = acc(X)
        V = [[V[c][i] + h * A[c][i] for i in range(n)] for c in range(3)]
    xo, vo, _ = oracle.kdk(x, v, m, eps, dt, S)
    xr = np.array([[float(q) for q in row] for row in X])
    vr = np.array([[float(q) for q in row] for row in V])
    assert np.max(np.abs(xo - xr)) <= 1e-14 * np.max(np.abs(xr))
    assert np.max(np.abs(vo - vr)) <= 1e-13 * np.max(np.abs(vr))
