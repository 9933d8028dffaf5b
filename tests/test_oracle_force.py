"""Pins of the oracle's force and potential (Eq. (1), section "N-body
simulation") against closed forms, symmetries and exact scaling identities.

Each check is chosen so that a plausible slip in the oracle fails it: a wrong
sign of r_j - r_i fails the two-body, ring and harmonic-limit cases, a wrong
exponent of (|d|^2 + eps^2) fails the exact scaling identities, a missing or
doubled mass factor fails the mass scaling and the two-body case, a dropped
component fails the triangle and ring cases.
"""

import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            key, *rest = line.split()
            vals[key] = [float(Fraction(t)) for t in rest]
    return vals


def test_two_body_closed_form():
    g = _read_golden("two_body_eq1.txt")
    x = np.array([g["r1"], g["r2"]]).T
    m = np.array([g["m1"][0], g["m2"][0]])
    a, phi = oracle.accel(x, m, g["eps"][0], G=g["G"][0], potential=True)
    np.testing.assert_allclose(a[:, 0], g["a1"], rtol=1e-15, atol=0)
    np.testing.assert_allclose(a[:, 1], g["a2"], rtol=1e-15, atol=0)
    np.testing.assert_allclose(phi, [g["phi1"][0], g["phi2"][0]], rtol=1e-15)


@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_equilateral_triangle(eps):
    # side l, equal masses, centroid at the origin: every |a_i| equals
    # sqrt(3) G m l / (l^2 + eps^2)^(3/2) and points at the centroid.
    l, mass, G = 1.7, 0.4, 1.3
    ang = np.array([0.0, 2 * np.pi / 3, 4 * np.pi / 3]) + 0.25
    R = l / np.sqrt(3.0)
    x = np.stack([R * np.cos(ang), R * np.sin(ang), np.zeros(3)])
    a = oracle.accel(x, np.full(3, mass), eps, G=G)
    expect = np.sqrt(3.0) * G * mass * l / (l * l + eps * eps) ** 1.5
    np.testing.assert_allclose(np.linalg.norm(a, axis=0), expect, rtol=1e-14)
    unit_to_centroid = -x / np.linalg.norm(x, axis=0)
    np.testing.assert_allclose(a / np.linalg.norm(a, axis=0), unit_to_centroid, atol=1e-14)


@pytest.mark.parametrize("k", [3, 8, 13])
def test_ring_on_axis(k):
    # k equal masses on a ring of radius R in the z = 0 plane; a sink on the
    # axis at height z feels -k m z / (R^2 + z^2 + eps^2)^(3/2) along z and
    # nothing in the plane.
    R, z, mass, eps, G = 0.8, 0.6, 0.125, 0.2, 1.0
    phi = 2 * np.pi * np.arange(k) / k + 0.1
    xj = np.stack([R * np.cos(phi), R * np.sin(phi), np.zeros(k)])
    xi = np.array([[0.0], [0.0], [z]])
    a = oracle.accel(xi, np.full(k, mass), eps, G=G, xj=xj)
    expect_z = -k * mass * z / (R * R + z * z + eps * eps) ** 1.5
    np.testing.assert_allclose(a[2, 0], expect_z, rtol=1e-14)
    assert abs(a[0, 0]) < 1e-15 and abs(a[1, 0]) < 1e-15


def test_harmonic_limit_large_softening():
    # For eps >> |d|, each term tends to m_j d / eps^3, so
    # a_i -> G (sum_j m_j r_j - M r_i) / eps^3 with relative corrections of
    # order |d|^2 / eps^2.
    rng = np.random.default_rng(7)
    n = 9
    x = rng.uniform(-1, 1, size=(3, n))
    m = rng.uniform(0.5, 1.5, size=n)
    eps = 1e4
    a = oracle.accel(x, m, eps)
    com_term = (x @ m)[:, None] - m.sum() * x  # includes the zero j = i term
    expect = com_term / eps ** 3
    np.testing.assert_allclose(a, expect, rtol=0, atol=1e-7 * np.abs(expect).max())
    # and the sign: every sink is pulled towards the others' centre of mass
    assert np.all(np.sign(a) == np.sign(expect))


def test_single_particle_zero():
    a = oracle.accel(np.array([[0.3], [0.1], [-2.0]]), np.array([5.0]), 0.1)
    assert np.all(a == 0.0)


def _plummer(n, seed):
    from nbody_inputs import plummer_sphere
    return plummer_sphere(n, seed)


def test_newton_third_law():
    x, _, m = _plummer(512, 11)
    a = oracle.accel(x, m, 2.0 ** -6)
    total = (a * m).sum(axis=1)
    scale = (np.abs(a) * m).sum()
    assert np.all(np.abs(total) <= 1e-14 * scale)


def test_exact_scaling_identities():
    # Powers of two scale every operation exactly, so these hold bitwise:
    #   a(2x, 2eps) = a(x, eps) / 4   (the -3/2 power of the squared length)
    #   a(x, 2m)    = 2 a(x, m)       (linear in the source masses)
    #   phi(2x, 2eps) = phi / 2,  phi(x, 2m) = 2 phi
    x, _, m = _plummer(300, 12)
    eps = 2.0 ** -5
    a, phi = oracle.accel(x, m, eps, potential=True)
    a2, phi2 = oracle.accel(2 * x, m, 2 * eps, potential=True)
    assert np.array_equal(a2, a / 4) and np.array_equal(phi2, phi / 2)
    a3, phi3 = oracle.accel(x, 2 * m, eps, potential=True)
    assert np.array_equal(a3, 2 * a) and np.array_equal(phi3, 2 * phi)


def test_translation_and_permutation():
    x, _, m = _plummer(256, 13)
    eps = 2.0 ** -6
    a = oracle.accel(x, m, eps)
    shift = np.array([[0.25], [-0.5], [0.125]])
    np.testing.assert_allclose(oracle.accel(x + shift, m, eps), a, rtol=1e-11, atol=1e-12)
    perm = np.random.default_rng(3).permutation(x.shape[1])
    ap = oracle.accel(x[:, perm], m[perm], eps)
    np.testing.assert_allclose(ap, a[:, perm], rtol=1e-12, atol=1e-13)


def test_force_is_minus_gradient_of_potential():
    # phi_i as a function of r_i alone has gradient -a_i (central differences).
    x, _, m = _plummer(64, 14)
    eps = 2.0 ** -4
    a = oracle.accel(x, m, eps)
    h = 1e-5
    for i in (0, 17, 63):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[c, i] += h
            xm[c, i] -= h
            _, pp = oracle.accel(xp, m, eps, potential=True)
            _, pm = oracle.accel(xm, m, eps, potential=True)
            grad = (pp[i] - pm[i]) / (2 * h)
            assert abs(grad + a[c, i]) <= 1e-7 * max(1.0, abs(a[c, i]))


def test_sampled_matches_full():
    x, _, m = _plummer(400, 15)
    eps = 2.0 ** -6
    a, phi = oracle.accel(x, m, eps, potential=True)
    idx = np.array([0, 5, 399, 123])
    s, sp = oracle.accel_sampled(x, m, eps, idx, potential=True)
    assert np.array_equal(s, a[:, idx]) and np.array_equal(sp, phi[idx])


def test_thread_count_independent():
    # OpenMP splits only the sink loop, so results are bitwise identical
    # whatever the thread count; run the same call in a 1-thread process.
    import subprocess, sys, json
    x, _, m = _plummer(200, 16)
    a = oracle.accel(x, m, 2.0 ** -6)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import json,sys; sys.path.insert(0, %r); import numpy as np, oracle;"
            "from nbody_inputs import plummer_sphere; x,_,m = plummer_sphere(200, 16);"
            "print(json.dumps(oracle.accel(x, m, 2.0**-6).ravel().tolist()))") % root
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                         text=True, check=True).stdout
    assert np.array_equal(np.array(json.loads(out)).reshape(a.shape), a)


def test_high_precision_brute_force():
    # The same sums at 50 significant digits: the oracle's rounding stays
    # at the level of a few ulps.
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    x, _, m = _plummer(12, 17)
    eps = 2.0 ** -4
    a = oracle.accel(x, m, eps)
    n = x.shape[1]
    for i in range(n):
        acc = [mpmath.mpf(0)] * 3
        for j in range(n):
            if j == i:
                continue
            d = [mpmath.mpf(x[c, j]) - mpmath.mpf(x[c, i]) for c in range(3)]
            s = d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + mpmath.mpf(eps) ** 2
            for c in range(3):
                acc[c] += mpmath.mpf(m[j]) * d[c] / s ** mpmath.mpf(1.5)
        for c in range(3):
            assert abs(float(acc[c]) - a[c, i]) <= 1e-14 * abs(float(acc[c])) + 1e-300


def test_set_num_threads_bitwise():
    x, _, m = _plummer(300, 19)
    k0 = oracle.num_threads()
    a = oracle.accel(x, m, 2.0 ** -6)
    try:
        oracle.set_num_threads(1)
        assert oracle.num_threads() == 1
        assert np.array_equal(oracle.accel(x, m, 2.0 ** -6), a)
        oracle.set_num_threads(3)
        assert np.array_equal(oracle.accel(x, m, 2.0 ** -6), a)
    finally:
        oracle.set_num_threads(k0)
