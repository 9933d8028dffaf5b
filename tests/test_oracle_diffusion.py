"""Pins of the oracle's 3-D diffusion step (section "3D diffusion equation").

* Discrete cosine modes cos(pi p (i + 1/2) / nx) cos(pi q (j + 1/2) / ny)
  cos(pi r (k + 1/2) / nz) are exact eigenvectors of the clamped 7-point
  update, with eigenvalue 1 - 4 (c_x sin^2(pi p / 2nx) + c_y sin^2(pi q / 2ny)
  + c_z sin^2(pi r / 2nz)), c_x = kappa dt / dx^2 etc.: catches a swapped
  axis, a wrong coefficient or a wrong boundary rule.
* A constant field is unchanged; the clamped (zero-flux) boundary conserves
  the sum of the field exactly up to rounding.
* A unit impulse spreads into exactly the seven coefficients.
"""

import numpy as np
import pytest

import oracle


def _mode(shape, p, q, r):
    nx, ny, nz = shape
    i = np.arange(nx)[:, None, None]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[None, None, :]
    return (np.cos(np.pi * p * (i + 0.5) / nx) * np.cos(np.pi * q * (j + 0.5) / ny)
            * np.cos(np.pi * r * (k + 0.5) / nz))


@pytest.mark.parametrize("shape,pqr", [((8, 6, 5), (1, 2, 3)), ((5, 9, 16), (4, 0, 7)),
                                        ((1, 7, 3), (0, 3, 1)), ((12, 12, 12), (11, 5, 2))])
def test_cosine_modes_are_eigenvectors(shape, pqr):
    dx, dy, dz, dt, kappa = 0.5, 0.25, 0.75, 0.01, 1.3
    f = _mode(shape, *pqr)
    fn = oracle.diffusion3d(f, dx, dy, dz, dt, kappa)
    c = [kappa * dt / (h * h) for h in (dx, dy, dz)]
    lam = 1.0 - 4.0 * sum(ck * np.sin(np.pi * m / (2 * n)) ** 2
                          for ck, m, n in zip(c, pqr, shape))
    np.testing.assert_allclose(fn, lam * f, rtol=0, atol=1e-14)


def test_constant_field_and_mass_conservation():
    dx, dy, dz, dt, kappa = 1.0, 2.0, 0.5, 0.02, 0.7
    f = np.full((7, 5, 11), 3.25)
    fn = oracle.diffusion3d(f, dx, dy, dz, dt, kappa)
    np.testing.assert_allclose(fn, f, rtol=0, atol=1e-14)
    g = np.random.default_rng(1).uniform(0, 1, size=(9, 13, 10))
    gn = oracle.diffusion3d(g, dx, dy, dz, dt, kappa)
    assert abs(gn.sum() - g.sum()) <= 1e-12 * g.sum()
    assert not np.allclose(gn, g)


def test_impulse_spreads_into_the_coefficients():
    dx, dy, dz, dt, kappa = 0.5, 1.0, 2.0, 0.05, 1.0
    f = np.zeros((5, 6, 7))
    f[2, 3, 4] = 1.0
    fn = oracle.diffusion3d(f, dx, dy, dz, dt, kappa)
    cx, cy, cz = (kappa * dt / (h * h) for h in (dx, dy, dz))
    expect = np.zeros_like(f)
    expect[2, 3, 4] = 1.0 - 2 * (cx + cy + cz)
    expect[1, 3, 4] = expect[3, 3, 4] = cx
    expect[2, 2, 4] = expect[2, 4, 4] = cy
    expect[2, 3, 3] = expect[2, 3, 5] = cz
    np.testing.assert_allclose(fn, expect, rtol=0, atol=1e-15)


def test_impulse_at_a_corner_reflects():
    # at i = 0 the missing neighbour i - 1 is replaced by i itself, so the
    # x-coefficient that would leave the grid stays at the corner
    dx, dy, dz, dt, kappa = 1.0, 1.0, 1.0, 0.1, 1.0
    f = np.zeros((3, 3, 3))
    f[0, 0, 0] = 1.0
    fn = oracle.diffusion3d(f, dx, dy, dz, dt, kappa)
    c = kappa * dt
    assert fn[0, 0, 0] == pytest.approx(1.0 - 6 * c + 3 * c, abs=1e-15)
    assert fn[1, 0, 0] == pytest.approx(c) and fn[0, 1, 0] == pytest.approx(c)
    assert fn[0, 0, 1] == pytest.approx(c)
    assert fn.sum() == pytest.approx(1.0, abs=1e-15)
