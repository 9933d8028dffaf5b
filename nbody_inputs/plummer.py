"""Seeded Plummer-sphere initial conditions (Aarseth, Henon & Wielen 1974).

Units: G = 1. A sphere of total mass ``M`` and scale radius ``a`` has the
cumulative mass profile M(<r) = M r^3 / (r^2 + a^2)^(3/2) and the isotropic
distribution function f(E) ~ (-E)^(7/2). Sampling:

* radius: draw the enclosed mass fraction X ~ U(0, 1) and invert the profile,
  r = a / sqrt(X^(-2/3) - 1); radii beyond ``rmax`` (10 a by default) are
  redrawn (truncation);
* speed: v = q * v_esc(r) with v_esc(r) = sqrt(2 G M / a) (1 + r^2/a^2)^(-1/4)
  and q drawn from g(q) ~ q^2 (1 - q^2)^(7/2) by von Neumann rejection against
  the box [0, 1] x [0, 0.1] (the maximum of g is about 0.0923);
* directions of position and velocity: isotropic, cos(theta) ~ U(-1, 1) and
  phi ~ U(0, 2 pi);
* finally the centre-of-mass position and velocity are subtracted.

The arrays are structure-of-arrays: positions and velocities have shape
(3, N) (rows x, y, z), masses shape (N,), all float64. Everything is drawn
from ``numpy.random.Generator(PCG64(seed))`` in a fixed order, so a seed
always yields bitwise the same arrays.
"""

from __future__ import annotations

import numpy as np


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    """n unit vectors, uniformly distributed on the sphere, shape (3, n)."""
    cos_t = 2.0 * rng.random(n) - 1.0
    phi = 2.0 * np.pi * rng.random(n)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    return np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t])


def _radii(rng: np.random.Generator, n: int, a: float, rmax: float) -> np.ndarray:
    out = np.empty(n)
    k = 0
    while k < n:
        batch = max(256, int((n - k) * 1.05) + 16)
        X = rng.random(batch)
        with np.errstate(divide="ignore"):
            r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        r = r[np.isfinite(r) & (r <= rmax)]
        take = min(n - k, r.size)
        out[k:k + take] = r[:take]
        k += take
    return out


def _speed_fractions(rng: np.random.Generator, n: int) -> np.ndarray:
    out = np.empty(n)
    k = 0
    while k < n:
        batch = max(256, int((n - k) * 11) + 16)  # acceptance rate is ~ 0.1
        q = rng.random(batch)
        y = 0.1 * rng.random(batch)
        q = q[y < q * q * (1.0 - q * q) ** 3.5]
        take = min(n - k, q.size)
        out[k:k + take] = q[:take]
        k += take
    return out


def _sphere(rng, n, M, a, rmax, G):
    r = _radii(rng, n, a, rmax)
    x = r * _isotropic(rng, n)
    q = _speed_fractions(rng, n)
    vesc = np.sqrt(2.0 * G * M / a) * (1.0 + (r / a) ** 2) ** -0.25
    v = (q * vesc) * _isotropic(rng, n)
    return x, v


def _to_com_frame(x, v, m):
    mt = m.sum()
    x = x - (x @ m / mt)[:, None]
    v = v - (v @ m / mt)[:, None]
    return np.ascontiguousarray(x), np.ascontiguousarray(v)


def plummer_sphere(n: int, seed: int, M: float = 1.0, a: float = 1.0,
                   rmax_over_a: float = 10.0, G: float = 1.0):
    """Equal-mass Plummer sphere of ``n`` particles, each of mass M/n.

    Returns ``(x, v, m)``: float64 arrays of shape (3, n), (3, n), (n,), in
    the centre-of-mass frame.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.Generator(np.random.PCG64(seed))
    x, v = _sphere(rng, n, M, a, rmax_over_a * a, G)
    m = np.full(n, M / n)
    x, v = _to_com_frame(x, v, m)
    return x, v, m


def plummer_with_subcluster(n_total: int, seed_main: int, seed_sub: int,
                            sub_fraction: float = 0.1, a_main: float = 1.0,
                            a_sub: float = 0.1, r_sub: float = 3.0,
                            rmax_over_a: float = 10.0, G: float = 1.0):
    """Plummer sphere plus an offset Plummer subcluster, equal masses 1/n_total.

    ``n_sub = round(sub_fraction * n_total)`` particles form a subcluster of
    scale ``a_sub`` centred at distance ``r_sub`` from the main sphere's
    centre, along a direction drawn from ``seed_sub``; it has zero bulk
    velocity relative to the main sphere. Each sphere's velocities are drawn
    from its own Plummer distribution function (its own mass and scale). The
    union is shifted to its centre-of-mass frame. Returns ``(x, v, m)``; the
    main sphere's particles come first.
    """
    n_sub = int(round(sub_fraction * n_total))
    n_main = n_total - n_sub
    mp = 1.0 / n_total
    rng_main = np.random.Generator(np.random.PCG64(seed_main))
    rng_sub = np.random.Generator(np.random.PCG64(seed_sub))
    xm, vm = _sphere(rng_main, n_main, n_main * mp, a_main, rmax_over_a * a_main, G)
    centre = r_sub * _isotropic(rng_sub, 1)
    xs, vs = _sphere(rng_sub, n_sub, n_sub * mp, a_sub, rmax_over_a * a_sub, G)
    x = np.concatenate([xm, xs + centre], axis=1)
    v = np.concatenate([vm, vs], axis=1)
    m = np.full(n_total, mp)
    x, v = _to_com_frame(x, v, m)
    return x, v, m


def plummer_positions_device(n: int, seed: int, device, a: float = 1.0, rmax: float = 10.0,
                             chunk: int = 1 << 26):
    """Positions only, (3, n) float64 torch tensor on `device`, drawn there
    from a seeded ``torch.Generator`` with the same recipe as
    ``plummer_sphere`` (radius by inverting the mass profile, truncated at
    rmax by redrawing; isotropic direction), in chunks so that sizes up to
    2^30 need no host memory. Not bitwise equal to ``plummer_sphere`` (a
    different generator), and not shifted to the centre-of-mass frame."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    out = torch.empty((3, n), dtype=torch.float64, device=device)
    for k0 in range(0, n, chunk):
        k = min(chunk, n - k0)
        r = torch.empty(k, dtype=torch.float64, device=device)
        todo = torch.arange(k, device=device)
        while todo.numel():
            X = torch.rand(todo.numel(), dtype=torch.float64, device=device, generator=g)
            rr = a / torch.sqrt(X ** (-2.0 / 3.0) - 1.0)
            ok = torch.isfinite(rr) & (rr <= rmax)
            r[todo[ok]] = rr[ok]
            todo = todo[~ok]
        cos_t = 2.0 * torch.rand(k, dtype=torch.float64, device=device, generator=g) - 1.0
        phi = 2.0 * torch.pi * torch.rand(k, dtype=torch.float64, device=device, generator=g)
        sin_t = torch.sqrt(torch.clamp(1.0 - cos_t * cos_t, min=0.0))
        out[0, k0:k0 + k] = r * sin_t * torch.cos(phi)
        out[1, k0:k0 + k] = r * sin_t * torch.sin(phi)
        out[2, k0:k0 + k] = r * cos_t
    return out
