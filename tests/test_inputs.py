"""The seeded input generator: determinism, layout, and the Plummer mass
profile M(<r) = r^3 / (1 + r^2)^(3/2) (truncated at r = 10)."""

import numpy as np
import pytest

from nbody_inputs import WORKLOADS, make_state, plummer_sphere, plummer_with_subcluster


def test_deterministic_and_layout():
    a = plummer_sphere(1000, 5)
    b = plummer_sphere(1000, 5)
    c = plummer_sphere(1000, 6)
    for p, q in zip(a, b):
        assert p.dtype == np.float64 and np.array_equal(p, q)
    assert not np.array_equal(a[0], c[0])
    x, v, m = a
    assert x.shape == (3, 1000) and v.shape == (3, 1000) and m.shape == (1000,)
    assert x.flags["C_CONTIGUOUS"] and v.flags["C_CONTIGUOUS"]
    assert np.all(m == 1.0 / 1000)


def test_centre_of_mass_frame():
    x, v, m = plummer_sphere(4096, 7)
    assert np.abs(x @ m).max() < 1e-15
    assert np.abs(v @ m).max() < 1e-15


def test_mass_profile_ks():
    scipy_stats = pytest.importorskip("scipy.stats")
    x, _, _ = plummer_sphere(16384, 8)
    # the COM shift moves the centre by ~1e-2 at most; measure from the
    # sample's own centre
    r = np.linalg.norm(x, axis=0)
    rmax = 10.0
    norm = rmax ** 3 / (1 + rmax ** 2) ** 1.5

    def cdf(q):
        q = np.minimum(q, rmax)
        return q ** 3 / (1 + q * q) ** 1.5 / norm

    assert r.max() <= rmax + 0.1
    assert scipy_stats.kstest(r, cdf).pvalue > 1e-3


def test_speed_fraction_distribution():
    # v / v_esc(r) follows g(q) ~ q^2 (1 - q^2)^(7/2) on [0, 1]; compare the
    # sample mean with the mean of the normalised density.
    x, v, _ = plummer_sphere(20000, 9)
    r = np.linalg.norm(x, axis=0)
    q = np.linalg.norm(v, axis=0) / (np.sqrt(2.0) * (1 + r * r) ** -0.25)
    assert q.max() < 1.05
    grid = np.linspace(0, 1, 20001)
    g = grid ** 2 * (1 - grid ** 2) ** 3.5
    mean = np.trapezoid(grid * g, grid) / np.trapezoid(g, grid)
    assert abs(q.mean() - mean) < 0.02


def test_workloads_table():
    assert WORKLOADS["fp64-1024"].n == 1024 and WORKLOADS["scale-2^20"].n == 1 << 20
    for w in WORKLOADS.values():
        # every non-integer constant is a power of two
        for val in (w.eps, w.dt):
            assert np.log2(val) == int(np.log2(val))
        assert w.dt == w.eps / 2


def test_subcluster_split():
    x, v, m = plummer_with_subcluster(4096, 3, 33)
    assert x.shape == (3, 4096) and np.all(m == 1 / 4096)
    n_sub = round(0.1 * 4096)
    sub = x[:, 4096 - n_sub:]
    centre = np.median(sub, axis=1)
    main_centre = np.median(x[:, : 4096 - n_sub], axis=1)
    assert np.linalg.norm(centre - main_centre) == pytest.approx(3.0, abs=0.1)
    assert np.median(np.linalg.norm(sub - centre[:, None], axis=0)) < 0.2


def test_make_state_override_n():
    x, _, m = make_state("adjoint-16384", n=256)
    assert x.shape == (3, 256) and np.all(m == 1 / 256)


def test_device_positions_profile_and_determinism():
    """The chunked torch generator used for the largest sizes: same seed
    and chunk, same array; the truncated Plummer mass profile (KS test) and
    isotropy (mean direction near 0)."""
    scipy_stats = pytest.importorskip("scipy.stats")
    torch = pytest.importorskip("torch")
    from nbody_inputs import plummer_positions_device
    n = 100000
    x = plummer_positions_device(n, 11, "cpu", chunk=30000)
    assert x.shape == (3, n) and x.dtype == torch.float64
    assert torch.equal(x, plummer_positions_device(n, 11, "cpu", chunk=30000))
    assert not torch.equal(x, plummer_positions_device(n, 12, "cpu", chunk=30000))
    r = torch.linalg.norm(x, dim=0).numpy()
    assert r.max() <= 10.0
    norm = 1000.0 / 101.0 ** 1.5
    ks = scipy_stats.kstest(r, lambda q: q ** 3 / (1 + q * q) ** 1.5 / norm)
    assert ks.pvalue > 1e-3, ks
    u = (x / torch.linalg.norm(x, dim=0)).mean(dim=1).abs().max().item()
    assert u < 5.0 / np.sqrt(n)
