"""GPU parity of the 3-D diffusion step (section "3D diffusion equation")
against the FP64 oracle on the same FP32 grid. The update is a convex-ish
combination of seven FP32 values with FP32 coefficients: its rounding error
is a few ulps of max|f|, bound here by 1e-6 of max|f|."""

import numpy as np
import pytest
import torch

import oracle
import paper_2411_18889_amd as nb
from tests.gpu_util import DEV

pytestmark = pytest.mark.gpu

PARAMS = dict(dx=0.5, dy=0.25, dz=1.0, dt=0.01, kappa=1.5)


def _check(f32):
    fd = torch.tensor(f32, device=DEV)
    fn = nb.api.diffusion3d_step(fd, **PARAMS).cpu().numpy().astype(np.float64)
    ref = oracle.diffusion3d(f32.astype(np.float64), **PARAMS)
    err = np.abs(fn - ref).max() / np.abs(ref).max()
    assert err <= 1e-6, err
    return fn, ref


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 5), (7, 9, 65), (33, 17, 130),
                                   (64, 64, 64), (40, 70, 129), (65, 8, 64)])
def test_random_grids(shape):
    f = np.random.default_rng(sum(shape)).uniform(-1, 1, size=shape).astype(np.float32)
    _check(f)


def test_cosine_mode_eigenvalue():
    shape = (48, 40, 96)
    nx, ny, nz = shape
    i = np.arange(nx)[:, None, None]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[None, None, :]
    p, q, r = 3, 5, 7
    f = (np.cos(np.pi * p * (i + 0.5) / nx) * np.cos(np.pi * q * (j + 0.5) / ny)
         * np.cos(np.pi * r * (k + 0.5) / nz)).astype(np.float32)
    fn, _ = _check(f)
    c = [PARAMS["kappa"] * PARAMS["dt"] / h ** 2 for h in (PARAMS["dx"], PARAMS["dy"], PARAMS["dz"])]
    lam = 1 - 4 * sum(ck * np.sin(np.pi * m / (2 * n)) ** 2 for ck, m, n in zip(c, (p, q, r), shape))
    assert np.abs(fn - lam * f).max() <= 1e-6


def test_paper_size_sampled_planes():
    """512^3 (the paper's best-performing size) in the launch shape the bench
    times; the oracle checks every point."""
    shape = (512, 512, 512)
    f = np.random.default_rng(5).uniform(0, 1, size=shape).astype(np.float32)
    _check(f)


def test_mass_conserved_on_gpu():
    f = np.random.default_rng(9).uniform(0, 1, size=(96, 80, 72)).astype(np.float32)
    fd = torch.tensor(f, device=DEV)
    fn = nb.api.diffusion3d_step(fd, **PARAMS)
    s0, s1 = float(fd.double().sum()), float(fn.double().sum())
    assert abs(s1 - s0) <= 1e-6 * s0
