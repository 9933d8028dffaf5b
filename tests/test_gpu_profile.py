"""The library's own device-time profile (nbody_profile_begin / _end): the
launch groups of a leapfrog and of its reverse walk are counted per kind and
timed with HIP events on the caller's stream."""

import ctypes

import pytest
import torch

import paper_2411_18889_amd as nb
from nbody_inputs import plummer_sphere
from paper_2411_18889_amd import _lib
from tests.gpu_util import DEV, to_dev

pytestmark = pytest.mark.gpu


def test_profile_counts_and_times():
    L = _lib.lib()
    x, v, m = plummer_sphere(4096, 90)
    xd, vd, md = to_dev(x, v, m, "mix_tilec")
    acc = torch.empty_like(xd)
    S = 4
    prof = _lib.nb_profile_t()
    assert L.nbody_profile_begin() == 0
    nb.step(xd, vd, md, acc, 2.0 ** -7, 2.0 ** -8, S, prec="mix_tilec")
    lx, lv = torch.zeros_like(xd), torch.ones_like(vd)
    lm = torch.zeros(4096, dtype=torch.float64, device=DEV)
    nb.step_adjoint(xd, vd, md, acc, lx, lv, lm, 2.0 ** -7, 2.0 ** -8, S, prec="mix_tilec",
                    entry_half=True)
    assert L.nbody_profile_end(ctypes.byref(prof)) == 0
    # forward: a(x_0) + S force passes, each with its closing kick and, but
    # for the last, the next step's kick and drift in its finishing kernel
    # (4096 sinks: split source ranges, so the pass has one), so one
    # separate kick-drift; adjoint: entry pass + S fused passes, each but the
    # last with the next step's reverse drift in its finishing kernel, so no
    # separate reverse drift
    assert list(prof.calls) == [S + 1, S + 1, 1, 0, 0]
    assert all(prof.ms[k] > 0 for k in range(3))
    # a graph replay is not taken while profiling: the launch groups are
    # timed one by one as in an eager call
    assert L.nbody_profile_begin() == 0
    nb.step(xd, vd, md, acc, 2.0 ** -7, 2.0 ** -8, S, prec="mix_tilec", graph=True)
    assert L.nbody_profile_end(ctypes.byref(prof)) == 0
    assert list(prof.calls) == [S + 1, 0, 1, 0, 0]
    # outside a profile window nothing is recorded
    nb.step(xd, vd, md, acc, 2.0 ** -7, 2.0 ** -8, 1, prec="mix_tilec")
    assert L.nbody_profile_begin() == 0
    assert L.nbody_profile_end(ctypes.byref(prof)) == 0
    assert list(prof.calls) == [0, 0, 0, 0, 0]
