"""nbody_accel_noalloc, the entry point for callers that cannot allocate:
called through the C ABI, its results are nbody_accel's (same pass, same
kernels: bitwise), on two calls in a row -- the second smaller -- for the
symmetric pass, the one-sided kernel with a split source range, and
separate sink and source sets; a call whose pass needs more scratch than
the library's array is refused before anything is launched."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2411_18889_amd as nb
from nbody_inputs import plummer_sphere
from paper_2411_18889_amd import _lib
from tests.gpu_util import DEV, host, rel, to_dev

pytestmark = pytest.mark.gpu

VP = ctypes.c_void_p


def _noalloc(xi, mj, eps, prec, xj=None, potential=False):
    ni = xi.shape[1]
    src = xi if xj is None else xj
    acc = torch.full_like(xi, float("nan"))
    pot = torch.full((ni,), float("nan"), dtype=xi.dtype, device=DEV) if potential else None
    st = _lib.lib().nbody_accel_noalloc(
        ni, VP(xi.data_ptr()), src.shape[1], VP(src.data_ptr()), VP(mj.data_ptr()), float(eps),
        1.0, _lib.PREC[prec], VP(acc.data_ptr()), VP(pot.data_ptr()) if potential else VP(0),
        VP(torch.cuda.current_stream().cuda_stream))
    _lib.check(st, "nbody_accel_noalloc")
    return (acc, pot) if potential else acc


# (n of the first call, n of the second, policy): symmetric pass then a
# smaller symmetric pass; one-sided kernel with split source ranges, twice
CASES = [(40000, 20000, "mix_tilec"), (65536 + 77, 12289, "f32"), (30000, 13000, "f64"),
         (6000, 3000, "mix_kahan"), (9000, 1000, "f64")]


@pytest.mark.parametrize("n1,n2,prec", CASES)
def test_noalloc_matches_nbody_accel(n1, n2, prec):
    eps = 2.0 ** -8
    for n, seed in ((n1, 31), (n2, 32)):
        print("noalloc %s n=%d" % (prec, n), flush=True)
        x, v, m = plummer_sphere(n, seed)
        xd, _, md = to_dev(x, v, m, prec)
        for potential in (False, True):
            got = _noalloc(xd, md, eps, prec, potential=potential)
            ref = nb.accel(xd, md, eps, prec=prec, potential=potential)
            if potential:
                assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
            else:
                assert torch.equal(got, ref)
        a = host(got[0])
        idx = np.arange(0, n, max(1, n // 512))
        e = rel(a[:, idx], oracle.accel_sampled(host(xd), host(md), eps, idx))
        assert e <= (1e-12 if prec == "f64" else 1e-5)


def test_noalloc_separate_sets():
    prec, eps = "mix_tilec", 2.0 ** -7
    for ns, nt, seed in ((20000, 700, 41), (5000, 64, 42)):
        xs, vs, ms = plummer_sphere(ns, seed)
        xt, _, _ = plummer_sphere(nt, seed + 100)
        xsd, _, msd = to_dev(xs, vs, ms, prec)
        xtd = torch.tensor(xt, dtype=torch.float64, device=DEV)
        got = _noalloc(xtd, msd, eps, prec, xj=xsd, potential=True)
        ref = nb.accel(xtd, msd, eps, prec=prec, xj=xsd, potential=True)
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
        r = oracle.accel(host(xtd), host(msd), eps, xj=host(xsd))
        assert rel(host(got[0]), r) <= 1e-5


def test_noalloc_bands_within_its_scratch():
    """262144 particles on themselves: 402 MB of partials in the symmetric
    pass (eight sinks per lane, blocks of 2048), which nbody_accel runs in
    one band; the no-alloc entry point runs it in bands within its 128 MiB,
    bitwise the same."""
    n, prec, eps = 262144, "mix_tilec", 2.0 ** -9
    assert nb.pass_info(1, n, prec)["workspace_bytes"] > (128 << 20)
    x, v, m = plummer_sphere(n, 33)
    xd, _, md = to_dev(x, v, m, prec)
    for _ in range(2):
        got = _noalloc(xd, md, eps, prec)
        assert torch.equal(got, nb.accel(xd, md, eps, prec=prec))
    idx = np.arange(0, n, n // 256)
    assert rel(host(got)[:, idx], oracle.accel_sampled(host(xd), host(md), eps, idx)) <= 1e-5


def test_noalloc_refuses_passes_beyond_its_scratch():
    """3 x 2^20 particles on themselves: the running sums and one block row
    of the banded symmetric pass need ~151 MB, more than the 128 MiB array,
    so NB_EWORKSPACE, and the output is left untouched."""
    n, prec = 3 << 20, "mix_tilec"
    x = torch.zeros((3, n), dtype=torch.float64, device=DEV)
    m = torch.zeros(n, dtype=torch.float32, device=DEV)
    acc = torch.full_like(x, 7.0)
    st = _lib.lib().nbody_accel_noalloc(n, VP(x.data_ptr()), n, VP(x.data_ptr()),
                                        VP(m.data_ptr()), 0.01, 1.0, _lib.PREC[prec],
                                        VP(acc.data_ptr()), VP(0),
                                        VP(torch.cuda.current_stream().cuda_stream))
    assert st == _lib.NB_EWORKSPACE
    torch.cuda.synchronize()
    assert bool((acc == 7.0).all())
