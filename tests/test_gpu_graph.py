"""The library only enqueues kernels and device-to-device copies on the
caller's stream and never allocates, so a leapfrog call can be captured into
a HIP graph (here through torch.cuda.CUDAGraph) to hide launch latency at
small N. Every replay must match the eager result bitwise, with the
program's own eager work and synchronisations between replays."""

import pytest
import torch

import paper_2411_18889_amd as nb
from nbody_inputs import plummer_sphere
from tests.gpu_util import DEV, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ("mix_tilec", "f32"))
def test_captured_steps_replay_bitwise(prec):
    n, S, eps, dt = 16384, 5, 2.0 ** -7, 2.0 ** -8
    x, v, m = plummer_sphere(n, 60)
    x0, v0, md = to_dev(x, v, m, prec)

    # eager reference: S steps from (x0, v0)
    xe, ve = x0.clone(), v0.clone()
    ae = torch.empty_like(xe)
    nb.step(xe, ve, md, ae, eps, dt, S, prec=prec)
    torch.cuda.synchronize()

    # static buffers for the graph
    xs, vs, acc = x0.clone(), v0.clone(), torch.empty_like(x0)
    ckpt = torch.empty((S // 2 + 1, 9 * n), dtype=x0.dtype, device=DEV)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside capture
        nb.step(xs, vs, md, acc, eps, dt, S, prec=prec, ckpt=ckpt, ckpt_every=2)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        nb.step(xs, vs, md, acc, eps, dt, S, prec=prec, ckpt=ckpt, ckpt_every=2)

    for rep in range(3):
        xs.copy_(x0)
        vs.copy_(v0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(xs, xe) and torch.equal(vs, ve) and torch.equal(acc, ae), rep
        assert torch.equal(ckpt[0, : 3 * n].view(3, n), x0), rep
        # unrelated eager work between replays
        junk = nb.accel(x0, md, eps, prec=prec)
        torch.cuda.synchronize()
        del junk
