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


@pytest.mark.parametrize("prec,n", [("mix_tilec", 16384), ("f32", 16384), ("mix_tilec", 40000)])
def test_captured_steps_replay_bitwise(prec, n):
    S, eps, dt = 5, 2.0 ** -7, 2.0 ** -8
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


def _reference(x0, v0, md, eps, dt, S, prec, ckpt_every):
    xe, ve, ae = x0.clone(), v0.clone(), torch.empty_like(x0)
    ce = torch.empty((S // ckpt_every + 1, 9 * x0.shape[1]), dtype=x0.dtype, device=DEV)
    nb.step(xe, ve, md, ae, eps, dt, S, prec=prec, ckpt=ce, ckpt_every=ckpt_every)
    return xe, ve, ae, ce


@pytest.mark.parametrize("prec,n", [("f64", 1024), ("mix_tilec", 16384), ("f32", 4096),
                                    ("mix_kahan", 300), ("mix_tilec", 40000)])
@pytest.mark.parametrize("side_stream", (False, True))
def test_library_graph_replays_bitwise(prec, n, side_stream):
    """NB_GRAPH: the library records the loop once, then relaunches the cached
    graph; every call equals the eager call bitwise."""
    S, K, eps, dt = 6, 4, 2.0 ** -7, 2.0 ** -8
    x, v, m = plummer_sphere(n, 61)
    x0, v0, md = to_dev(x, v, m, prec)
    xe, ve, ae, ce = _reference(x0, v0, md, eps, dt, S, prec, K)
    xs, vs, acc = x0.clone(), v0.clone(), torch.empty_like(x0)
    ckpt = torch.empty_like(ce)
    ws = torch.empty(max(1, nb.workspace_size(1, n, prec)), dtype=torch.uint8, device=DEV)
    stream = torch.cuda.Stream() if side_stream else torch.cuda.current_stream()
    for rep in range(3):
        xs.copy_(x0)
        vs.copy_(v0)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            nb.step(xs, vs, md, acc, eps, dt, S, prec=prec, ckpt=ckpt, ckpt_every=K,
                    graph=True, workspace=ws)
        torch.cuda.current_stream().wait_stream(stream)
        torch.cuda.synchronize()
        assert torch.equal(xs, xe) and torch.equal(vs, ve) and torch.equal(acc, ae), rep
        assert torch.equal(ckpt, ce), rep
        junk = nb.accel(x0, md, eps, prec=prec)  # eager work between launches
        torch.cuda.synchronize()
        del junk
    nb.graph_cache_clear()


def test_library_graph_cache_eviction():
    """More distinct argument sets than the cache holds: each call still gives
    the eager result, and clearing the cache leaves later calls working."""
    n, eps, dt, prec = 512, 2.0 ** -6, 2.0 ** -7, "f64"
    x, v, m = plummer_sphere(n, 62)
    x0, v0, md = to_dev(x, v, m, prec)
    for S in list(range(1, 21)) + [3, 1]:
        xe, ve, ae = x0.clone(), v0.clone(), torch.empty_like(x0)
        nb.step(xe, ve, md, ae, eps, dt, S, prec=prec)
        xs, vs, acc = x0.clone(), v0.clone(), torch.empty_like(x0)
        nb.step(xs, vs, md, acc, eps, dt, S, prec=prec, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(xs, xe) and torch.equal(vs, ve) and torch.equal(acc, ae), S
    nb.graph_cache_clear()
    xs, vs, acc = x0.clone(), v0.clone(), torch.empty_like(x0)
    nb.step(xs, vs, md, acc, eps, dt, 2, prec=prec, graph=True)
    xe, ve, ae = x0.clone(), v0.clone(), torch.empty_like(x0)
    nb.step(xe, ve, md, ae, eps, dt, 2, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(xs, xe) and torch.equal(vs, ve)
    nb.graph_cache_clear()


def test_library_graph_flag_inside_caller_capture():
    """With the caller's stream under capture the flag is ignored and the
    launches go into the caller's graph."""
    n, S, eps, dt, prec = 2048, 4, 2.0 ** -7, 2.0 ** -8, "mix_tilec"
    x, v, m = plummer_sphere(n, 63)
    x0, v0, md = to_dev(x, v, m, prec)
    xe, ve, ae, _ = _reference(x0, v0, md, eps, dt, S, prec, 1)
    xs, vs, acc = x0.clone(), v0.clone(), torch.empty_like(x0)
    ws = torch.empty(max(1, nb.workspace_size(1, n, prec)), dtype=torch.uint8, device=DEV)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        nb.step(xs, vs, md, acc, eps, dt, S, prec=prec, graph=True, workspace=ws)
    for rep in range(2):
        xs.copy_(x0)
        vs.copy_(v0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(xs, xe) and torch.equal(vs, ve) and torch.equal(acc, ae), rep
