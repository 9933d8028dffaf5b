"""Large-N check of the symmetric passes in bands (not a test: about three
minutes on one MI355X): one force pass and one adjoint entry pass at 2^23
and 2^24 particles (tile-compensated policy, default workspace of 4 GiB
bands), each timed with HIP events and checked on sampled sinks against the
oracle (e_glob; J^T lam and G^T lam), the force also by the third law.

    python tests/large_n_report.py

Test infrastructure: it uses the oracle (oracle/) for the reference values,
as the GPU tests do."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import numpy as np  # noqa: E402
import torch  # noqa: E402

import oracle  # noqa: E402
import paper_2411_18889_amd as nb  # noqa: E402
from nbody_inputs import plummer_positions_device  # noqa: E402
from tests.gpu_util import host, rel, sample_indices  # noqa: E402


def main():
    dev = torch.device("cuda:0")
    for n in (1 << 23, 1 << 24):
        eps, dt = 2.0 ** -12, 2.0 ** -12
        xd = plummer_positions_device(n, 901, dev)
        md = torch.full((n,), 1.0 / n, dtype=torch.float32, device=dev)
        print("n=%d pass_info force %s adjoint %s" % (n, nb.pass_info(1, n, "mix_tilec"),
                                                       nb.pass_info(2, n, "mix_tilec")), flush=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        a = nb.accel(xd, md, eps)
        e1.record()
        torch.cuda.synchronize()
        tf = e0.elapsed_time(e1)
        xh, mh = host(xd), host(md)
        idx = sample_indices(xh, 128, 16, seed=n % 97)
        ah = host(a)
        e = rel(ah[:, idx], oracle.accel_sampled(xh, mh, eps, idx))
        law = np.abs((ah * mh).sum(axis=1)).max() / (np.abs(ah) * mh).sum()
        print("n=%d force pass %.0f ms (%.0f G interactions/s), sampled e_glob %.3g, third law %.2g"
              % (n, tf, n * n / tf / 1e6, e, law), flush=True)
        # the entry pass of a reverse walk: J^T lam and G^T lam at x, weight dt/2
        lam = torch.tensor(np.random.default_rng(3).normal(size=(3, n)), device=dev)
        lx = torch.zeros_like(lam)
        lm = torch.zeros(n, dtype=torch.float64, device=dev)
        vd = torch.zeros_like(xd)
        e0.record()
        nb.step_adjoint(xd, vd, md, a, lx, lam, lm, eps, dt, 0, entry_half=True)
        e1.record()
        torch.cuda.synchronize()
        ta = e0.elapsed_time(e1)
        c = 0.5 * dt
        jt, gt = oracle.vjp_sampled(xh, mh, host(lam), eps, idx)
        print("n=%d adjoint entry pass %.0f ms (%.0f G interactions/s), J^T lam %.3g, G^T lam %.3g"
              % (n, ta, n * n / ta / 1e6, rel(host(lx)[:, idx] / c, jt), rel(host(lm)[idx] / c, gt)),
              flush=True)
        del xd, md, a, lam, lx, lm, vd
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
