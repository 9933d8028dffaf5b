"""torch.autograd wrapper of a KDK rollout with a hand-written adjoint.

forward: nbody_step over nsteps with the state (x, v, a) stored every
ckpt_every steps into a checkpoint tensor (one native call).
backward: one nbody_step_adjoint call from the final state, which walks the
rollout back step by step (time-reversed KDK), reloads the stored state at
every checkpoint, and accumulates dL/dx_0, dL/dv_0 and dL/dm with the fused
adjoint pair kernel.
"""

from __future__ import annotations

import torch

from . import api


class NBodyRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, v0, m, eps, dt, nsteps, ckpt_every=20, prec="mix_tilec", G=1.0):
        n = x0.shape[1]
        x = x0.detach().clone()
        v = v0.detach().clone()
        acc = torch.empty_like(x)
        K = max(1, int(ckpt_every))
        ckpt = torch.empty((nsteps // K + 1, 9 * n), dtype=x.dtype, device=x.device)
        api.step(x, v, m.detach(), acc, eps, dt, nsteps, G=G, prec=prec, ckpt=ckpt, ckpt_every=K)
        ctx.save_for_backward(m.detach(), ckpt, x, v, acc)
        ctx.cfg = (float(eps), float(dt), int(nsteps), K, prec, float(G))
        return x.clone(), v.clone()

    @staticmethod
    def backward(ctx, gx, gv):
        m, ckpt, xS, vS, aS = ctx.saved_tensors
        eps, dt, nsteps, K, prec, G = ctx.cfg
        x, v, acc = xS.clone(), vS.clone(), aS.clone()
        lam_x = torch.zeros_like(x) if gx is None else gx.detach().to(x.dtype).contiguous().clone()
        lam_v = torch.zeros_like(v) if gv is None else gv.detach().to(v.dtype).contiguous().clone()
        lam_m = torch.zeros(x.shape[1], dtype=torch.float64, device=x.device)
        api.step_adjoint(x, v, m, acc, lam_x, lam_v, lam_m, eps, dt, nsteps, G=G, prec=prec,
                         entry_half=True, exit_full=False, ckpt=ckpt, ckpt_every=K,
                         step_end=nsteps)
        return lam_x, lam_v, lam_m.to(m.dtype), None, None, None, None, None, None


def rollout(x0, v0, m, eps, dt, nsteps, ckpt_every=20, prec="mix_tilec", G=1.0):
    """(x_S, v_S) after nsteps KDK steps, differentiable in x0, v0 and m."""
    return NBodyRollout.apply(x0, v0, m, eps, dt, nsteps, ckpt_every, prec, G)
