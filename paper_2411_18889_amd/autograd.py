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


def checkpoint_interval(nsteps, n, elem_bytes, budget_bytes):
    """The smallest interval K >= 1 whose nsteps // K + 1 checkpoint slots of
    9 n values (x, v, a) fit in budget_bytes; nsteps if none does. With a
    checkpoint every step the reverse walk reloads every state, and every
    adjoint pass skips the force sums."""
    for K in range(1, max(1, nsteps) + 1):
        if (nsteps // K + 1) * 9 * n * elem_bytes <= budget_bytes:
            return K
    return max(1, nsteps)


class NBodyRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, v0, m, eps, dt, nsteps, ckpt_every=20, prec="mix_tilec", G=1.0):
        n = x0.shape[1]
        x = x0.detach().clone()
        v = v0.detach().clone()
        acc = torch.empty_like(x)
        if ckpt_every == "auto":  # a quarter of the free device memory for the checkpoints
            free, _ = torch.cuda.mem_get_info(x.device)
            K = checkpoint_interval(int(nsteps), n, x.element_size(), free // 4)
        else:
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
    """(x_S, v_S) after nsteps KDK steps, differentiable in x0, v0 and m.
    ckpt_every: the checkpoint interval of the forward pass, or "auto" (the
    smallest interval whose checkpoints fit in a quarter of the free device
    memory; every step where they fit, which makes the backward pass about
    a fifth faster)."""
    return NBodyRollout.apply(x0, v0, m, eps, dt, nsteps, ckpt_every, prec, G)
