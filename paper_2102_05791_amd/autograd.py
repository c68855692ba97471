"""PyTorch autograd wrappers over the C ABI (marshalling only).

ImplicitStep: one step as a differentiable layer (the integration cell of Sec. 5, Fig.
dynamics-cell): the forward is isb_step; the backward is the adjoint solve of Eq. 9
(isb_solve_adjoint) followed by isb_vjp_params, which also carries the explicit
v1 = (x1 - x0)/h path of Eq. 14, and, when the per-element Lame pair and fibre stiffness are
passed as inputs, their cotangents.

CheckpointedRollout: backpropagation through time over T steps (Sec. 5.1) storing only every
K-th state; the backward recomputes one K-step segment at a time from its checkpoint, so
memory is O(T/K + K) states and the cost is one extra forward step per step.
"""
from __future__ import annotations

import torch

from .isb import Context


class ImplicitStep(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx: Context, x0, v0, a, mu=None, lam=None, kf=None):
        if mu is not None:
            ctx.set_material_params(mu, lam, kf)
        x1, v1, _, _ = ctx.step(x0, v0, a, stats=False)
        if v1 is None:
            v1 = torch.zeros_like(x1)
        fctx.ctx = ctx
        fctx.with_material = mu is not None
        # the material this step ran with: the context may hold another one by the time backward runs
        fctx.material = (mu.detach().clone(), lam.detach().clone(), kf.detach().clone()) if mu is not None else None
        fctx.save_for_backward(x0, a, x1)
        return x1, v1

    @staticmethod
    def backward(fctx, x1_bar, v1_bar):
        ctx = fctx.ctx
        x0, a, x1 = fctx.saved_tensors
        if fctx.material is not None:
            ctx.set_material_params(*fctx.material)   # a no-op when the context still holds it
        x1_bar = torch.zeros_like(x1) if x1_bar is None else x1_bar.contiguous()
        v1_bar = None if v1_bar is None else v1_bar.contiguous()
        w, _, _ = ctx.solve_adjoint(x1, x0, a, x1_bar, v1_bar, stats=False)
        want = ("a_bar", "x0_bar", "v0_bar") + (("mu_bar", "lam_bar", "kf_bar") if fctx.with_material else ())
        out = ctx.vjp_params(w, x1, x0, a, v1_bar, want=want)
        mat = (out["mu_bar"], out["lam_bar"], out["kf_bar"]) if fctx.with_material else (None, None, None)
        return (None, out["x0_bar"], out["v0_bar"], out["a_bar"]) + mat


def implicit_step(ctx: Context, x0, v0, a, mu=None, lam=None, kf=None):
    """One differentiable step. With mu, lam, kf (device tensors [n_e], e.g. requiring grad) the
    step runs with that Lame pair and fibre stiffness, uploaded when they differ from the context's
    current ones (a host copy), and the backward also returns their cotangents (Eq. 9)."""
    if (mu is None) != (lam is None) or (mu is None) != (kf is None):
        raise ValueError("give all of mu, lam, kf or none of them")
    return ImplicitStep.apply(ctx, x0, v0, a, mu, lam, kf)


class CheckpointedRollout(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx: Context, every: int, x0, v0, actions):
        T = actions.shape[0]
        cps = [(x0, v0)]
        x, v = x0, v0
        for t in range(T):
            x, v, _, _ = ctx.step(x, v, actions[t].contiguous(), stats=False)
            if (t + 1) % every == 0 and t + 1 < T:
                cps.append((x, v))
        fctx.ctx, fctx.every, fctx.T = ctx, every, T
        flat = [t for xv in cps for t in xv]
        fctx.save_for_backward(actions, *flat)
        return x.clone(), v.clone()

    @staticmethod
    def backward(fctx, xT_bar, vT_bar):
        ctx, K, T = fctx.ctx, fctx.every, fctx.T
        actions, *flat = fctx.saved_tensors
        cps = [(flat[2 * i], flat[2 * i + 1]) for i in range(len(flat) // 2)]
        a_bar = torch.zeros_like(actions)
        xb = xT_bar.contiguous() if xT_bar is not None else None
        vb = vT_bar.contiguous() if vT_bar is not None else None
        if xb is None:
            xb = torch.zeros_like(cps[0][0])
        # each adjoint CG starts from the one of the step after (ISB_OPT_ADJ_WARM_START), in place:
        # that adjoint is no longer needed once its VJP is taken
        w = None
        for seg in range((T - 1) // K, -1, -1):
            t0, t1 = seg * K, min(seg * K + K, T)
            states = [cps[seg]]
            for t in range(t0, t1):
                x, v, _, _ = ctx.step(states[-1][0], states[-1][1], actions[t].contiguous(), stats=False)
                states.append((x, v))
            for t in range(t1 - 1, t0 - 1, -1):
                x_prev, x_next = states[t - t0][0], states[t - t0 + 1][0]
                a_t = actions[t].contiguous()
                w, _, _ = ctx.solve_adjoint(x_next, x_prev, a_t, xb, vb, stats=False, w=w, w_init=w)
                out = ctx.vjp_params(w, x_next, x_prev, a_t, vb, want=("a_bar", "x0_bar", "v0_bar"))
                a_bar[t] = out["a_bar"]
                xb, vb = out["x0_bar"], out["v0_bar"]
        return None, None, xb, vb, a_bar


def rollout(ctx: Context, x0, v0, actions, checkpoint_every: int = 10):
    """Differentiable T-step rollout; returns (x_T, v_T)."""
    return CheckpointedRollout.apply(ctx, int(checkpoint_every), x0, v0, actions)
