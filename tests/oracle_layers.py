"""The FP64 oracle's backward-Euler step as a PyTorch autograd layer on CPU tensors (test
infrastructure only): forward = Newton with a direct solve, backward = the direct adjoint solve of
Eq. 9 and the closed-form VJPs. Used as the reference for rollouts with a policy in the loop."""
import numpy as np
import torch

from oracle import solve


class OracleStep(torch.autograd.Function):
    """The oracle's backward-Euler step as an autograd layer on CPU tensors: forward = Newton with
    a direct solve, backward = the direct adjoint solve of Eq. 9 and the closed-form VJPs."""

    @staticmethod
    def forward(fctx, prob, x0, v0, a):
        x1, v1, _ = solve.step(prob, x0.numpy(), v0.numpy(), a.numpy(), tol=1e-13)
        x1 = torch.from_numpy(x1)
        fctx.prob = prob
        fctx.save_for_backward(x0, a, x1)
        return x1, torch.from_numpy(v1)

    @staticmethod
    def backward(fctx, x1_bar, v1_bar):
        p = fctx.prob
        x0, a, x1 = (t.numpy() for t in fctx.saved_tensors)
        xb = np.zeros_like(x1) if x1_bar is None else x1_bar.numpy()
        vb = np.zeros_like(x1) if v1_bar is None else v1_bar.numpy()
        w = solve.adjoint(p, x1, x0, a, xb, vb)
        out = solve.vjp_params(p, w, x1, x0, a, vb)
        return None, torch.from_numpy(out["x0_bar"]), torch.from_numpy(out["v0_bar"]), torch.from_numpy(out["a_bar"])


def oracle_step(prob, x, v, a):
    return OracleStep.apply(prob, x, v, a)
