"""Adjoint-method gradients behind torch.autograd.Function.

``AdjointExpval.apply(params, n, template, terms, dtype)`` returns E(theta) =
<psi(theta)|H|psi(theta)> for a parameterised circuit (RX/RY/RZ rotations exp(-i theta P/2)
carrying parameter indices, plus fixed gates), for a (P,) or (B, P) tensor of angles.
The forward call runs libqsv's forward sweep and reverse (adjoint) sweep once and keeps
dE/dtheta; backward scales it by the incoming gradient.  The angles may live on any
device; energies come back on the angles' device and dtype.
"""
import torch

from . import qsv


class AdjointExpval(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, n, template, terms, dtype="c128"):
        p = params.detach().to("cpu", torch.float64).numpy()
        E, G = qsv.adjoint_grad(n, template, p, terms, dtype)
        ctx.save_for_backward(torch.as_tensor(G, dtype=params.dtype, device=params.device))
        return torch.as_tensor(E, dtype=params.dtype, device=params.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out.unsqueeze(-1) * g, None, None, None, None


def expval(params, n, template, terms, dtype="c128"):
    return AdjointExpval.apply(params, n, template, terms, dtype)
