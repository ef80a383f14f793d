"""``torch.autograd.Function`` over the fused log-likelihood + adjoint pass.

The forward pass enqueues one ``hawkes_grad_device`` call on the current torch stream: the HIP
kernels write (ell, d ell / d Theta) into a 7-element float64 device tensor.  The gradient is a
by-product of that same pairwise pass, so backward is only ``grad_output * saved_gradient``.
There is no gradient with respect to the event data.  torch supplies device memory and the
stream; it computes nothing of the likelihood.
"""
from __future__ import annotations

import torch

from . import binding


class HawkesLogLik(torch.autograd.Function):
    """ell(Theta) for a device-resident dataset; Theta = (mu0, tau_x, tau_t, theta, omega, h)."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, hctx: binding.Context, ds: binding.Dataset, precision="fp32c"):
        if theta.shape != (6,):
            raise ValueError("theta must have shape (6,)")
        values = theta.detach().to("cpu", torch.float64).tolist()
        out = torch.empty(7, dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream()
        hctx.grad_device(ds, values, precision, out.data_ptr(), stream.cuda_stream)
        ctx.save_for_backward(out[1:].to(theta.device, theta.dtype))
        return out[0].to(theta.device, theta.dtype)

    @staticmethod
    def backward(ctx, grad_output):
        (grad,) = ctx.saved_tensors
        return grad_output * grad, None, None, None


def loglik(theta: torch.Tensor, hctx: binding.Context, ds: binding.Dataset, precision="fp32c"):
    return HawkesLogLik.apply(theta, hctx, ds, precision)
