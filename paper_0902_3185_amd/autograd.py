"""dmrg_hpsi as a differentiable torch operation.

``hpsi(psi, c, sb)`` returns y = H(c) psi with H(c) = sum_k c_k A_k (x) B_k.
The backward pass calls the library's adjoint: grad_psi = H^T g and
grad_c_k = < g, (A_k (x) B_k) psi >, so coupling derivatives such as dE/dJ2
follow from E = <psi|H(c)|psi> by the chain rule.
"""
from __future__ import annotations

import numpy as np
import torch


class DmrgHpsi(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi, c, sb):
        sb.set_coeffs(c.detach().to("cpu", torch.float64).numpy())
        y = sb.hpsi(psi.contiguous())
        ctx.save_for_backward(psi, c)
        ctx.sb = sb
        return y

    @staticmethod
    def backward(ctx, g):
        psi, c = ctx.saved_tensors
        sb = ctx.sb
        sb.set_coeffs(c.detach().to("cpu", torch.float64).numpy())
        need_psi, need_c = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gpsi, gc = sb.adjoint(psi.detach().contiguous(), g.contiguous(), want_psi=need_psi,
                              want_c=need_c)
        gc_t = torch.as_tensor(np.asarray(gc), dtype=c.dtype, device=c.device) if need_c else None
        return gpsi, gc_t, None


def hpsi(psi, c, sb):
    """Differentiable y = H(c) psi on a built Superblock."""
    return DmrgHpsi.apply(psi, c, sb)
