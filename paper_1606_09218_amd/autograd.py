"""torch.autograd binding of the RS interaction energy.

RSEnergy.apply(pos, q, ctx, factors, opts) assembles the RS-Tucker tensor of
the particle system, returns E_N (Lemma InterEnergy) as a 0-d FP64 tensor,
and in backward returns dE/dx from the library's adjoint force kernel
(rs_forces, F = -dE/dx with the Tucker basis held fixed) and dE/dz from
rs_energy.  The forward and backward computations all run in librs.so;
this module only moves pointers and applies the chain rule's scalar factor.
"""
from __future__ import annotations

import torch

from . import _lib


class RSEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, q, rsctx, factors, opts=None):
        pos_d = pos.detach().to(torch.float64).contiguous()
        q_d = q.detach().to(torch.float64).contiguous()
        T = _lib.assemble(rsctx, factors, pos_d, q_d, None, opts or _lib.make_aopts())
        N = q_d.numel()
        E = torch.empty(1, dtype=torch.float64, device=pos_d.device)
        dEdq = torch.empty(N, dtype=torch.float64, device=pos_d.device)
        _lib.energy(T, E, dEdq)
        ctx.T = T
        ctx.N = N
        ctx.dEdq = dEdq
        ctx.shape = pos.shape
        ctx.dtypes = (pos.dtype, q.dtype)
        return E.reshape(())

    @staticmethod
    def backward(ctx, gE):
        T = ctx.T
        g = float(gE.detach().reshape(()).item())
        grad_pos = grad_q = None
        if ctx.needs_input_grad[0]:
            F = torch.empty(3 * ctx.N, dtype=torch.float64, device=ctx.dEdq.device)
            # rs_forces writes -scale * dE/dx; scale = -g gives g * dE/dx
            _lib.forces(T, F, -g)
            grad_pos = F.view(ctx.shape).to(ctx.dtypes[0])
        if ctx.needs_input_grad[1]:
            grad_q = (ctx.dEdq * g).to(ctx.dtypes[1])
        T.free()
        ctx.T = None
        return grad_pos, grad_q, None, None, None


def rs_energy(pos, q, rsctx, factors, opts=None):
    """E_N of the particle system, differentiable in pos and q."""
    return RSEnergy.apply(pos, q, rsctx, factors, opts)
