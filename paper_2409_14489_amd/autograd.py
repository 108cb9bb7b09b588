"""torch.autograd binding of the CB-ESSFM forward and its hand-written adjoint.

``cbessfm(field, coeffs, rho, plan)`` behaves like a differentiable function of
the field (complex64, (2, T) or (B, 2, T)), the applied coefficients
(float32 [steps][n_sb][n_sb][n_taps]) and the split ratio (float32 scalar
tensor), all on the device.  The forward is ``cbessfm_run``; the backward is
``cbessfm_backward`` (reverse sweep over the stored step fields and phases,
or over segments recomputed from stored spectra when checkpointing).
The plan holds one coefficient set at a time, so both passes load the
tensors they were given before running.
"""
from __future__ import annotations

import torch


class CBESSFMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, field_in, coeffs, rho, plan, checkpoint_every=1):
        ctx.rho_shape = rho.shape
        coeffs = coeffs.detach().contiguous()
        rho = rho.detach().reshape(1).contiguous()
        plan.set_coeffs(coeffs, rho)
        out = plan.run(field_in.detach())
        ctx.save_for_backward(field_in.detach(), coeffs, rho)
        ctx.plan = plan
        ctx.checkpoint_every = checkpoint_every
        return out

    @staticmethod
    def backward(ctx, grad_out):
        field_in, coeffs, rho = ctx.saved_tensors
        plan = ctx.plan
        plan.set_coeffs(coeffs, rho)
        need_in = ctx.needs_input_grad[0]
        gi, gc, gr = plan.backward(field_in, grad_out.contiguous(), need_grad_in=need_in,
                                   checkpoint_every=ctx.checkpoint_every)
        return (gi if need_in else None,
                gc if ctx.needs_input_grad[1] else None,
                gr.reshape(ctx.rho_shape) if ctx.needs_input_grad[2] else None,
                None, None)


def cbessfm(field_in: torch.Tensor, coeffs: torch.Tensor, rho: torch.Tensor, plan,
            checkpoint_every: int = 1) -> torch.Tensor:
    """Differentiable CB-ESSFM backpropagation of field_in with the given coefficients and rho."""
    out = CBESSFMFunction.apply(field_in, coeffs, rho, plan, checkpoint_every)
    return out


class CBESSFMStepsFunction(torch.autograd.Function):
    """Differentiable in the field, the coefficients and the N_st + 1
    dispersion segment lengths (free step sizes and split per step)."""

    @staticmethod
    def forward(ctx, field_in, coeffs, lengths, plan, checkpoint_every=1):
        coeffs = coeffs.detach().contiguous()
        lengths = lengths.detach().reshape(-1).contiguous()
        plan.set_coeffs(coeffs)
        plan.set_gvd_lengths(lengths)
        out = plan.run(field_in.detach())
        ctx.save_for_backward(field_in.detach(), coeffs, lengths)
        ctx.plan = plan
        ctx.checkpoint_every = checkpoint_every
        return out

    @staticmethod
    def backward(ctx, grad_out):
        field_in, coeffs, lengths = ctx.saved_tensors
        plan = ctx.plan
        plan.set_coeffs(coeffs)
        plan.set_gvd_lengths(lengths)
        need_in = ctx.needs_input_grad[0]
        gi, gc, _, gl = plan.backward_gvd(field_in, grad_out.contiguous(), need_grad_in=need_in,
                                          checkpoint_every=ctx.checkpoint_every)
        return (gi if need_in else None, gc if ctx.needs_input_grad[1] else None,
                gl if ctx.needs_input_grad[2] else None, None, None)


def cbessfm_steps(field_in: torch.Tensor, coeffs: torch.Tensor, lengths: torch.Tensor, plan,
                  checkpoint_every: int = 1) -> torch.Tensor:
    """CB-ESSFM with free dispersion segment lengths (float64 [steps + 1], km)."""
    return CBESSFMStepsFunction.apply(field_in, coeffs, lengths, plan, checkpoint_every)
