"""Differentiable QTAM: torch.autograd.Function wrappers whose backward passes
are the library's hand-written adjoint kernels.

The forward transform x -> Y and the canonical-dual inverse Y -> x are linear
(Sec. III), so their gradients are their adjoints as real-linear maps (App. C:
the adjoint of analysis is synthesis). PyTorch hands a complex tensor's
gradient over as dL/dRe + i dL/dIm, which is exactly what
``qtam_forward_adjoint`` consumes and ``qtam_inverse_adjoint`` produces.
"""
from __future__ import annotations

import torch

from .binding import Plan


class QtamForwardFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.forward(x.contiguous())

    @staticmethod
    def backward(ctx, gy: torch.Tensor):
        gx = ctx.plan.forward_adjoint(gy.resolve_conj().contiguous())
        return gx, None


class QtamInverseFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.inverse(y.resolve_conj().contiguous())

    @staticmethod
    def backward(ctx, gx: torch.Tensor):
        gy = ctx.plan.inverse_adjoint(gx.contiguous())
        return gy, None


def qtam_forward(x: torch.Tensor, plan: Plan) -> torch.Tensor:
    return QtamForwardFn.apply(x, plan)


def qtam_inverse(y: torch.Tensor, plan: Plan) -> torch.Tensor:
    return QtamInverseFn.apply(y, plan)


class QTAM(torch.nn.Module):
    """Module form: ``forward`` analyses, ``inverse`` synthesises; both
    differentiable. Holds one plan (one shape, Q, grid and precision)."""

    def __init__(self, plan: Plan | None = None, **params):
        super().__init__()
        self.plan = plan if plan is not None else Plan(**params)

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        return qtam_forward(x, self.plan)

    def inverse(self, y: torch.Tensor) -> torch.Tensor:
        return qtam_inverse(y, self.plan)


class SoftThresholdGainFn(torch.autograd.Function):
    """Y' = g_k * m * Y with m = max(0, 1 - lambda_k / |Y|) on row k (the row
    axis is the second to last of Y), forward and gradient both in the
    library's mask kernels (qtam_mask_forward / qtam_mask_backward). With G
    the incoming gradient (dL/dRe + i dL/dIm) and p = Re(conj(Y) G):
        dY = g_k * (m G + [|Y| > lambda_k] * lambda_k p / |Y|^3 * Y),
        dg_k = sum over every other axis of m p;
    where |Y| <= lambda_k the mask is zero and locally constant, so dY = 0.
    The thresholds get no gradient."""

    @staticmethod
    def forward(ctx, y: torch.Tensor, gain: torch.Tensor, thresholds: torch.Tensor, plan: Plan) -> torch.Tensor:
        y = y.resolve_conj().contiguous()
        ctx.plan = plan
        ctx.save_for_backward(y, gain, thresholds)
        return plan.mask_forward(y, gain.contiguous(), thresholds.contiguous())

    @staticmethod
    def backward(ctx, gout: torch.Tensor):
        y, gain, thresholds = ctx.saved_tensors
        gy, gg = ctx.plan.mask_backward(y, gain.contiguous(), thresholds.contiguous(),
                                        gout.resolve_conj().contiguous())
        return (gy if ctx.needs_input_grad[0] else None), (gg if ctx.needs_input_grad[1] else None), None, None


def soft_threshold_gain(y: torch.Tensor, gain: torch.Tensor, thresholds: torch.Tensor, plan: Plan) -> torch.Tensor:
    return SoftThresholdGainFn.apply(y, gain, thresholds, plan)


class MaskedInverseFn(torch.autograd.Function):
    """x = inverse(g_k * m * Y), the mask of SoftThresholdGainFn and the
    inverse transform in one pass (qtam_inverse_masked: the mask is applied
    as the inverse rows load Y); the backward pass is the inverse adjoint with
    the mask's gradient in its rows kernel (qtam_inverse_masked_adjoint). The
    same values and gradients as soft_threshold_gain followed by qtam_inverse,
    without the masked envelopes or their gradient in memory."""

    @staticmethod
    def forward(ctx, y: torch.Tensor, gain: torch.Tensor, thresholds: torch.Tensor, plan: Plan) -> torch.Tensor:
        y = y.resolve_conj().contiguous()
        gain, thresholds = gain.contiguous(), thresholds.contiguous()
        ctx.plan = plan
        ctx.save_for_backward(y, gain, thresholds)
        return plan.inverse_masked(y, gain, thresholds)

    @staticmethod
    def backward(ctx, gx: torch.Tensor):
        y, gain, thresholds = ctx.saved_tensors
        gy, gg = ctx.plan.inverse_masked_adjoint(gx.contiguous(), y, gain, thresholds)
        return (gy if ctx.needs_input_grad[0] else None), (gg if ctx.needs_input_grad[1] else None), None, None


def masked_inverse(y: torch.Tensor, gain: torch.Tensor, thresholds: torch.Tensor, plan: Plan) -> torch.Tensor:
    """inverse(soft_threshold_gain(y, ...)), fused where the plan allows it
    (rows transformed in one workgroup), else the two steps."""
    if plan.masked_inverse_supported:
        return MaskedInverseFn.apply(y, gain, thresholds, plan)
    return qtam_inverse(soft_threshold_gain(y, gain, thresholds, plan), plan)


class GainThresholdDenoiser(torch.nn.Module):
    """Forward transform, a learnable gain per row times a soft-threshold mask
    on the envelope magnitudes, and the inverse transform:
        Y' = g_k * Y * max(0, 1 - lambda_k / |Y|),   x_hat = inverse(Y').
    lambda_k are fixed thresholds per row; g starts at 1."""

    def __init__(self, plan: Plan, thresholds: torch.Tensor):
        super().__init__()
        self.qtam = QTAM(plan)
        rdt = torch.float64 if plan.fp64 else torch.float32
        self.gain = torch.nn.Parameter(torch.ones(plan.R, dtype=rdt, device=thresholds.device))
        self.register_buffer("thresholds", thresholds.to(rdt))

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        return masked_inverse(self.qtam(x), self.gain, self.thresholds, self.qtam.plan)
