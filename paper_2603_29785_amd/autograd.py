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
        Y = self.qtam(x)
        mag = Y.abs()
        tiny = torch.finfo(mag.dtype).tiny
        mask = torch.clamp(1.0 - self.thresholds[:, None] / torch.clamp(mag, min=tiny), min=0.0)
        Yp = Y * (self.gain[:, None] * mask)
        return self.qtam.inverse(Yp)
