"""Reference of the denoiser's gain x soft-threshold mask in plain torch
arithmetic (any device), with its gradient written out: what the library's
mask kernels compute, checked on the CPU against autograd through the
elementwise composition (test_autograd_cpu.py) and against the kernels on the
GPU (test_gpu_mask.py).
    Y' = g_k * m * Y,  m = max(0, 1 - lambda_k / max(|Y|, tiny)),
    dY = g_k * (m G + [m > 0, lambda_k > 0] (lambda/|Y|)(p/|Y|)/|Y| * Y),
    dg_k = sum of m p,  p = Re(conj(Y) G)."""
import torch


class ReferenceSoftThresholdGain(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, gain, thresholds):
        y = y.resolve_conj()
        yr = torch.view_as_real(y)
        r = y.abs().clamp_min_(torch.finfo(yr.dtype).tiny)
        lam = thresholds[:, None]
        one = torch.ones((), dtype=r.dtype, device=r.device)
        m = torch.addcdiv(one, lam, r, value=-1.0).clamp_min_(0.0)
        ctx.save_for_backward(y, gain, thresholds, r, m)
        return torch.view_as_complex(yr * (m * gain[:, None])[..., None])

    @staticmethod
    def backward(ctx, gout):
        y, gain, thresholds, r, m = ctx.saved_tensors
        yr = torch.view_as_real(y)
        gr = torch.view_as_real(gout.resolve_conj())
        p = (yr * gr).sum(-1)
        gy = gg = None
        if ctx.needs_input_grad[0]:
            lam = thresholds[:, None]
            c = torch.where((m > 0) & (lam > 0), (lam / r) * (p / r) / r,
                            torch.zeros((), dtype=p.dtype, device=p.device))
            g = gain[:, None]
            gy = torch.view_as_complex(torch.addcmul(gr * (m * g)[..., None], yr, (c * g)[..., None]))
        if ctx.needs_input_grad[1]:
            dims = [d for d in range(p.dim()) if d != p.dim() - 2]
            gg = (m * p).sum(dim=dims)
        return gy, gg, None


def reference_soft_threshold_gain(y, gain, thresholds):
    return ReferenceSoftThresholdGain.apply(y, gain, thresholds)
