"""The reference of the denoiser's soft-threshold gain with its hand-written
gradient (tests/mask_reference.py, the formula the library's mask kernels
implement), on CPU tensors: gradcheck in FP64, and values and gradients equal
to autograd through the elementwise composition
Y * (g * max(0, 1 - lambda / max(|Y|, tiny)))."""
import pytest
import torch

from mask_reference import reference_soft_threshold_gain as soft_threshold_gain


def composed(y, gain, lam):
    mag = y.abs()
    mask = torch.clamp(1.0 - lam[:, None] / torch.clamp(mag, min=torch.finfo(mag.dtype).tiny), min=0.0)
    return y * (gain[:, None] * mask)


def inputs(shape, dtype, seed, zeros=False):
    g = torch.Generator().manual_seed(seed)
    cdt = torch.complex128 if dtype == torch.float64 else torch.complex64
    y = torch.randn(shape, generator=g, dtype=cdt)
    R = shape[-2]
    lam = 0.3 + torch.rand(R, generator=g, dtype=dtype)
    # keep |Y| away from the kink at lambda, so finite differences see one branch
    mag = y.abs()
    near = (mag - lam[:, None]).abs() < 0.05
    y = torch.where(near, y * 1.2, y)
    if zeros:
        y[..., 0] = 0
    gain = torch.linspace(-0.5, 1.5, R, dtype=dtype)
    return y, gain, lam


def test_gradcheck_fp64():
    y, gain, lam = inputs((2, 5, 7), torch.float64, 0)
    y.requires_grad_(True)
    gain.requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: soft_threshold_gain(a, b, lam), (y, gain), eps=1e-6, atol=1e-9)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-13), (torch.float32, 2e-6)])
@pytest.mark.parametrize("shape", [(3, 6, 33), (6, 1), (2, 2, 4, 9)])
def test_matches_composed_autograd(dtype, tol, shape):
    y, gain, lam = inputs(shape, dtype, 1, zeros=True)
    ya, ga = y.clone().requires_grad_(True), gain.clone().requires_grad_(True)
    yb, gb = y.clone().requires_grad_(True), gain.clone().requires_grad_(True)
    out_a = soft_threshold_gain(ya, ga, lam)
    out_b = composed(yb, gb, lam)
    assert torch.allclose(out_a, out_b, rtol=tol, atol=tol)
    w = torch.randn(out_a.shape, generator=torch.Generator().manual_seed(2), dtype=out_a.dtype)
    (out_a * w.conj()).real.sum().backward()
    (out_b * w.conj()).real.sum().backward()
    scale = float(yb.grad.abs().max())
    assert float((ya.grad - yb.grad).abs().max()) <= tol * 10 * scale
    assert torch.allclose(ga.grad, gb.grad, rtol=tol * 100, atol=tol * 100 * float(gb.grad.abs().max()))
    assert ga.grad.shape == gain.shape


def test_gain_only_and_input_only():
    y, gain, lam = inputs((2, 4, 8), torch.float64, 3)
    g1 = gain.clone().requires_grad_(True)
    soft_threshold_gain(y, g1, lam).abs().sum().backward()
    assert g1.grad is not None and g1.grad.shape == gain.shape
    y1 = y.clone().requires_grad_(True)
    soft_threshold_gain(y1, gain, lam).abs().sum().backward()
    assert y1.grad is not None and y1.grad.shape == y.shape


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_zero_thresholds_and_tiny_envelopes(dtype):
    """Rows with a zero threshold (gain only) and envelope values that are 0
    or far below every threshold: the gradient stays finite and equals the
    composed autograd one."""
    y, gain, lam = inputs((2, 5, 12), dtype, 4)
    lam[1] = 0.0
    lam[3] = 0.0
    y[..., 0] = 0
    y[..., 1] = 1e-20
    y[:, 3, 2] = 1e-30 + 0j
    ya, ga = y.clone().requires_grad_(True), gain.clone().requires_grad_(True)
    yb, gb = y.clone().requires_grad_(True), gain.clone().requires_grad_(True)
    out_a = soft_threshold_gain(ya, ga, lam)
    out_b = composed(yb, gb, lam)
    assert torch.isfinite(torch.view_as_real(out_a)).all()
    w = torch.randn(out_a.shape, generator=torch.Generator().manual_seed(5), dtype=out_a.dtype)
    (out_a * w.conj()).real.sum().backward()
    (out_b * w.conj()).real.sum().backward()
    assert torch.isfinite(torch.view_as_real(ya.grad)).all() and torch.isfinite(ga.grad).all()
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    # autograd through |Y| itself turns NaN at |Y| = 1e-20 in FP32 (the
    # square underflows); there the mask is locally constant (1 on a zero
    # threshold row, 0 elsewhere), so the gradient is m g G
    fin = torch.isfinite(torch.view_as_real(yb.grad)).all(-1)
    scale = float(yb.grad[fin].abs().max())
    assert float((ya.grad - yb.grad)[fin].abs().max()) <= tol * scale
    m = (lam[:, None] == 0).to(dtype).expand(y.shape)
    closed = w * (gain[:, None] * m)
    if (~fin).any():
        assert float((ya.grad - closed)[~fin].abs().max()) <= tol * scale
    assert torch.allclose(ga.grad, gb.grad, rtol=tol, atol=tol * float(gb.grad.abs().max()))
