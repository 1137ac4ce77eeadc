"""The denoiser's mask fused into the inverse transform and its adjoint
(qtam_inverse_masked / qtam_inverse_masked_adjoint, through the C ABI)
against the two-step path on the same GPU tensors (qtam_mask_forward then
qtam_inverse; qtam_inverse_adjoint then qtam_mask_backward): the same kernels'
arithmetic on the same values, so the reconstructions and the input
gradients are compared bit for bit; the gain gradient adds its terms in
another order and is held to the FP32 / FP64 bars (1e-5 / 1e-12 relative to
its largest entry). Also: the fused inverse of the oracle's coefficients
against the oracle's inverse of the masked coefficients, a workspace that
forces chunks, an empty batch, and the two-step fallback on plans whose rows
take more than one workgroup."""
import numpy as np
import pytest

import synthetic
from oracle import oracle as o

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-12}

# (what, fs, N, Q, f_min, f_max, R): the training step's plan (N_out 2048,
# one row per pair of waves) and a small one (N_out 256: four rows per wave)
PLANS = [("training plan", 4096.0, 32768, 8.0, 20.0, 2000.0, 128),
         ("small plan", 1024.0, 4096, 8.0, 10.0, 400.0, 12)]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_max(a, b):
    return float((a - b).abs().max() / max(float(b.abs().max()), 1e-300))


def inputs(torch, p, B, seed):
    rdt = torch.float64 if p.fp64 else torch.float32
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn(B, p.N, dtype=rdt, device="cuda", generator=g)
    y = p.forward(x)
    lam = 0.5 * y.abs().median(dim=-1).values.median(dim=0).values   # a median-level threshold per row
    lam[1] = 0.0                                                      # a gain-only row
    gain = torch.linspace(-0.5, 1.5, p.R, dtype=rdt, device="cuda")
    gx = torch.randn(B, p.N, dtype=rdt, device="cuda", generator=g)
    return y, gain, lam.contiguous(), gx


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("spec", PLANS, ids=[s[0].replace(" ", "_") for s in PLANS])
def test_fused_equals_two_step(torch_dev, spec, precision):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    what, fs, n, q, fmin, fmax, rows = spec
    p = qt.Plan(fs, n, q, fmin, fmax, rows, precision=precision)
    assert p.masked_inverse_supported
    y, gain, lam, gx = inputs(torch, p, 5, 3)
    x_f = p.inverse_masked(y, gain, lam)
    x_2 = p.inverse(p.mask_forward(y, gain, lam))
    gy_f, gg_f = p.inverse_masked_adjoint(gx, y, gain, lam)
    gy_2, gg_2 = p.mask_backward(y, gain, lam, p.inverse_adjoint(gx))
    e = rel_max(gg_f, gg_2)
    print(f"{what} {precision}: reconstruction equal {torch.equal(x_f, x_2)}, input gradient equal "
          f"{torch.equal(gy_f, gy_2)}, gain gradient {e:.3e}", flush=True)
    assert torch.equal(x_f, x_2)
    assert torch.equal(gy_f, gy_2)
    assert e <= TOL[precision]
    # the adjoint again: identical bits
    gy_3, gg_3 = p.inverse_masked_adjoint(gx, y, gain, lam)
    assert torch.equal(gy_3, gy_f) and torch.equal(gg_3, gg_f)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_fused_inverse_against_oracle(torch_dev, precision):
    """x = inverse(mask(Y)) for the oracle's coefficients of two segments,
    against the oracle's inverse of the same coefficients masked in FP64."""
    torch = torch_dev
    import paper_2603_29785_amd as qt
    _, fs, n, q, fmin, fmax, rows = PLANS[1]
    p = qt.Plan(fs, n, q, fmin, fmax, rows, precision=precision)
    op = o.OraclePlan(fs=fs, n=n, q=q, f_min=fmin, f_max=fmax, rows=rows)
    x = np.stack([synthetic.injected_segment(n, fs, synthetic.rng_for(41, i))[0] for i in range(2)])
    if precision == "fp32":
        x = x.astype(np.float32).astype(np.float64)
    Y = op.forward(x)
    if precision == "fp32":
        Y = Y.astype(np.complex64).astype(np.complex128)
    lam = 0.5 * np.median(np.abs(Y), axis=(0, 2))
    gain = np.linspace(-0.5, 1.5, rows)
    cdt = torch.complex64 if precision == "fp32" else torch.complex128
    rdt = torch.float32 if precision == "fp32" else torch.float64
    xr = p.inverse_masked(torch.from_numpy(Y).to(cdt).cuda(), torch.from_numpy(gain).to(rdt).cuda(),
                          torch.from_numpy(lam).to(rdt).cuda()).cpu().numpy()
    r = np.maximum(np.abs(Y), np.finfo(np.float64).tiny)
    Ym = Y * (gain[:, None] * np.maximum(0.0, 1.0 - lam[:, None] / r))
    ref = op.inverse(Ym)
    e = np.linalg.norm(xr - ref, axis=1) / np.linalg.norm(ref, axis=1)
    print(f"{precision}: fused inverse vs oracle {e.max():.3e}", flush=True)
    assert e.max() <= TOL[precision]


def test_chunked_workspace_and_empty_batch(torch_dev):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    _, fs, n, q, fmin, fmax, rows = PLANS[0]
    p = qt.Plan(fs, n, q, fmin, fmax, rows)
    y, gain, lam, gx = inputs(torch, p, 6, 5)
    gy_a, gg_a = p.inverse_masked_adjoint(gx, y, gain, lam)
    # the partial sums of all 6 segments plus the transform workspace of one segment: 6 chunks
    part = (6 * rows * 4 + 255) // 256 * 256
    small = torch.empty(part + p.workspace_bytes(1), dtype=torch.uint8, device="cuda")
    gy_b, gg_b = p.inverse_masked_adjoint(gx, y, gain, lam, ws=small)
    assert torch.equal(gy_a, gy_b) and torch.equal(gg_a, gg_b)
    x_a = p.inverse_masked(y, gain, lam)
    x_b = p.inverse_masked(y, gain, lam, ws=torch.empty(p.workspace_bytes(1), dtype=torch.uint8, device="cuda"))
    assert torch.equal(x_a, x_b)
    with pytest.raises(qt.QtamError):   # not even the partial sums fit
        p.inverse_masked_adjoint(gx, y, gain, lam, ws=torch.empty(part, dtype=torch.uint8, device="cuda"))
    e = torch.zeros((0, p.R, p.N_out), dtype=torch.complex64, device="cuda")
    assert p.inverse_masked(e, gain, lam).shape == (0, p.N)
    gy0, gg0 = p.inverse_masked_adjoint(torch.zeros((0, p.N), device="cuda"), e, gain, lam)
    assert gy0.shape == e.shape and torch.equal(gg0, torch.zeros_like(gain))


def test_two_step_fallback_on_long_rows(torch_dev):
    """Rows of 16384 points in FP64 take two passes: the fused calls report
    QTAM_ERR_UNSUPPORTED and masked_inverse runs the mask and the inverse as
    two steps, with the same results as those two calls."""
    torch = torch_dev
    import paper_2603_29785_amd as qt
    from paper_2603_29785_amd.autograd import masked_inverse
    p = qt.Plan(4096.0, 24576, 8.0, 10.0, 2048.0, 62, precision="fp64", n_out=16384)
    assert not p.masked_inverse_supported
    y, gain, lam, gx = inputs(torch, p, 2, 7)
    with pytest.raises(qt.QtamError) as ex:
        p.inverse_masked(y, gain, lam)
    assert ex.value.status == qt.binding.QTAM_ERR_UNSUPPORTED
    assert torch.equal(masked_inverse(y, gain, lam, p), p.inverse(p.mask_forward(y, gain, lam)))
