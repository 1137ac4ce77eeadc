"""Adjoint kernels and autograd on the GPU.

* dot-product identities <F x, g> = <x, F^T g> and <G y, z> = <y, G^T z> at the
  differentiable workload's full size (64 x 32768 samples, Q = 8, 128 rows,
  20-2000 Hz) and on rows of 32768 points;
* the adjoints against the oracle's explicit transposes on a tiny plan
  (matrices built column by column from the FP64 CPU oracle);
* torch.autograd.gradcheck on a tiny FP64 plan, and central finite
  differences (eps = 1e-3) of the gain/threshold denoising loss.
"""
import numpy as np
import pytest

import synthetic
from oracle import oracle as o

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def vdot_real(a, b):
    """Real inner product of complex arrays seen as pairs of reals."""
    import torch
    return float(torch.sum(a.real * b.real + a.imag * b.imag))


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-12)])
def test_dot_product_identities_full_size(torch_dev, precision, tol):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    p = qt.Plan(4096.0, 32768, 8.0, 20.0, 2000.0, 128, precision=precision)
    rdt = torch.float64 if precision == "fp64" else torch.float32
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    g = torch.Generator(device="cuda").manual_seed(1)
    B = 64 if precision == "fp32" else 16
    x = torch.randn(B, 32768, device="cuda", dtype=rdt, generator=g)
    gy = torch.randn(B, p.R, p.N_out, device="cuda", dtype=cdt, generator=g)
    lhs = vdot_real(p.forward(x).to(torch.complex128), gy.to(torch.complex128))
    rhs = float(torch.sum(x.double() * p.forward_adjoint(gy).double()))
    assert abs(lhs - rhs) <= tol * max(abs(lhs), 1.0) * 10, (lhs, rhs)
    y = torch.randn(B, p.R, p.N_out, device="cuda", dtype=cdt, generator=g)
    z = torch.randn(B, 32768, device="cuda", dtype=rdt, generator=g)
    lhs = float(torch.sum(p.inverse(y).double() * z.double()))
    rhs = vdot_real(y.to(torch.complex128), p.inverse_adjoint(z).to(torch.complex128))
    assert abs(lhs - rhs) <= tol * max(abs(lhs), 1.0) * 10, (lhs, rhs)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-12)])
def test_dot_product_identities_long_rows(torch_dev, precision, tol):
    """Rows of 32768 points: one workgroup per row in FP32, the two-pass form
    through the workspace in FP64; both adjoints."""
    torch = torch_dev
    import paper_2603_29785_amd as qt
    n = 1 << 20
    p = qt.Plan(16384.0, n, 8.0, 20.0, 4000.0, 64, precision=precision)
    assert p.N_out == 32768
    print("long-row adjoints", precision, flush=True)
    rdt = torch.float64 if precision == "fp64" else torch.float32
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    g = torch.Generator(device="cuda").manual_seed(2)
    B = 2
    x = torch.randn(B, n, device="cuda", dtype=rdt, generator=g)
    gy = torch.randn(B, p.R, p.N_out, device="cuda", dtype=cdt, generator=g)
    lhs = vdot_real(p.forward(x).to(torch.complex128), gy.to(torch.complex128))
    rhs = float(torch.sum(x.double() * p.forward_adjoint(gy).double()))
    assert abs(lhs - rhs) <= tol * max(abs(lhs), 1.0) * 10, (lhs, rhs)
    y = torch.randn(B, p.R, p.N_out, device="cuda", dtype=cdt, generator=g)
    z = torch.randn(B, n, device="cuda", dtype=rdt, generator=g)
    lhs = float(torch.sum(p.inverse(y).double() * z.double()))
    rhs = vdot_real(y.to(torch.complex128), p.inverse_adjoint(z).to(torch.complex128))
    assert abs(lhs - rhs) <= tol * max(abs(lhs), 1.0) * 10, (lhs, rhs)


def test_adjoints_match_oracle_transposes(torch_dev):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    kw = dict(fs=256.0, n=256, q=4.0, f_min=6.0, f_max=100.0, rows=6)
    op = o.OraclePlan(**kw)
    p = qt.Plan(256.0, 256, 4.0, 6.0, 100.0, 6, precision="fp64")
    N, R, M = op.n, op.R, op.N_out
    F = np.stack([op.forward(e).ravel() for e in np.eye(N)], axis=1)              # [R*M, N] complex
    Fr = np.concatenate([F.real, F.imag], axis=0)                                   # [2RM, N]
    G = np.concatenate([np.stack([op.inverse(c.reshape(R, M)) for c in np.eye(R * M)], axis=1),
                        np.stack([op.inverse(1j * c.reshape(R, M)) for c in np.eye(R * M)], axis=1)],
                       axis=1)                                                      # [N, 2RM]
    rng = np.random.default_rng(3)
    gy = rng.standard_normal((3, R, M)) + 1j * rng.standard_normal((3, R, M))
    gx = p.forward_adjoint(torch.from_numpy(gy).cuda()).cpu().numpy()
    ref = (Fr.T @ np.concatenate([gy.real.reshape(3, -1), gy.imag.reshape(3, -1)], axis=1).T).T
    assert np.linalg.norm(gx - ref) <= 1e-12 * np.linalg.norm(ref)
    z = rng.standard_normal((3, N))
    gyz = p.inverse_adjoint(torch.from_numpy(z).cuda()).cpu().numpy()
    refz = (G.T @ z.T).T
    refc = (refz[:, :R * M] + 1j * refz[:, R * M:]).reshape(3, R, M)
    assert np.linalg.norm(gyz - refc) <= 1e-12 * np.linalg.norm(refc)


def test_gradcheck_tiny_fp64(torch_dev):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    from paper_2603_29785_amd.autograd import qtam_forward, qtam_inverse
    p = qt.Plan(128.0, 128, 3.0, 5.0, 60.0, 5, precision="fp64")
    x = torch.randn(2, 128, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: qtam_forward(t, p), (x,), eps=1e-6, atol=1e-8)
    y = torch.randn(2, p.R, p.N_out, dtype=torch.complex128, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: qtam_inverse(t, p), (y,), eps=1e-6, atol=1e-8)


def thresholds_for(plan, torch, fs, n):
    """3 x the median envelope magnitude per row of a noise-only segment."""
    rng = synthetic.rng_for(5, 10_000)
    noise = synthetic.coloured(n, fs, rng)
    rdt = torch.float64 if plan.fp64 else torch.float32
    Y = plan.forward(torch.from_numpy(noise).to(device="cuda", dtype=rdt))
    return 3.0 * Y.abs().median(dim=-1).values


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_denoiser_central_differences(torch_dev, precision):
    """loss = mean((inverse(g * Y * softmask) - clean)^2): autograd (adjoint
    kernels) against central differences with eps = 1e-3 on random gains and,
    in FP64, on input samples (in FP32 a one-sample step moves the loss below
    its own rounding, so only the gains are checked there)."""
    torch = torch_dev
    import paper_2603_29785_amd as qt
    from paper_2603_29785_amd.autograd import GainThresholdDenoiser
    fs, n, B = 4096.0, 32768, 4
    p = qt.Plan(fs, n, 8.0, 20.0, 2000.0, 128, precision=precision)
    rdt = torch.float64 if precision == "fp64" else torch.float32
    noisy, clean = synthetic.differentiable_pairs(B, n, fs, dtype=np.float64)
    xn = torch.from_numpy(noisy).to(device="cuda", dtype=rdt).requires_grad_(True)
    xc = torch.from_numpy(clean).to(device="cuda", dtype=rdt)
    model = GainThresholdDenoiser(p, thresholds_for(p, torch, fs, n))
    with torch.no_grad():
        model.gain.mul_(torch.linspace(0.8, 1.2, p.R, device="cuda", dtype=rdt))

    def loss_fn():
        return torch.mean((model(xn).double() - xc.double()) ** 2)

    loss = loss_fn()
    loss.backward()
    g_gain = model.gain.grad.detach().double().clone()
    g_x = xn.grad.detach().double().clone()
    scale = float(g_gain.abs().max())
    rng = np.random.default_rng(7)
    eps = 1e-3
    rtol = 1e-6 if precision == "fp64" else 5e-2
    for k in rng.choice(p.R, 16, replace=False):
        with torch.no_grad():
            model.gain[k] += eps
            lp = float(loss_fn())
            model.gain[k] -= 2 * eps
            lm = float(loss_fn())
            model.gain[k] += eps
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - float(g_gain[k])) <= rtol * max(abs(fd), 1e-3 * scale), (k, fd, float(g_gain[k]))
    if precision == "fp32":
        return
    xscale = float(g_x.abs().max())
    for idx in rng.choice(B * n, 16, replace=False):
        b, t = divmod(int(idx), n)
        with torch.no_grad():
            xn[b, t] += eps
            lp = float(loss_fn())
            xn[b, t] -= 2 * eps
            lm = float(loss_fn())
            xn[b, t] += eps
        fd = (lp - lm) / (2 * eps)
        ga = float(g_x[b, t])
        assert abs(fd - ga) <= 1e-5 * max(abs(fd), 1e-3 * xscale), (b, t, fd, ga)
