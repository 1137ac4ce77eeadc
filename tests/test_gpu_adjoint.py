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


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-12)])
def test_adjoints_match_oracle_transposes(torch_dev, precision, tol):
    """Both adjoints against the transposes of the oracle's forward and
    inverse, built column by column. FP32 runs on the FP32-cast inputs (the
    reference uses the same cast values) at the FP32 parity bar 1e-5: the
    adjoints run the forward and inverse kernels with other tables, so their
    rounding is that of the forward and inverse."""
    torch = torch_dev
    import paper_2603_29785_amd as qt
    kw = dict(fs=256.0, n=256, q=4.0, f_min=6.0, f_max=100.0, rows=6)
    op = o.OraclePlan(**kw)
    p = qt.Plan(256.0, 256, 4.0, 6.0, 100.0, 6, precision=precision)
    rdt = torch.float64 if precision == "fp64" else torch.float32
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    cast = (lambda a: a.astype(np.complex64).astype(np.complex128)) if precision == "fp32" else (lambda a: a)
    castr = (lambda a: a.astype(np.float32).astype(np.float64)) if precision == "fp32" else (lambda a: a)
    N, R, M = op.n, op.R, op.N_out
    F = np.stack([op.forward(e).ravel() for e in np.eye(N)], axis=1)              # [R*M, N] complex
    Fr = np.concatenate([F.real, F.imag], axis=0)                                   # [2RM, N]
    G = np.concatenate([np.stack([op.inverse(c.reshape(R, M)) for c in np.eye(R * M)], axis=1),
                        np.stack([op.inverse(1j * c.reshape(R, M)) for c in np.eye(R * M)], axis=1)],
                       axis=1)                                                      # [N, 2RM]
    rng = np.random.default_rng(3)
    gy = cast(rng.standard_normal((3, R, M)) + 1j * rng.standard_normal((3, R, M)))
    gx = p.forward_adjoint(torch.from_numpy(gy).to(dtype=cdt, device="cuda")).cpu().numpy()
    ref = (Fr.T @ np.concatenate([gy.real.reshape(3, -1), gy.imag.reshape(3, -1)], axis=1).T).T
    e1 = np.linalg.norm(gx - ref) / np.linalg.norm(ref)
    z = castr(rng.standard_normal((3, N)))
    gyz = p.inverse_adjoint(torch.from_numpy(z).to(dtype=rdt, device="cuda")).cpu().numpy()
    refz = (G.T @ z.T).T
    refc = (refz[:, :R * M] + 1j * refz[:, R * M:]).reshape(3, R, M)
    e2 = np.linalg.norm(gyz - refc) / np.linalg.norm(refc)
    print(f"{precision}: forward adjoint {e1:.3e}, inverse adjoint {e2:.3e}", flush=True)
    assert e1 <= tol and e2 <= tol


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


def _central(loss_fn, bump, coord, eps):
    import torch
    with torch.no_grad():
        bump(coord, eps)
        lp = float(loss_fn())
        bump(coord, -2 * eps)
        lm = float(loss_fn())
        bump(coord, eps)
    return (lp - lm) / (2 * eps)


def _fd_errors(fds, grads, scale):
    return [abs(f - g) / max(abs(f), 1e-3 * scale) for f, g in zip(fds, grads)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_denoiser_central_differences(torch_dev, precision):
    """loss = mean((inverse(g * Y * softmask) - clean)^2): the autograd
    gradient (adjoint kernels) against central differences with eps = 1e-3 on
    32 random gains and 32 random input samples. Bars: FP64 1e-6, FP32 1e-2,
    relative to max(|fd|, 1e-3 x the largest gradient entry of that kind).

    FP32 input samples: the FP32 gradient is checked against central
    differences of the same loss (same thresholds, gains and input bits)
    evaluated through the FP64 path. A one-sample step of 1e-3 moves the FP32
    loss by less than its own rounding here: the spectrum's FP32 rounding is
    relative to the whole signal, whose coloured noise below 20 Hz carries
    orders of magnitude more energy than the band the rows keep (measured:
    FP32 differences of FP32 losses miss by a median 27%)."""
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
    rng = np.random.default_rng(7)
    eps = 1e-3
    rtol = 1e-6 if precision == "fp64" else 1e-2

    def bump_gain(k, d):
        model.gain[int(k)] += d

    ks = rng.choice(p.R, 32, replace=False)
    e_gain = _fd_errors([_central(loss_fn, bump_gain, k, eps) for k in ks],
                        [float(g_gain[int(k)]) for k in ks], float(g_gain.abs().max()))

    idx = rng.choice(B * n, 32, replace=False)
    if precision == "fp64":
        xf, mf, lf = xn, model, loss_fn
    else:
        # the same loss through the FP64 path: same input bits, thresholds and gains
        p64 = qt.Plan(fs, n, 8.0, 20.0, 2000.0, 128, precision="fp64")
        mf = GainThresholdDenoiser(p64, model.thresholds.detach().double())
        with torch.no_grad():
            mf.gain.copy_(model.gain.detach().double())
        xf = xn.detach().double()
        xc64 = xc.double()

        def lf():
            return torch.mean((mf(xf) - xc64) ** 2)

    def bump_x(i, d):
        b, t = divmod(int(i), n)
        xf[b, t] += d

    e_x = _fd_errors([_central(lf, bump_x, i, eps) for i in idx],
                     [float(g_x.reshape(-1)[int(i)]) for i in idx], float(g_x.abs().max()))
    for kind, errs in (("gain", e_gain), ("input", e_x)):
        print(f"{precision} {kind}: relative FD error max {max(errs):.3e} median {np.median(errs):.3e}"
              f" over {len(errs)} coordinates", flush=True)
    assert max(e_gain) <= rtol and max(e_x) <= rtol, (e_gain, e_x)
