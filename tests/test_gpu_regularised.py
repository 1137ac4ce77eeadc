"""Regularised stop-band windows on the GPU (Sec. III; App. A): coefficients
and canonical inverse against the oracle, and recovery of the signal from a
single tile by spectral division.

Bars: coefficients and canonical inverse as for plain plans (rel-L2 per
segment FP32 <= 1e-5, FP64 <= 1e-12). Single-tile recovery divides by the
window, so rounding is amplified by about max W / min W = 1/eps: the bar is
2000 * u / eps with u the unit roundoff (FP32 eps = 1e-2: 1.2e-3; FP64
eps = 1e-6: 2.2e-7), against the oracle's recovery from the same envelopes
and, in FP64, against the signal itself.
"""
import numpy as np
import pytest

import synthetic
from oracle import oracle as o

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-12}
UNIT = {"fp32": 2.0 ** -24, "fp64": 2.0 ** -53}
EPS = {"fp32": 1e-2, "fp64": 1e-6}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_rows(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


# (fs, N, N_out): N a power of two (N_out = N), the 6 s x 4096 Hz segment
# (N/2 = 3 * 4096, N_out = 16384 < N), N/2 = 5 * 512 (N_out = 4096 < N) and
# N/2 = 3 * 8192 (N_out = 32768 < N).
# With N_out < N a row's band 0..N/2 reaches beyond N_out/2 on one side of
# its centre for most rows, and only the wrap of slots (c - s) mod N_out
# places those bins.
SIZES = [(1024.0, 4096, 4096), (4096.0, 24576, 16384), (1024.0, 5120, 4096), (4096.0, 49152, 32768)]


@pytest.mark.parametrize("fs,n,n_out", SIZES)
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_regularised_forward_inverse_and_single_tile(torch_dev, precision, fs, n, n_out):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    q, fmin, fmax, R, B = 8.0, 10.0, 400.0, 16, 3
    eps = EPS[precision]
    gp = qt.Plan(fs, n, q, fmin, fmax, R, precision=precision, window_eps=eps)
    op = o.OraclePlan(fs=fs, n=n, q=q, f_min=fmin, f_max=fmax, rows=R, eps=eps)
    assert gp.N_out == op.N_out == n_out
    if n_out < n:
        t = op.row_table()
        off = (t["centre"] - t["lo"] > n_out // 2) | (t["hi"] - t["centre"] >= n_out // 2)
        assert off.sum() >= R // 2
    print("regularised", precision, "eps", eps, "N", n, "N_out", n_out, flush=True)
    x = np.stack([synthetic.injected_segment(n, fs, synthetic.rng_for(15, i))[0] for i in range(B)])
    dt = torch.float64 if precision == "fp64" else torch.float32
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    xd = torch.from_numpy(x).to(dtype=dt, device="cuda")
    xh = xd.double().cpu().numpy()
    Yo = op.forward(xh)
    Y = gp.forward(xd)
    assert rel_rows(Y.cpu().numpy(), Yo).max() <= TOL[precision]
    Yc = torch.from_numpy(Yo).to(dtype=cdt, device="cuda")
    Ych = Yc.cpu().numpy().astype(np.complex128)
    assert rel_rows(gp.inverse(Yc).cpu().numpy(), op.inverse(Ych)).max() <= TOL[precision]
    bar = 2000.0 * UNIT[precision] / eps
    # rows of 16384 (FP64) and 32768 points take the two-pass transforms
    # (FP32 32768: one workgroup exchanging through half the row in LDS)
    for k in (0, R // 2, R - 1):
        xt = gp.tile_inverse(Yc, k).cpu().numpy()
        assert rel_rows(xt, op.tile_inverse(Ych, k)).max() <= bar, k
        if precision == "fp64":
            assert rel_rows(gp.tile_inverse(Y, k).cpu().numpy(), xh).max() <= bar, k


def test_single_tile_needs_regularised_windows(torch_dev):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    gp = qt.Plan(1024.0, 4096, 8.0, 10.0, 400.0, 16)
    y = torch.zeros((1, 16, gp.N_out), dtype=torch.complex64, device="cuda")
    with pytest.raises(qt.QtamError) as e:
        gp.tile_inverse(y, 0)
    assert e.value.status == 1


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_planck_taper_tails_single_tile(torch_dev, precision):
    """A Planck-taper plan whose tapers fall far below eps inside their
    supports (N = 3072 at 256 Hz, Q 4.1, 15 rows from 20.9 Hz): eps floors
    every window, so the single-tile inverse of every row stays within the
    conditioning bar of the oracle's (with only the zeros replaced it missed
    by order 1 in both precisions)."""
    torch = torch_dev
    import paper_2603_29785_amd as qt
    fs, n, q, fmin, fmax, R = 256.0, 3072, 4.107609620941872, 20.927358999587156, 128.0, 15
    eps = EPS[precision]
    gp = qt.Plan(fs, n, q, fmin, fmax, R, window="planck", window_param=0.25, precision=precision, window_eps=eps)
    op = o.OraclePlan(fs=fs, n=n, q=q, f_min=fmin, f_max=fmax, rows=R, window=o.WIN_PLANCK, window_param=0.25,
                      eps=eps)
    x = np.stack([synthetic.injected_segment(n, fs, synthetic.rng_for(16, i))[0] for i in range(2)])
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    Yo = op.forward(x.astype(np.float32).astype(np.float64) if precision == "fp32" else x)
    Yc = torch.from_numpy(Yo).to(dtype=cdt, device="cuda")
    Ych = Yc.cpu().numpy().astype(np.complex128)
    bar = 2000.0 * UNIT[precision] / eps
    worst = max(rel_rows(gp.tile_inverse(Yc, k).cpu().numpy(), op.tile_inverse(Ych, k)).max() for k in range(R))
    print(f"planck {precision}: single-tile inverse vs oracle, worst row {worst:.3e} (bar {bar:.1e})", flush=True)
    assert worst <= bar


def _random_regularised():
    import test_gpu_parity as tp
    return tp.random_plans(5102, 8, log2n=(11, 16), log2n_odd=(10, 14), row_range=(3, 25), kinds=(0,))


RANDOM_REG = _random_regularised()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("spec", RANDOM_REG, ids=[f"N{s[1]}_R{s[5]}_{s[6]}" for s in RANDOM_REG])
def test_random_regularised_plans(torch_dev, spec, precision):
    """Seeded random plans (every window, N = r 2^k) with the stop band:
    coefficients and inverse at the bars, and the single-tile inverse of the
    first, middle and last rows within the conditioning bar of the oracle's
    (the sweep that found the taper tails of reading 21)."""
    torch = torch_dev
    import paper_2603_29785_amd as qt
    fs, n, q, fmin, fmax, rows, wname, wid, wparam, _ = spec
    eps = EPS[precision]
    gp = qt.Plan(fs, n, q, fmin, fmax, rows, window=wname, window_param=wparam, precision=precision, window_eps=eps)
    op = o.OraclePlan(fs=fs, n=n, q=q, f_min=fmin, f_max=fmax, rows=rows, window=wid, window_param=wparam, eps=eps)
    x = np.stack([synthetic.injected_segment(n, fs, synthetic.rng_for(62, j))[0] for j in range(2)])
    dt = torch.float64 if precision == "fp64" else torch.float32
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    xd = torch.from_numpy(x).to(dtype=dt, device="cuda")
    xh = xd.double().cpu().numpy()
    Yo = op.forward(xh)
    e_y = rel_rows(gp.forward(xd).cpu().numpy(), Yo).max()
    Yc = torch.from_numpy(Yo).to(dtype=cdt, device="cuda")
    Ych = Yc.cpu().numpy().astype(np.complex128)
    e_x = rel_rows(gp.inverse(Yc).cpu().numpy(), op.inverse(Ych)).max()
    bar = 2000.0 * UNIT[precision] / eps
    e_t = max(rel_rows(gp.tile_inverse(Yc, k).cpu().numpy(), op.tile_inverse(Ych, k)).max()
              for k in (0, rows // 2, rows - 1))
    print(f"random regularised {spec[:6]} {wname} {precision}: coef {e_y:.2e} inverse {e_x:.2e} tile {e_t:.2e} "
          f"(bar {bar:.1e})", flush=True)
    assert e_y <= TOL[precision] and e_x <= TOL[precision] and e_t <= bar
