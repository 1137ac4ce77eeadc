"""Composite multi-Q / multi-window banks on the GPU (App. A extension):
coefficients and reconstruction against the FP64 oracle, fused row statistics
against the oracle's, and optimal-plane selection per segment.

Bars: coefficients and reconstruction as for plain plans (rel-L2 per segment
FP32 <= 1e-5, FP64 <= 1e-12); row statistics rel <= 1e-5 (FP32) / 1e-12 (FP64)
on rows holding at least 1e-6 of the segment's energy; the selected plane is
the oracle's unless the oracle's two best scores lie within 1e-4 of each
other (then either is valid: the choice must still score within 1e-4 of the
best); the gathered rows are a bitwise copy of the chosen plane.
"""
import numpy as np
import pytest

import synthetic
from oracle import oracle as o

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-12}
WINS = {"bisquare": o.WIN_BISQUARE, "hann": o.WIN_HANN, "kaiser": o.WIN_KAISER, "tukey": o.WIN_TUKEY,
        "planck": o.WIN_PLANCK}


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


def plans(planes, precision, fs, n, f_min, f_max, rows, **kw):
    import paper_2603_29785_amd as qt
    gp = qt.Plan(fs, n, 1.0, f_min, f_max, rows, precision=precision, planes=planes, **kw)
    op = o.OraclePlan(fs=fs, n=n, q=1.0, f_min=f_min, f_max=f_max, rows=rows,
                      planes=[(q, WINS[w], a) for q, w, a in planes], **kw)
    assert gp.R == op.R and gp.N_out == op.N_out and gp.planes == len(planes)
    return gp, op


def device_signal(torch, x, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dtype=dt, device="cuda")
    return xd, xd.double().cpu().numpy()


CASES = [
    # three bisquare planes, the workload's Q set (analytic forward weights)
    ("bisq3", [(4.0, "bisquare", 0.0), (8.0, "bisquare", 0.0), (16.0, "bisquare", 0.0)],
     dict(fs=4096.0, n=65536, f_min=10.0, f_max=2048.0, rows=96)),
    # mixed windows (table weights), rows of several lengths
    ("mixed", [(3.0, "hann", 0.0), (9.0, "kaiser", 6.0), (27.0, "tukey", 0.4), (12.0, "planck", 0.3)],
     dict(fs=4096.0, n=32768, f_min=16.0, f_max=1800.0, rows=40)),
]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("name,planes,kw", CASES, ids=[c[0] for c in CASES])
def test_composite_forward_inverse_and_metrics(torch_dev, name, planes, kw, precision):
    torch = torch_dev
    print("composite", name, precision, flush=True)
    gp, op = plans(planes, precision, **kw)
    batch = 3
    x = synthetic.batched_segments(batch, kw["n"], kw["fs"], workload=21)
    xd, xh = device_signal(torch, x, precision)
    Y, M = gp.forward_metric(xd)
    Y2 = gp.forward(xd)
    torch.cuda.synchronize()
    assert torch.equal(Y, Y2)                       # statistics do not change the coefficients
    Yo = op.forward(xh)
    Yg = Y.cpu().numpy()
    assert rel_rows(Yg, Yo).max() <= TOL[precision]
    # reconstruction from the whole bank
    xr = gp.inverse(Y).double().cpu().numpy()
    assert rel_rows(xr, op.inverse(Yo)).max() <= TOL[precision]
    assert rel_rows(xr, op.project(xh)).max() <= TOL[precision]
    # fused row statistics
    e_o, p_o = op.row_stats(Yo)
    Mg = M.cpu().numpy()
    tot = e_o.sum(axis=1, keepdims=True)
    live = e_o >= 1e-6 * tot
    assert (np.abs(Mg.real - e_o) / e_o)[live].max() <= TOL[precision]
    assert (np.abs(Mg.imag - p_o) / p_o)[live].max() <= 10 * TOL[precision]
    assert np.all(np.abs(Mg.real - e_o)[~live] <= 1e-4 * tot.repeat(e_o.shape[1], 1)[~live])


def check_selection(gp, op, Y, M, Yo, kind, precision):
    score, best, Yb = gp.select_planes(Y, M, kind)
    s_o = op.plane_scores(Yo, kind)
    sg, bg, Ybg = score.cpu().numpy(), best.cpu().numpy(), Yb.cpu().numpy()
    assert np.all(np.abs(sg - s_o) <= 10 * TOL[precision] * np.abs(s_o).max(axis=1, keepdims=True))
    R = gp.rows_per_plane
    Yg = Y.cpu().numpy()
    for b in range(Yg.shape[0]):
        top = np.sort(s_o[b])[::-1]
        if len(top) < 2 or top[0] - top[1] > 1e-4 * top[0]:
            assert bg[b] == int(np.argmax(s_o[b])), (b, kind)
        else:
            assert s_o[b, bg[b]] >= (1 - 1e-4) * top[0]
        assert np.array_equal(Ybg[b], Yg[b, R * bg[b]:R * (bg[b] + 1)])
    return bg


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_selection_per_segment(torch_dev, precision):
    """A steady tone and a click in one batch: under the peak metric the tone
    keeps the high-Q plane and the click the low-Q plane."""
    torch = torch_dev
    print("selection", precision, flush=True)
    planes = [(2.0, "bisquare", 0.0), (8.0, "bisquare", 0.0), (32.0, "bisquare", 0.0)]
    gp, op = plans(planes, precision, fs=4096.0, n=16384, f_min=20.0, f_max=1500.0, rows=48)
    N = gp.N
    b0 = int(op.row_table()["centre"][30])
    tone = np.cos(2 * np.pi * (b0 + 0.25) * np.arange(N) / N)
    click = np.zeros(N)
    click[N // 3] = 40.0
    noise = synthetic.batched_segments(2, N, 4096.0, workload=22).astype(np.float64)
    x = np.stack([tone, click, noise[0], noise[1]])
    xd, xh = device_signal(torch, x, precision)
    Y, M = gp.forward_metric(xd)
    Yo = op.forward(xh)
    bp = check_selection(gp, op, Y, M, Yo, "peak", precision)
    assert bp[0] == 2 and bp[1] == 0
    check_selection(gp, op, Y, M, Yo, "energy", precision)


def test_long_row_composite_statistics(torch_dev):
    """Rows longer than one workgroup take the four-step row path, whose
    statistics are read back from Y."""
    torch = torch_dev
    print("long-row composite", flush=True)
    planes = [(2.0, "bisquare", 0.0), (6.0, "hann", 0.0)]
    gp, op = plans(planes, "fp32", fs=4096.0, n=262144, f_min=200.0, f_max=2000.0, rows=8, cap_mode=o.CAP_NONE)
    assert gp.N_out > 16384
    x = synthetic.batched_segments(2, gp.N, 4096.0, workload=23)
    xd, xh = device_signal(torch, x, "fp32")
    Y, M = gp.forward_metric(xd)
    Yo = op.forward(xh)
    assert rel_rows(Y.cpu().numpy(), Yo).max() <= 1e-5
    e_o, p_o = op.row_stats(Yo)
    Mg = M.cpu().numpy()
    assert np.abs(Mg.real / e_o - 1).max() <= 1e-5
    assert np.abs(Mg.imag / p_o - 1).max() <= 1e-4
    check_selection(gp, op, Y, M, Yo, "energy", "fp32")


def test_composite_statistics_rows_32768(torch_dev):
    """Rows of 32768 points run in one workgroup (FP32): statistics taken from
    the registers of a 1024-thread transform."""
    torch = torch_dev
    print("composite rows 32768", flush=True)
    planes = [(2.0, "bisquare", 0.0), (6.0, "hann", 0.0)]
    gp, op = plans(planes, "fp32", fs=4096.0, n=262144, f_min=200.0, f_max=1000.0, rows=8, cap_mode=o.CAP_NONE)
    assert gp.N_out == 32768
    x = synthetic.batched_segments(2, gp.N, 4096.0, workload=23)
    xd, xh = device_signal(torch, x, "fp32")
    Y, M = gp.forward_metric(xd)
    Yo = op.forward(xh)
    assert rel_rows(Y.cpu().numpy(), Yo).max() <= 1e-5
    assert torch.equal(Y, gp.forward(xd))
    e_o, p_o = op.row_stats(Yo)
    Mg = M.cpu().numpy()
    assert np.abs(Mg.real / e_o - 1).max() <= 1e-5
    assert np.abs(Mg.imag / p_o - 1).max() <= 1e-4
    check_selection(gp, op, Y, M, Yo, "peak", "fp32")


def test_selection_empty_and_errors(torch_dev):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    gp, _ = plans([(4.0, "bisquare", 0.0), (8.0, "bisquare", 0.0)], "fp32", fs=1024.0, n=4096, f_min=10.0,
                  f_max=400.0, rows=16)
    Y = torch.zeros((0, gp.R, gp.N_out), dtype=torch.complex64, device="cuda")
    M = torch.zeros((0, gp.R), dtype=torch.complex64, device="cuda")
    s, b, yb = gp.select_planes(Y, M, "energy")
    assert s.shape == (0, 2) and b.shape == (0,) and yb.shape == (0, 16, gp.N_out)
    with pytest.raises(ValueError):
        gp.select_planes(torch.zeros((1, gp.R, gp.N_out), dtype=torch.complex64, device="cuda"),
                         torch.zeros((1, gp.R + 1), dtype=torch.complex64, device="cuda"))
    with pytest.raises(qt.QtamError):
        gp.select_planes(torch.zeros((1, gp.R, gp.N_out), dtype=torch.complex64, device="cuda"),
                         torch.zeros((1, gp.R), dtype=torch.complex64, device="cuda"), kind=5)
