"""Precision study on long segments: 32 segments x 256 s at 8192 Hz (2^21
samples), 512 rows from 5 to 4096 Hz, Q = 12 (N_out 32768).

Every segment: FP32 GPU against FP64 GPU (forward coefficients) and the round
trip of both against the projection x_M. Four sampled segments against the
FP64 CPU oracle in both precisions, on the same input bits: the forward
coefficients, the inverse of the oracle's coefficients (FP32: cast to
complex64 first; both sides invert the same values) and the round trip.
Bars: rel-L2 per segment FP32 <= 1e-5, FP64 <= 1e-12. The per-segment errors
are printed.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import synthetic
from oracle import oracle as o

pytestmark = pytest.mark.gpu

FS, N, Q, FMIN, FMAX, R, B = 8192.0, 1 << 21, 12.0, 5.0, 4096.0, 512, 32
SAMPLED = (0, 11, 22, 31)
TOL = {"fp32": 1e-5, "fp64": 1e-12}


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def gpu_plans():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_29785_amd as qt
    p32 = qt.Plan(FS, N, Q, FMIN, FMAX, R, precision="fp32")
    p64 = qt.Plan(FS, N, Q, FMIN, FMAX, R, precision="fp64")
    assert p32.N_out == p64.N_out == 32768
    return torch, p32, p64


def test_precision_study_every_segment(gpu_plans):
    torch, p32, p64 = gpu_plans
    mask = torch.from_numpy(p64.mask).cuda()
    e_coef, e_rt32, e_rt64 = [], [], []
    chunk = 4
    for b0 in range(0, B, chunk):
        x = synthetic.batched_segments(chunk, N, FS, workload=4, first=b0, dtype=np.float64)
        x32 = torch.from_numpy(x.astype(np.float32)).cuda()
        x64 = x32.double()                      # same input bits for both precisions
        Y32 = p32.forward(x32)
        Y64 = p64.forward(x64)
        d = (Y32.to(torch.complex128) - Y64).reshape(chunk, -1)
        e_coef += (torch.linalg.norm(d, dim=1) / torch.linalg.norm(Y64.reshape(chunk, -1), dim=1)).tolist()
        xm = torch.fft.irfft(torch.fft.rfft(x64, dim=-1) * mask, n=N, dim=-1)
        r32 = p32.inverse(Y32).double()
        r64 = p64.inverse(Y64)
        e_rt32 += (torch.linalg.norm(r32 - xm, dim=1) / torch.linalg.norm(xm, dim=1)).tolist()
        e_rt64 += (torch.linalg.norm(r64 - xm, dim=1) / torch.linalg.norm(xm, dim=1)).tolist()
        del Y32, Y64
    print("coef rel-L2 FP32 vs FP64 per segment: max %.3e median %.3e" % (max(e_coef), np.median(e_coef)))
    print("round trip rel-L2 FP32: max %.3e median %.3e" % (max(e_rt32), np.median(e_rt32)))
    print("round trip rel-L2 FP64: max %.3e median %.3e" % (max(e_rt64), np.median(e_rt64)))
    assert max(e_coef) <= 1e-5 and max(e_rt32) <= 1e-5 and max(e_rt64) <= 1e-12


def _oracle_segment(op, x):
    """Oracle results of one segment: Y, x_M, inverse of Y (FP64) and of Y
    cast to complex64 (what the FP32 inverse is handed)."""
    Yo = op.forward(x)
    Yc = Yo.astype(np.complex64).astype(np.complex128)
    return Yo, Yc, op.project(x), op.inverse(Yo), op.inverse(Yc)


def test_precision_study_against_oracle(gpu_plans):
    torch, p32, p64 = gpu_plans
    op = o.OraclePlan(fs=FS, n=N, q=Q, f_min=FMIN, f_max=FMAX, rows=R)
    xs = {s: synthetic.batched_segments(1, N, FS, workload=4, first=s, dtype=np.float64)[0]
          .astype(np.float32).astype(np.float64) for s in SAMPLED}
    with ThreadPoolExecutor(max_workers=len(SAMPLED)) as ex:
        ora = dict(zip(SAMPLED, ex.map(lambda s: _oracle_segment(op, xs[s]), SAMPLED)))
    for s in SAMPLED:
        Yo, Yc, xm, xo, xoc = ora[s]
        for prec, plan, dt, cdt, Yin, xin_ref in (
                ("fp32", p32, torch.float32, torch.complex64, Yc, xoc),
                ("fp64", p64, torch.float64, torch.complex128, Yo, xo)):
            xd = torch.from_numpy(xs[s]).to(dtype=dt, device="cuda")
            Yg = plan.forward(xd)
            e_y = rel(Yg.cpu().numpy(), Yo)
            e_rt = rel(plan.inverse(Yg).cpu().numpy(), xm)
            del Yg
            Yd = torch.from_numpy(Yin).to(dtype=cdt, device="cuda")
            e_inv = rel(plan.inverse(Yd).cpu().numpy(), xin_ref)
            del Yd
            print("segment %2d %s vs oracle: coef %.3e, inverse of oracle coef %.3e, round trip %.3e"
                  % (s, prec, e_y, e_inv, e_rt), flush=True)
            assert e_y <= TOL[prec] and e_inv <= TOL[prec] and e_rt <= TOL[prec], (s, prec)
