"""Precision study on long segments: 32 segments x 256 s at 8192 Hz (2^21
samples), 512 rows from 5 to 4096 Hz, Q = 12 (N_out 32768).

FP32 GPU against FP64 GPU on every segment (forward coefficients and round
trip), and FP64 GPU against the FP64 CPU oracle on sampled segments. The
per-segment errors are printed."""
import numpy as np
import pytest

import synthetic
from oracle import oracle as o

pytestmark = pytest.mark.gpu

FS, N, Q, FMIN, FMAX, R, B = 8192.0, 1 << 21, 12.0, 5.0, 4096.0, 512, 32


def test_precision_study():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_29785_amd as qt
    p32 = qt.Plan(FS, N, Q, FMIN, FMAX, R, precision="fp32")
    p64 = qt.Plan(FS, N, Q, FMIN, FMAX, R, precision="fp64")
    assert p32.N_out == 32768
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
    # FP64 GPU against the FP64 CPU oracle on two sampled segments
    op = o.OraclePlan(fs=FS, n=N, q=Q, f_min=FMIN, f_max=FMAX, rows=R)
    for s in (0, B - 1):
        x = synthetic.batched_segments(1, N, FS, workload=4, first=s, dtype=np.float64)[0]
        x = x.astype(np.float32).astype(np.float64)
        Yo = op.forward(x)
        Yg = p64.forward(torch.from_numpy(x).cuda()).cpu().numpy()
        e = np.linalg.norm(Yg - Yo) / np.linalg.norm(Yo)
        print("segment %d: FP64 GPU vs oracle coef rel-L2 %.3e" % (s, e))
        assert e <= 1e-12
