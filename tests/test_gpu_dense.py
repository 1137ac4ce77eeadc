"""Dense full-rate tiles on the GPU (App. C): the envelopes re-modulated and
up-sampled to N samples per row, against the oracle's direct evaluation of
T_k[tau] = (1/N) sum_b X[b] W_k[b] e^{+2 pi i b tau / N}.

Bars: rel-L2 per segment FP32 <= 1e-5, FP64 <= 1e-12 (from the GPU's own
forward output, and from the oracle's envelopes cast to the device precision).
"""
import numpy as np
import pytest

import synthetic
from oracle import oracle as o

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-12}


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


CASES = [
    # (fs, N, Q, f_min, f_max, R, batch, n_out) one-pass and two-pass N-point transforms
    (1024.0, 4096, 8.0, 10.0, 400.0, 12, 3, 0),
    (4096.0, 32768, 16.0, 40.0, 500.0, 8, 2, 0),        # N beyond one workgroup: two passes
    (1024.0, 4096, 8.0, 10.0, 400.0, 12, 2, -1),        # odd N_out (chirp-z inverse rows)
    # N = r * 2^k: radix-r combination around power-of-two transforms
    (4096.0, 24576, 8.0, 20.0, 1000.0, 16, 2, 0),       # 6 s at 4096 Hz (the paper's segment), r = 3
    (4096.0, 40960, 8.0, 100.0, 2048.0, 8, 1, 0),       # 10 s, r = 5, band to Nyquist
    (4096.0, 196608, 32.0, 100.0, 200.0, 4, 1, 0),      # 48 s, r = 3 around two-pass 65536-point transforms
]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", CASES, ids=[f"N{c[1]}_R{c[5]}_nout{c[7]}" for c in CASES])
def test_dense_tiles_match_oracle(torch_dev, case, precision):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    fs, n, q, fmin, fmax, R, B, n_out = case
    if n_out < 0:
        n_out = qt.Plan(fs, n, q, fmin, fmax, R, host_only=True).info.max_len
    print("dense", case, precision, flush=True)
    gp = qt.Plan(fs, n, q, fmin, fmax, R, precision=precision, n_out=n_out)
    op = o.OraclePlan(fs=fs, n=n, q=q, f_min=fmin, f_max=fmax, rows=R, n_out=n_out)
    x = np.stack([synthetic.injected_segment(n, fs, synthetic.rng_for(14, i))[0] for i in range(B)])
    dt = torch.float64 if precision == "fp64" else torch.float32
    xd = torch.from_numpy(x).to(dtype=dt, device="cuda")
    xh = xd.double().cpu().numpy()
    D = gp.dense(gp.forward(xd)).cpu().numpy()
    assert D.shape == (B, R, n)
    T = np.stack([op.dense(xh[b]) for b in range(B)])
    e1 = rel_rows(D, T).max()
    # from the oracle's envelopes, cast to the device precision
    Yo = op.forward(xh)
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    D2 = gp.dense(torch.from_numpy(Yo).to(dtype=cdt, device="cuda")).cpu().numpy()
    e2 = rel_rows(D2, T).max()
    print(f"  dense rel-L2: from the device forward {e1:.3e}, from the oracle's envelopes {e2:.3e}", flush=True)
    assert e1 <= TOL[precision] and e2 <= TOL[precision]


def test_dense_empty(torch_dev):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    gp = qt.Plan(1024.0, 4096, 8.0, 10.0, 400.0, 12)
    y = torch.zeros((0, 12, gp.N_out), dtype=torch.complex64, device="cuda")
    assert gp.dense(y).shape == (0, 12, 4096)
    g3 = qt.Plan(4096.0, 24576, 8.0, 20.0, 1000.0, 16)          # N = 3 * 8192
    assert g3.dense(torch.zeros((0, 16, g3.N_out), dtype=torch.complex64, device="cuda")).shape == (0, 16, 24576)
