"""The forward transform that allocates nothing (qtam_forward_noalloc: the
library's static device workspace) against qtam_forward with a caller
workspace, through the C ABI: two calls in a row on the batched workload's
plan (the second with a smaller batch), then a call on another plan sharing
the same static workspace, each compared with the ordinary entry point."""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-12}


def rel_rows(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def test_noalloc_forward_matches_forward():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_29785_amd as qt
    # batched workload plan (N = 131072, 256 rows, Q = 8): one segment takes
    # about 3 MiB of workspace, so 40 segments run in several chunks
    cases = [((4096.0, 131072, 8.0, 10.0, 2048.0, 256, "fp32"), 40),
             ((4096.0, 131072, 8.0, 10.0, 2048.0, 256, "fp32"), 5),
             ((4096.0, 16384, 8.0, 20.0, 1000.0, 64, "fp64"), 3)]
    plans = {}
    for (fs, n, q, fmin, fmax, R, prec), B in cases:
        key = (fs, n, q, fmin, fmax, R, prec)
        if key not in plans:
            plans[key] = qt.Plan(fs, n, q, fmin, fmax, R, precision=prec)
        p = plans[key]
        assert p.workspace_bytes(1) <= qt.binding.NOALLOC_WORKSPACE_BYTES
        print(f"noalloc forward: N={n} R={R} {prec} batch {B}", flush=True)
        dt = torch.float64 if prec == "fp64" else torch.float32
        x = torch.from_numpy(synthetic.batched_segments(B, n, fs, workload=9, dtype=np.float64)).to(
            device="cuda", dtype=dt)
        y0 = p.forward(x)
        y1 = torch.full_like(y0, float("nan"))
        p.forward_noalloc(x, out=y1)
        torch.cuda.synchronize()
        a, b = y1.cpu().numpy(), y0.cpu().numpy()
        e = rel_rows(a, b).max()
        print(f"  max rel-L2 per segment {e:.3e}, identical bits: {np.array_equal(a, b)}", flush=True)
        assert np.all(np.isfinite(a)) and e <= TOL[prec]
