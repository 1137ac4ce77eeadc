"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle,
element by element on the same seeded inputs.

Bars (rel-L2 per segment): FP32 <= 1e-5, FP64 <= 1e-12, on coefficients and on
reconstruction, for plans without frame holes.
"""
import math

import numpy as np
import pytest

import synthetic
from oracle import oracle as o

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-12}


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def rel_rows(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def plans(fs, n, q, f_min, f_max, rows, precision, **kw):
    import paper_2603_29785_amd as qt
    gp = qt.Plan(fs, n, q, f_min, f_max, rows, precision=precision, **kw)
    ckw = dict(cap_mode=o.CAP_COVER)
    if "cap_mode" in kw:
        ckw["cap_mode"] = {"cover": 0, "paper": 1, "none": 2, "manual": 3}[kw["cap_mode"]]
    for k in ("n_out", "p_floor_rel", "max_window"):
        if k in kw:
            ckw[k] = kw[k]
    op = o.OraclePlan(fs=fs, n=n, q=q, f_min=f_min, f_max=f_max, rows=rows, **ckw)
    assert gp.N_out == op.N_out and gp.R == op.R
    return gp, op


def to_dev(torch, a, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dt, device="cuda")


def host_input(x, precision):
    return x.astype(np.float32).astype(np.float64) if precision == "fp32" else x.astype(np.float64)


CASES = [
    # (fs, N, Q, f_min, f_max, R, batch) spanning single-pass and four-step
    # spectra, small to large N_out, ragged batches
    (4096.0, 16384, 8.0, 20.0, 1000.0, 64, 3),      # the one-segment workload plan (N_out 512)
    (1024.0, 1024, 4.0, 8.0, 400.0, 12, 5),         # tiny: N/2 = 512, N_out 64
    (256.0, 256, 2.0, 4.0, 128.0, 7, 9),            # band reaches Nyquist
    (4096.0, 32768, 8.0, 20.0, 2000.0, 128, 2),     # differentiable-workload plan, four-step spectrum
    (2048.0, 65536, 16.0, 10.0, 1024.0, 40, 2),     # N_out 8192 / 4096
    (4096.0, 131072, 4.0, 10.0, 2048.0, 256, 1),    # batched-workload plan, N_out 4096
    # N/2 = r * 2^k: decimation by 3 or 5 around power-of-two transforms
    (4096.0, 24576, 8.0, 20.0, 2000.0, 62, 3),      # 6 s at 4096 Hz (the paper's segment length), r = 3
    (4096.0, 40960, 8.0, 16.0, 2048.0, 100, 2),     # 10 s, r = 5, band to Nyquist
    (4096.0, 196608, 12.0, 10.0, 1500.0, 128, 1),   # 48 s, r = 3 around a four-step 32768-point transform
    (96.0, 96, 2.0, 4.0, 48.0, 5, 4),               # tiny: N/2 = 48 = 3 * 16, band to Nyquist
    (160.0, 160, 2.0, 4.0, 80.0, 8, 3),             # tiny: N/2 = 80 = 5 * 16
]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", CASES, ids=[f"N{c[1]}_R{c[5]}_Q{int(c[2])}" for c in CASES])
def test_forward_inverse_parity(torch_dev, case, precision):
    torch = torch_dev
    fs, n, q, fmin, fmax, R, B = case
    gp, op = plans(fs, n, q, fmin, fmax, R, precision)
    print(f"case N={n} R={R} Q={q} N_out={gp.N_out} B={B} {precision}", flush=True)
    x = np.stack([synthetic.injected_segment(n, fs, synthetic.rng_for(9, i))[0] for i in range(B)])
    xh = host_input(x, precision)
    Y_ref = op.forward(xh)
    Y = gp.forward(to_dev(torch, xh, precision)).cpu().numpy()
    assert Y.shape == Y_ref.shape
    err = rel_rows(Y, Y_ref)
    print("forward rel-L2", err.max(), flush=True)
    assert err.max() <= TOL[precision]
    # inverse of the oracle's coefficients (cast to the device precision)
    Yc = Y_ref.astype(np.complex64).astype(np.complex128) if precision == "fp32" else Y_ref
    x_ref = op.inverse(Yc)
    ydev = torch.from_numpy(Yc).to(torch.complex64 if precision == "fp32" else torch.complex128).cuda()
    xr = gp.inverse(ydev).cpu().numpy()
    err = rel_rows(xr, x_ref)
    print("inverse rel-L2", err.max(), flush=True)
    assert err.max() <= TOL[precision]
    # round trip through the GPU vs the projection x_M
    xm = op.project(xh)
    rt = gp.inverse(gp.forward(to_dev(torch, xh, precision))).cpu().numpy()
    err = rel_rows(rt, xm)
    print("round-trip rel-L2", err.max(), flush=True)
    assert err.max() <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_single_segment_workload(torch_dev, precision):
    """4 s of white noise + sine-Gaussian, Q = 8, 64 rows 20-1000 Hz."""
    torch = torch_dev
    gp, op = plans(4096.0, 16384, 8.0, 20.0, 1000.0, 64, precision)
    x = host_input(synthetic.single_segment(), precision)
    Y = gp.forward(to_dev(torch, x, precision)).cpu().numpy()
    assert rel(Y, op.forward(x)) <= TOL[precision]
    # a sine-Gaussian at 100 Hz peaks in the row containing 100 Hz
    k = int(np.argmax(np.abs(Y).max(axis=1)))
    f = gp.freqs
    assert f[max(k - 2, 0)] <= 100.0 <= f[min(k + 2, len(f) - 1)]
    xr = gp.inverse(torch.from_numpy(Y).cuda()).cpu().numpy()
    assert rel(xr, op.project(x)) <= TOL[precision]


def test_paper_cap_plan_parity(torch_dev):
    """The literal App. A cap (frame holes masked out)."""
    torch = torch_dev
    gp, op = plans(4096.0, 16384, 8.0, 20.0, 1000.0, 64, "fp64", cap_mode="paper")
    x = np.random.default_rng(4).standard_normal((2, 16384))
    Y = gp.forward(to_dev(torch, x, "fp64")).cpu().numpy()
    assert rel(Y, op.forward(x)) <= 1e-12
    xr = gp.inverse(torch.from_numpy(Y).cuda()).cpu().numpy()
    assert rel(xr, op.inverse(op.forward(x))) <= 1e-10


def test_paper_minimal_output_size_parity(torch_dev):
    """The paper's smallest envelope, N_out = ceil(T max_gap) + 1 under the
    literal cap (App. A), on its 6 s x 4096 Hz segments with 62 rows: an odd
    length, so chirp-z rows around a radix-3 spectrum."""
    torch = torch_dev
    import math
    fs, n, R, fmin, fmax = 4096.0, 24576, 62, 20.0, 2000.0
    f = fmin * (fmax / fmin) ** (np.arange(R) / (R - 1))
    n_out = math.ceil(n / fs * np.max(np.diff(f))) + 1
    gp, op = plans(fs, n, 8.0, fmin, fmax, R, "fp64", cap_mode="paper", n_out=n_out)
    assert gp.N_out == n_out and n_out & (n_out - 1)
    x = np.random.default_rng(6).standard_normal((2, n))
    Y = gp.forward(to_dev(torch, x, "fp64")).cpu().numpy()
    assert Y.shape == (2, R, n_out)
    assert rel(Y, op.forward(x)) <= 1e-12
    xr = gp.inverse(torch.from_numpy(Y).cuda()).cpu().numpy()
    assert rel(xr, op.inverse(op.forward(x))) <= 1e-10


# Chirp-z rows beyond one workgroup on the long-segment plan (2^21 samples at
# 8192 Hz, Q = 12, 512 rows from 5 to 4096 Hz): the paper's minimal
# N_out = ceil(T max_gap) + 1 = 13677 under the literal cap (convolution
# length 32768), and under the default cap N_out = 27440, the first length
# >= the longest window (27353) with no prime factor above 7 (convolution
# length 65536). The oracle's transforms of 512 rows of these lengths take
# minutes, so sampled rows are compared with the oracle (forward_rows: the
# same arithmetic row by row), and the reconstruction with the oracle's
# projection x_M. Both precisions take the same (FP32-cast) input. The frame
# has condition number kappa ~ 8e4 (default cap) and ~ 1e6 (literal cap) on
# its mask: the reconstruction bars are the plain bars scaled by
# sqrt(kappa / 1e4) (the dual frame amplifies rounding by up to sqrt(kappa);
# the plain bars are stated for kappa <= 1e4).
LONG_CHIRP = [("paper", 13677), ("cover", 27440)]
_long_chirp_oracle = {}


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("cap,n_out", LONG_CHIRP, ids=[c[0] for c in LONG_CHIRP])
def test_long_chirp_rows_parity(torch_dev, cap, n_out, precision):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    fs, n, q, fmin, fmax, R = 8192.0, 1 << 21, 12.0, 5.0, 4096.0, 512
    gp, op = plans(fs, n, q, fmin, fmax, R, precision, cap_mode=cap, n_out=n_out)
    assert n_out >= gp.info.max_len and n_out & (n_out - 1)
    info = gp.info
    kappa = info.frame_B / info.frame_A
    scale = max(1.0, math.sqrt(kappa / 1e4))
    rows = sorted({0, 1, R // 4, R // 2, int(np.argmax(gp.half_width)), R - 2, R - 1})
    print(f"long chirp-z rows: cap {cap} N_out={n_out} {precision} kappa={kappa:.3g} rows {rows}", flush=True)
    x = host_input(synthetic.batched_segments(1, n, fs, workload=4, first=0, dtype=np.float64), "fp32")
    if cap not in _long_chirp_oracle:
        print("  oracle: sampled rows and x_M", flush=True)
        _long_chirp_oracle[cap] = (op.forward_rows(x, rows), op.project(x))
    Yo, xm = _long_chirp_oracle[cap]
    Y = gp.forward(to_dev(torch, x, precision))
    e_y = rel(Y[:, rows].cpu().numpy(), Yo)
    e_rt = rel(gp.inverse(Y).cpu().numpy(), xm)
    print(f"  sampled rows coef {e_y:.3e}, round trip {e_rt:.3e} (bar x{scale:.3g})", flush=True)
    assert e_y <= TOL[precision] and e_rt <= TOL[precision] * scale
    # both adjoints through the same rows: dot-product identities
    g = torch.Generator(device="cuda").manual_seed(3)
    gy = torch.randn(Y.shape, device="cuda", dtype=Y.dtype, generator=g)
    lhs = float(torch.sum((Y.conj() * gy).real.double()))
    rhs = float(torch.sum(to_dev(torch, x, precision).double() * gp.forward_adjoint(gy).double()))
    z = torch.randn((1, n), device="cuda", dtype=torch.float64 if precision == "fp64" else torch.float32,
                    generator=g)
    lhs2 = float(torch.sum(gp.inverse(gy).double() * z.double()))
    rhs2 = float(torch.sum((gy.conj() * gp.inverse_adjoint(z)).real.double()))
    # relative to the Cauchy-Schwarz bound of each inner product
    s1 = float(torch.linalg.norm(Y.to(torch.complex128)) * torch.linalg.norm(gy.to(torch.complex128)))
    s2 = float(torch.linalg.norm(gp.inverse(gy).double()) * torch.linalg.norm(z.double()))
    print(f"  adjoint identities: {abs(lhs - rhs) / s1:.3e}, {abs(lhs2 - rhs2) / s2:.3e}", flush=True)
    assert abs(lhs - rhs) <= TOL[precision] * s1 and abs(lhs2 - rhs2) <= TOL[precision] * s2


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batched_workload_sampled(torch_dev, precision):
    """256 segments x 131072 samples at the benchmark's launch configuration;
    sampled segments against the oracle, every segment against invariants."""
    torch = torch_dev
    B = 256 if precision == "fp32" else 32
    gp, op = plans(4096.0, 131072, 8.0, 10.0, 2048.0, 256, precision)
    x = synthetic.batched_segments(B, dtype=np.float64)
    xh = host_input(x, precision)
    xd = to_dev(torch, xh, precision)
    Y = gp.forward(xd)
    xr = gp.inverse(Y)
    for i in (0, B // 2 + 3, B - 1):
        Yr = op.forward(xh[i])
        assert rel(Y[i].cpu().numpy(), Yr) <= TOL[precision], i
        assert rel(xr[i].cpu().numpy(), op.project(xh[i])) <= TOL[precision], i
    # every segment: round trip leaves only the out-of-mask part; the
    # energy of each row equals the energy of its dense tile (Parseval)
    Xd = torch.fft.rfft(xd.double(), dim=-1)
    Mk = torch.from_numpy(gp.mask).cuda()
    xm = torch.fft.irfft(Xd * Mk, n=131072, dim=-1)
    e = torch.linalg.norm(xr.double() - xm, dim=-1) / torch.linalg.norm(xm, dim=-1)
    assert float(e.max()) <= TOL[precision]


def test_batched_sweep_sampled(torch_dev):
    """The benchmark's step at full size: the Q set {4, 8, 16} as one forward
    sweep over 256 x 131072 samples, then each plan's inverse; sampled
    segments of every plan against the oracle, every segment's round trip
    against the projection onto the plan's mask."""
    torch = torch_dev
    import paper_2603_29785_amd as qt
    B, n = 256, 131072
    specs = [plans(4096.0, n, q, 10.0, 2048.0, 256, "fp32") for q in (4.0, 8.0, 16.0)]
    gps = [g for g, _ in specs]
    x = synthetic.batched_segments(B, dtype=np.float64)
    xh = host_input(x, "fp32")
    xd = to_dev(torch, xh, "fp32")
    ys = qt.forward_sweep(gps, xd)
    Xd = torch.fft.rfft(xd.double(), dim=-1)
    for (gp, op), Y in zip(specs, ys):
        print("sweep plan Q", gp.params["q"], flush=True)
        for i in (1, B // 3, B - 2):
            assert rel(Y[i].cpu().numpy(), op.forward(xh[i])) <= TOL["fp32"], i
        xr = gp.inverse(Y)
        xm = torch.fft.irfft(Xd * torch.from_numpy(gp.mask).cuda(), n=n, dim=-1)
        e = torch.linalg.norm(xr.double() - xm, dim=-1) / torch.linalg.norm(xm, dim=-1)
        assert float(e.max()) <= TOL["fp32"]
        del xr, xm


def test_linearity_and_determinism(torch_dev):
    torch = torch_dev
    gp, _ = plans(4096.0, 32768, 8.0, 20.0, 2000.0, 128, "fp32")
    g = torch.Generator(device="cuda").manual_seed(0)
    x1 = torch.randn(4, 32768, device="cuda", generator=g)
    x2 = torch.randn(4, 32768, device="cuda", generator=g)
    a, b = 0.75, -1.25
    lhs = gp.forward(a * x1 + b * x2)
    rhs = a * gp.forward(x1) + b * gp.forward(x2)
    assert float(torch.linalg.norm(lhs - rhs) / torch.linalg.norm(rhs)) < 1e-5
    y1 = gp.forward(x1)
    y2 = gp.forward(x1)
    assert torch.equal(y1, y2)
    # a segment alone and inside a batch gives the same bits
    alone = gp.forward(x1[2:3].contiguous())
    assert torch.equal(alone[0], y1[2])
    inv_all = gp.inverse(y1)
    inv_one = gp.inverse(y1[1:2].contiguous())
    assert torch.equal(inv_one[0], inv_all[1])


def test_chunked_workspace_matches(torch_dev):
    torch = torch_dev
    gp, _ = plans(4096.0, 65536, 8.0, 10.0, 2048.0, 96, "fp32")
    x = torch.randn(7, 65536, device="cuda")
    full = gp.forward(x)
    one = gp.workspace_bytes(1)
    ws = torch.empty(one * 2 + 10, dtype=torch.uint8, device="cuda")   # two segments per chunk
    part = gp.forward(x, ws=ws)
    assert torch.equal(full, part)
    xi_full = gp.inverse(full)
    xi_part = gp.inverse(full, ws=ws)
    assert torch.equal(xi_full, xi_part)


def test_errors_and_empty(torch_dev):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    gp, _ = plans(1024.0, 4096, 8.0, 10.0, 400.0, 16, "fp32")
    x = torch.zeros(0, 4096, device="cuda")
    y = gp.forward(x)
    assert y.shape == (0, 16, gp.N_out)
    tiny = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(qt.QtamError) as e:
        gp.forward(torch.zeros(2, 4096, device="cuda"), ws=tiny)
    assert e.value.status == 3
    # N/2 with an odd factor other than 3 or 5 is not on the GPU path
    bad = qt.Plan(4096.0, 14336, 8.0, 20.0, 1000.0, 62)
    with pytest.raises(qt.QtamError) as e:
        bad.forward(torch.zeros(1, 14336, device="cuda"))
    assert e.value.status == 2


# Envelope lengths that are not powers of two (chirp-z rows): the smallest
# valid N_out (the longest window), as the paper's minimal output size.
ODD_NOUT = [
    # (fs, N, Q, f_min, f_max, R, batch, precision)
    (4096.0, 24576, 8.0, 20.0, 2000.0, 62, 2, "fp32"),
    (4096.0, 24576, 8.0, 20.0, 2000.0, 62, 2, "fp64"),
    (4096.0, 16384, 8.0, 20.0, 1000.0, 64, 3, "fp32"),
    (1024.0, 1024, 4.0, 8.0, 400.0, 12, 5, "fp64"),
]


@pytest.mark.parametrize("case", ODD_NOUT, ids=[f"N{c[1]}_R{c[5]}_{c[7]}" for c in ODD_NOUT])
def test_odd_envelope_length_parity(torch_dev, case):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    fs, n, q, fmin, fmax, R, B, precision = case
    n_out = qt.Plan(fs, n, q, fmin, fmax, R, host_only=True).info.max_len
    assert n_out & (n_out - 1)
    gp, op = plans(fs, n, q, fmin, fmax, R, precision, n_out=n_out)
    print(f"odd N_out: N={n} R={R} N_out={n_out} {precision}", flush=True)
    x = np.stack([synthetic.injected_segment(n, fs, synthetic.rng_for(12, i))[0] for i in range(B)])
    xh = host_input(x, precision)
    Y_ref = op.forward(xh)
    Y = gp.forward(to_dev(torch, xh, precision)).cpu().numpy()
    assert rel_rows(Y, Y_ref).max() <= TOL[precision]
    Yc = Y_ref.astype(np.complex64).astype(np.complex128) if precision == "fp32" else Y_ref
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    xr = gp.inverse(torch.from_numpy(np.ascontiguousarray(Yc)).to(dtype=dt, device="cuda")).cpu().numpy()
    assert rel_rows(xr, op.inverse(Yc)).max() <= TOL[precision]
    # round trip returns the projection onto the covered bins
    xr2 = gp.inverse(gp.forward(to_dev(torch, xh, precision))).cpu().numpy()
    assert rel_rows(xr2, op.project(xh)).max() <= TOL[precision]


LONG_ROWS = [
    # rows longer than one workgroup's LDS transform: four-step rows
    ("fp32", 16384.0, 1 << 20, 8.0, 10.0, 2048.0, 64, 2),      # 64 s at 16384 Hz, 64 rows: N_out 32768
    ("fp64", 4096.0, 1 << 18, 4.0, 10.0, 2048.0, 64, 1),       # FP64 N_out 16384
    ("fp32", 8192.0, 1 << 21, 12.0, 5.0, 4096.0, 512, 1),      # long-segment precision workload plan
    ("fp64", 8192.0, 1 << 21, 12.0, 5.0, 4096.0, 512, 1),
]


@pytest.mark.parametrize("case", LONG_ROWS, ids=[f"{c[0]}_N{c[2]}_R{c[6]}" for c in LONG_ROWS])
def test_long_rows_parity(torch_dev, case):
    torch = torch_dev
    precision, fs, n, q, fmin, fmax, R, B = case
    gp, op = plans(fs, n, q, fmin, fmax, R, precision)
    print(f"long rows: N={n} R={R} N_out={gp.N_out} {precision}", flush=True)
    x = np.stack([synthetic.injected_segment(n, fs, synthetic.rng_for(12, i))[0] for i in range(B)])
    xh = host_input(x, precision)
    Y = gp.forward(to_dev(torch, xh, precision))
    xr = gp.inverse(Y).cpu().numpy()
    Y = Y.cpu().numpy()
    xm = op.project(xh)
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    for b in range(B):
        Yr = op.forward(xh[b])
        e_y, e_rt = rel(Y[b], Yr), rel(xr[b], xm[b])
        # the inverse alone: both sides invert the same (cast) coefficients
        Yc = Yr.astype(np.complex64).astype(np.complex128) if precision == "fp32" else Yr
        xi = gp.inverse(torch.from_numpy(Yc[None]).to(dtype=cdt, device="cuda")).cpu().numpy()[0]
        e_inv = rel(xi, op.inverse(Yc))
        print(f"  segment {b}: coef {e_y:.3e}, inverse {e_inv:.3e}, round trip {e_rt:.3e}", flush=True)
        assert e_y <= TOL[precision] and e_inv <= TOL[precision] and e_rt <= TOL[precision], b


@pytest.mark.parametrize("window,param", [("hann", 0.0), ("kaiser", 6.0), ("tukey", 0.5), ("planck", 0.3)])
def test_window_family_parity(torch_dev, window, param):
    """Non-bisquare windows (App. A) take the table-weight path."""
    torch = torch_dev
    import paper_2603_29785_amd as qt
    wi = {"hann": o.WIN_HANN, "kaiser": o.WIN_KAISER, "tukey": o.WIN_TUKEY, "planck": o.WIN_PLANCK}[window]
    for precision in ("fp32", "fp64"):
        gp = qt.Plan(4096.0, 32768, 8.0, 20.0, 2000.0, 96, window=window, window_param=param, precision=precision)
        op = o.OraclePlan(fs=4096.0, n=32768, q=8.0, f_min=20.0, f_max=2000.0, rows=96, window=wi, window_param=param)
        x = host_input(synthetic.batched_segments(2, 32768, 4096.0, workload=13, dtype=np.float64), precision)
        Y = gp.forward(to_dev(torch, x, precision))
        Yo = op.forward(x)
        e_y = rel_rows(Y.cpu().numpy(), Yo).max()
        e_rt = rel_rows(gp.inverse(Y).cpu().numpy(), op.project(x)).max()
        Yc = Yo.astype(np.complex64).astype(np.complex128) if precision == "fp32" else Yo
        cdt = torch.complex128 if precision == "fp64" else torch.complex64
        e_inv = rel_rows(gp.inverse(torch.from_numpy(Yc).to(dtype=cdt, device="cuda")).cpu().numpy(),
                         op.inverse(Yc)).max()
        print(f"  {window} {precision}: coef {e_y:.3e}, inverse {e_inv:.3e}, round trip {e_rt:.3e}", flush=True)
        assert e_y <= TOL[precision] and e_inv <= TOL[precision] and e_rt <= TOL[precision]


def test_masked_coefficients_inverse(torch_dev):
    """Inverting a masked coefficient set (keep only the strongest rows) is the
    canonical-dual synthesis of the masked set, as in the oracle."""
    torch = torch_dev
    gp, op = plans(4096.0, 16384, 8.0, 20.0, 1000.0, 64, "fp64")
    x = synthetic.single_segment()
    Y = op.forward(x)
    keep = np.zeros_like(Y)
    top = np.argsort(np.abs(Y).max(axis=1))[-8:]
    keep[top] = Y[top]
    keep[:, 100:200] = 0
    xr = gp.inverse(torch.from_numpy(keep).cuda()).cpu().numpy()
    assert rel(xr, op.inverse(keep)) <= 1e-12


def smooth_at_least(m):
    """The first length >= m, not a power of two, with no prime factor above 7."""
    v = max(m, 3)
    while True:
        r = v
        for p_ in (2, 3, 5, 7):
            while r % p_ == 0:
                r //= p_
        if r == 1 and v & (v - 1):
            return v
        v += 1


def random_plans(seed, count, log2n=(7, 16), log2n_odd=(5, 13), row_range=(3, 97), q_range=(2.0, 24.0),
                 odd_range=(4, 4096), kinds=(0, 1, 2), smooth=False):
    """Seeded random plans over the supported shapes: N = r 2^k (r = 1, 3, 5),
    bands from near DC to Nyquist, every window family, automatic, odd
    (chirp-z) and oversized power-of-two N_out; only frames with condition
    number <= 1e3, where the bars apply. Odd N_out within odd_range: the
    longest window's length, or with smooth the first length from there with
    no prime factor above 7 (the oracle's transforms of lengths with large
    prime factors are direct sums, too slow at these sizes)."""
    import paper_2603_29785_amd as qt
    rng = np.random.default_rng(seed)
    wins = [("bisquare", o.WIN_BISQUARE, 0.0), ("hann", o.WIN_HANN, 0.0), ("kaiser", o.WIN_KAISER, 5.0),
            ("tukey", o.WIN_TUKEY, 0.4), ("planck", o.WIN_PLANCK, 0.25)]
    out = []
    while len(out) < count:
        r = int(rng.choice([1, 3, 5]))
        n = r * 2 ** int(rng.integers(*(log2n if r == 1 else log2n_odd)))
        fs = float(rng.choice([256.0, 1024.0, 4096.0]))
        nyq = fs / 2
        fmin = float(rng.uniform(0.005, 0.2)) * nyq
        fmax = float(rng.choice([nyq, rng.uniform(0.4, 0.95) * nyq]))
        if fmin < 2 * fs / n:          # at least two bins above DC
            continue
        rows = int(rng.integers(*row_range))
        q = float(rng.uniform(*q_range))
        wname, wid, wparam = wins[int(rng.integers(len(wins)))]
        host = qt.Plan(fs, n, q, fmin, fmax, rows, window=wname, window_param=wparam, host_only=True)
        kind = int(rng.integers(3))
        if kind not in kinds:
            continue
        n_out = 0 if kind == 0 else (host.info.max_len if kind == 1 else 2 * host.N_out)
        if kind == 1 and smooth:
            n_out = smooth_at_least(n_out)
        if n_out and (n_out > 32768 or n_out < 4 or (kind == 1 and not odd_range[0] <= n_out <= odd_range[1])):
            continue
        info = host.info
        if not (info.frame_A > 0 and info.frame_B / info.frame_A <= 1e3):
            continue
        out.append((fs, n, q, fmin, fmax, rows, wname, wid, wparam, n_out))
    return out


RANDOM = (random_plans(2026, 16) + random_plans(2027, 8, log2n=(15, 19), log2n_odd=(13, 16), row_range=(16, 257),
                                                  q_range=(2.0, 8.0))
          # odd N_out above 4096: chirp-z rows beyond one workgroup in FP64 (and above 8192 in FP32)
          + random_plans(2028, 4, log2n=(15, 19), log2n_odd=(13, 17), row_range=(8, 65), q_range=(2.0, 6.0),
                         odd_range=(4097, 32768), kinds=(1,), smooth=True))


# FP32 error budget of the forward coefficients. Three sources: the
# spectrum's rounding, which is relative to the whole signal; the row
# transforms' rounding, relative to each row; the weights' rounding to FP32.
# With u = 2^-24, Pbar the mean frame value P over bins 0..N/2 and P_X the
# mean of P weighted by the signal's energy |X|^2 (so Pbar / P_X grows when
# the signal's energy sits where the rows cover little, e.g. coloured noise
# below the band),
#   rel-L2(Y) ~ u sqrt(0.36 log2(N) Pbar / P_X + 0.33 log2(N_out) + 0.18),
# constants fitted from each source alone (FP32 spectrum, weights or row
# transforms against FP64) on white noise. The FP32 bar 1e-5 holds while
# Pbar / P_X stays below about 1500.
def fp32_coef_budget(op, x):
    P, _ = op.frame()
    E = np.abs(np.fft.rfft(x)) ** 2
    ratio = P.mean() / (np.sum(E * P) / np.sum(E))
    u = 2.0 ** -24
    return u * math.sqrt(0.36 * math.log2(op.n) * ratio + 0.33 * math.log2(op.N_out) + 0.18), ratio


BUDGET_PLANS = [
    # (what, fs, N, Q, f_min, f_max, R, window, window id, parameter, N_out)
    ("batched plan Q 8", 4096.0, 131072, 8.0, 10.0, 2048.0, 256, "bisquare", o.WIN_BISQUARE, 0.0, 0),
    ("256 Hz Kaiser from 4.6 Hz", 256.0, 262144, 5.8947755089717955, 4.5749963722033815, 128.0, 60, "kaiser",
     o.WIN_KAISER, 5.0, 32768),
    ("256 Hz Kaiser from 10 Hz", 256.0, 262144, 5.8947755089717955, 10.0, 128.0, 60, "kaiser",
     o.WIN_KAISER, 5.0, 32768),
    # random plans found nearest the FP32 bar (about 5e-6) in a sweep: bands
    # from 15-22 Hz at 256 Hz, Pbar / P_X about 1000-1500, the budget's edge
    ("256 Hz Kaiser Q 2 from 21 Hz, odd N_out", 256.0, 81920, 2.009339606116827, 21.419685991304572, 128.0, 12,
     "kaiser", o.WIN_KAISER, 5.0, 12348),
    ("256 Hz Kaiser Q 6.6 from 21.5 Hz", 256.0, 65536, 6.64808106438729, 21.528150558862084, 128.0, 35, "kaiser",
     o.WIN_KAISER, 5.0, 0),
    ("256 Hz Kaiser Q 5 from 15 Hz", 256.0, 98304, 5.046765315259778, 15.241534846108705, 128.0, 19, "kaiser",
     o.WIN_KAISER, 5.0, 0),
]


@pytest.mark.parametrize("spec", BUDGET_PLANS, ids=[b[0].replace(" ", "_") for b in BUDGET_PLANS])
def test_fp32_coefficient_error_budget(torch_dev, spec):
    """FP32 coefficients on coloured noise with injections: within the bar and
    within twice the budget above, on plans whose coloured noise below the
    band raises Pbar / P_X from about 4 to about 1500."""
    torch = torch_dev
    import paper_2603_29785_amd as qt
    what, fs, n, q, fmin, fmax, rows, wname, wid, wparam, n_out = spec
    gp = qt.Plan(fs, n, q, fmin, fmax, rows, window=wname, window_param=wparam, n_out=n_out)
    op = o.OraclePlan(fs=fs, n=n, q=q, f_min=fmin, f_max=fmax, rows=rows, window=wid, window_param=wparam,
                      n_out=n_out)
    x = host_input(np.stack([synthetic.injected_segment(n, fs, synthetic.rng_for(21, i))[0] for i in range(2)]),
                   "fp32")
    e = rel_rows(gp.forward(to_dev(torch, x, "fp32")).cpu().numpy(), op.forward(x))
    for b in range(2):
        budget, ratio = fp32_coef_budget(op, x[b])
        print(f"{what}: segment {b} Pbar/P_X {ratio:.3g} coef rel-L2 {e[b]:.3e} budget {budget:.3e}", flush=True)
        assert e[b] <= TOL["fp32"] and e[b] <= 2 * budget


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("spec", RANDOM, ids=[f"N{s[1]}_R{s[5]}_{s[6]}_nout{s[9]}" for s in RANDOM])
def test_random_plans_parity(torch_dev, spec, precision):
    torch = torch_dev
    import paper_2603_29785_amd as qt
    fs, n, q, fmin, fmax, rows, wname, wid, wparam, n_out = spec
    print("random plan", spec, precision, flush=True)
    gp = qt.Plan(fs, n, q, fmin, fmax, rows, window=wname, window_param=wparam, precision=precision, n_out=n_out)
    op = o.OraclePlan(fs=fs, n=n, q=q, f_min=fmin, f_max=fmax, rows=rows, window=wid, window_param=wparam,
                      n_out=n_out)
    assert gp.N_out == op.N_out and gp.R == op.R
    B = 3
    x = host_input(np.stack([synthetic.injected_segment(n, fs, synthetic.rng_for(21, i))[0] for i in range(B)]),
                   precision)
    Y_ref = op.forward(x)
    Y = gp.forward(to_dev(torch, x, precision)).cpu().numpy()
    e_y = rel_rows(Y, Y_ref).max()
    Yc = Y_ref.astype(np.complex64).astype(np.complex128) if precision == "fp32" else Y_ref
    cdt = torch.complex64 if precision == "fp32" else torch.complex128
    xr = gp.inverse(torch.from_numpy(Yc).to(cdt).cuda()).cpu().numpy()
    e_x = rel_rows(xr, op.inverse(Yc)).max()
    print(f"  coef {e_y:.3e}, inverse {e_x:.3e}", flush=True)
    assert e_y <= TOL[precision] and e_x <= TOL[precision]


def random_mode_plans(seed, count):
    """Seeded random plans over the cap modes (cover, paper, none, manual),
    the normalisations, explicit frequency lists with a duplicated centre and
    mask floors; frames with kappa up to 1e8."""
    import paper_2603_29785_amd as qt
    rng = np.random.default_rng(seed)
    caps = [("cover", o.CAP_COVER), ("paper", o.CAP_PAPER), ("none", o.CAP_NONE), ("manual", o.CAP_MANUAL)]
    norms = [("unit_energy", o.NORM_UNIT_ENERGY), ("paper_inv_energy", o.NORM_PAPER_INV_ENERGY),
             ("none", o.NORM_NONE)]
    wins = [("bisquare", o.WIN_BISQUARE, 0.0), ("hann", o.WIN_HANN, 0.0), ("kaiser", o.WIN_KAISER, 5.0),
            ("tukey", o.WIN_TUKEY, 0.4), ("planck", o.WIN_PLANCK, 0.25)]
    out = []
    while len(out) < count:
        r = int(rng.choice([1, 3, 5]))
        n = r * 2 ** int(rng.integers(10, 17 if r == 1 else 14))
        fs = float(rng.choice([256.0, 1024.0, 4096.0]))
        nyq = fs / 2
        fmin = float(rng.uniform(0.01, 0.2)) * nyq
        fmax = float(rng.choice([nyq, rng.uniform(0.4, 0.95) * nyq]))
        if fmin < 2 * fs / n:
            continue
        rows = int(rng.integers(4, 80))
        q = float(rng.uniform(2.0, 24.0))
        cap = caps[int(rng.integers(4))]
        norm = norms[int(rng.integers(3))]
        win = wins[int(rng.integers(5))]
        freqs = None
        if rng.random() < 0.25:
            freqs = np.sort(rng.uniform(fmin, fmax, rows))
            freqs[rows // 2] = freqs[rows // 2 - 1]
        max_window = int(rng.integers(3, 400)) if cap[0] == "manual" else 0
        floor = float(rng.choice([1e-6, 1e-3, 0.0]))
        kw = dict(window=win[0], window_param=win[2], cap_mode=cap[0], max_window=max_window, norm_mode=norm[0],
                  p_floor_rel=floor, freqs=freqs)
        try:
            host = qt.Plan(fs, n, q, fmin, fmax, rows, host_only=True, **kw)
        except qt.QtamError:
            continue
        if not (host.info.frame_A > 0) or host.info.frame_B / host.info.frame_A > 1e8:
            continue
        okw = dict(window=win[1], window_param=win[2], cap_mode=cap[1], max_window=max_window, norm_mode=norm[1],
                   p_floor_rel=floor, freqs=freqs)
        out.append((fs, n, q, fmin, fmax, rows, kw, okw, host.info.frame_B / host.info.frame_A))
    return out


MODES = random_mode_plans(9101, 8)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("spec", MODES, ids=[f"N{s[1]}_R{s[5]}_{s[6]['cap_mode']}_{s[6]['norm_mode']}" for s in MODES])
def test_random_mode_plans_parity(torch_dev, spec, precision):
    """Cap modes, normalisations, explicit grids and mask floors on seeded
    random plans: coefficients at the bars, the inverse at the bars scaled by
    sqrt(kappa / 1e4) above kappa = 1e4 (reading 22)."""
    torch = torch_dev
    import paper_2603_29785_amd as qt
    fs, n, q, fmin, fmax, rows, kw, okw, kappa = spec
    gp = qt.Plan(fs, n, q, fmin, fmax, rows, precision=precision, **kw)
    op = o.OraclePlan(fs=fs, n=n, q=q, f_min=fmin, f_max=fmax, rows=rows, **okw)
    assert gp.N_out == op.N_out and gp.R == op.R
    x = host_input(np.stack([synthetic.injected_segment(n, fs, synthetic.rng_for(71, j))[0] for j in range(2)]),
                   precision)
    Yo = op.forward(x)
    e_y = rel_rows(gp.forward(to_dev(torch, x, precision)).cpu().numpy(), Yo).max()
    Yc = Yo.astype(np.complex64).astype(np.complex128) if precision == "fp32" else Yo
    cdt = torch.complex64 if precision == "fp32" else torch.complex128
    e_x = rel_rows(gp.inverse(torch.from_numpy(Yc).to(cdt).cuda()).cpu().numpy(), op.inverse(Yc)).max()
    scale = max(1.0, math.sqrt(kappa / 1e4))
    print(f"modes {kw['cap_mode']} {kw['norm_mode']} kappa {kappa:.2g} {precision}: coef {e_y:.2e} inverse {e_x:.2e}",
          flush=True)
    assert e_y <= TOL[precision] and e_x <= TOL[precision] * scale
