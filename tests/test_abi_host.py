"""Host-side checks of the C ABI (no GPU needed): every symbol include/qtam.h
declares is exported, host-only plans build the same tables as the oracle,
and invalid calls return status codes without touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import paper_2603_29785_amd as qt
from paper_2603_29785_amd import binding
from oracle import oracle as o

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtam.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qtam_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    names = declared_functions()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (qtam_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(binding.lib, n)
    assert set(binding.EXPORTED) <= set(names)


def test_status_strings_and_version():
    for s in range(6):
        assert qt.status_string(s)
    assert qt.version().startswith("qtam-gfx950")


def host_plan(**kw):
    return qt.Plan(host_only=True, **kw)


def compare_tables(gp, op):
    t = op.row_table()
    assert gp.N_out == op.N_out and gp.R == op.R
    assert gp.info.sum_len == op.sum_len and gp.info.max_len == op.max_len
    assert np.array_equal(gp.centre, t["centre"])
    assert np.array_equal(gp.half_width, t["half"])
    assert np.array_equal(gp.lo, t["lo"])
    assert np.array_equal(gp.hi, t["hi"])
    assert np.array_equal(gp.freqs, t["freq"])
    W = op.windows()
    assert np.abs(gp.windows_dense() - W).max() <= 1e-14 * np.abs(W).max()
    P, M = op.frame()
    assert np.abs(gp.frame - P).max() <= 1e-13 * P.max()
    assert np.array_equal(gp.mask, M)
    assert gp.info.l_max == op.l_max


WORKLOAD_PLANS = [
    dict(sample_rate=4096.0, n_samples=16384, q=8.0, f_min=20.0, f_max=1000.0, n_rows=64),
    dict(sample_rate=4096.0, n_samples=131072, q=4.0, f_min=10.0, f_max=2048.0, n_rows=256),
    dict(sample_rate=4096.0, n_samples=131072, q=16.0, f_min=10.0, f_max=2048.0, n_rows=256),
    dict(sample_rate=8192.0, n_samples=2097152, q=12.0, f_min=5.0, f_max=4096.0, n_rows=512),
    dict(sample_rate=4096.0, n_samples=32768, q=8.0, f_min=20.0, f_max=2000.0, n_rows=128),
]


@pytest.mark.parametrize("kw", WORKLOAD_PLANS)
def test_workload_plan_tables_match_oracle(kw):
    gp = host_plan(**kw)
    op = o.OraclePlan(fs=kw["sample_rate"], n=kw["n_samples"], q=kw["q"], f_min=kw["f_min"],
                      f_max=kw["f_max"], rows=kw["n_rows"])
    compare_tables(gp, op)


CAPS = {"cover": o.CAP_COVER, "paper": o.CAP_PAPER, "none": o.CAP_NONE}
WINS = {"bisquare": o.WIN_BISQUARE, "hann": o.WIN_HANN, "kaiser": o.WIN_KAISER, "tukey": o.WIN_TUKEY,
        "planck": o.WIN_PLANCK}


@settings(max_examples=60, deadline=None)
@given(log2n=st.integers(6, 14), rows=st.integers(1, 40), q=st.floats(0.5, 40.0),
       fmin_frac=st.floats(0.02, 0.4), span=st.floats(1.0, 50.0), cap=st.sampled_from(list(CAPS)),
       win=st.sampled_from(list(WINS)), param=st.floats(0.1, 0.9))
def test_random_plan_tables_match_oracle(log2n, rows, q, fmin_frac, span, cap, win, param):
    n = 2 ** log2n
    fs = float(n) / 2.0          # T = 2 s
    f_min = fmin_frac * fs / 2
    f_max = min(f_min * span, fs / 2)
    kw = dict(sample_rate=fs, n_samples=n, q=q, f_min=f_min, f_max=f_max, n_rows=rows, cap_mode=cap,
              window=win, window_param=param * (8.0 if win == "kaiser" else 1.0))
    try:
        op = o.OraclePlan(fs=fs, n=n, q=q, f_min=f_min, f_max=f_max, rows=rows, cap_mode=CAPS[cap],
                          window=WINS[win], window_param=kw["window_param"])
    except ValueError:
        with pytest.raises(qt.QtamError):
            host_plan(**kw)
        return
    compare_tables(host_plan(**kw), op)


def test_explicit_frequency_list_and_duplicates():
    freqs = np.array([10.0, 10.0, 13.5, 20.0, 20.1, 44.0])
    gp = host_plan(sample_rate=256.0, n_samples=1024, q=4.0, freqs=freqs)
    op = o.OraclePlan(fs=256.0, n=1024, q=4.0, f_min=0, f_max=0, rows=6, freqs=freqs)
    compare_tables(gp, op)


@pytest.mark.parametrize("kw", [
    dict(sample_rate=0.0, n_samples=1024, q=4.0, f_min=10.0, f_max=100.0, n_rows=8),
    dict(sample_rate=1024.0, n_samples=1023, q=4.0, f_min=10.0, f_max=100.0, n_rows=8),
    dict(sample_rate=1024.0, n_samples=1024, q=-1.0, f_min=10.0, f_max=100.0, n_rows=8),
    dict(sample_rate=1024.0, n_samples=1024, q=4.0, f_min=10.0, f_max=600.0, n_rows=8),
    dict(sample_rate=1024.0, n_samples=1024, q=4.0, f_min=10.0, f_max=100.0, n_rows=0),
    dict(sample_rate=1024.0, n_samples=1024, q=4.0, f_min=10.0, f_max=100.0, n_rows=8, n_out=8),
    dict(sample_rate=1024.0, n_samples=1024, q=4.0, f_min=10.0, f_max=100.0, n_rows=8, cap_mode="manual"),
])
def test_invalid_parameters_rejected(kw):
    with pytest.raises(qt.QtamError) as e:
        host_plan(**kw)
    assert e.value.status == binding.QTAM_ERR_INVALID_ARG


def test_calls_without_device_return_status():
    gp = host_plan(sample_rate=1024.0, n_samples=4096, q=8.0, f_min=10.0, f_max=400.0, n_rows=16)
    L = binding.lib
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: the call fails validation first
    ws = gp.workspace_bytes(2)
    assert ws >= 2 * gp.info.workspace_bytes_per_segment - 2048
    for fn in (L.qtam_forward, L.qtam_inverse, L.qtam_forward_adjoint, L.qtam_inverse_adjoint):
        assert fn(gp._h, dummy, dummy, 2, dummy, ws, None) == binding.QTAM_ERR_INVALID_ARG
        assert fn(gp._h, dummy, dummy, 0, dummy, ws, None) == binding.QTAM_OK     # empty batch
        assert fn(gp._h, None, dummy, 2, dummy, ws, None) == binding.QTAM_ERR_INVALID_ARG
        assert fn(None, dummy, dummy, 2, dummy, ws, None) == binding.QTAM_ERR_INVALID_ARG
    assert L.qtam_plan_info(None, None) == binding.QTAM_ERR_INVALID_ARG
    L.qtam_plan_destroy(None)


def test_forward_sweep_validation_without_device():
    a = host_plan(sample_rate=1024.0, n_samples=4096, q=4.0, f_min=10.0, f_max=400.0, n_rows=16)
    b = host_plan(sample_rate=1024.0, n_samples=4096, q=16.0, f_min=20.0, f_max=300.0, n_rows=9)
    other_n = host_plan(sample_rate=1024.0, n_samples=8192, q=4.0, f_min=10.0, f_max=400.0, n_rows=16)
    other_p = host_plan(sample_rate=1024.0, n_samples=4096, q=4.0, f_min=10.0, f_max=400.0, n_rows=16,
                        precision=binding.FP64)
    L = binding.lib
    d = ctypes.c_void_p(0x1000)   # never dereferenced: the call fails validation first
    ws = max(a.workspace_bytes(1), b.workspace_bytes(1))

    def call(plans, batch, ys=None, x=d):
        n = len(plans)
        hs = (ctypes.c_void_p * max(n, 1))(*[p._h.value for p in plans])
        ys = (ctypes.c_void_p * max(n, 1))(*([d.value] * n if ys is None else ys))
        return L.qtam_forward_sweep(hs, n, x, ys, batch, d, ws, None)

    assert call([a, b], 0) == binding.QTAM_OK                                  # empty batch
    assert call([a, b], 1) == binding.QTAM_ERR_INVALID_ARG                     # host-only plans
    assert call([a, other_n], 0) == binding.QTAM_ERR_INVALID_ARG               # N differs
    assert call([a, other_p], 0) == binding.QTAM_ERR_INVALID_ARG               # precision differs
    assert call([], 1) == binding.QTAM_ERR_INVALID_ARG                         # no plans
    assert call([a, b], 1, ys=[d.value, None]) == binding.QTAM_ERR_INVALID_ARG  # missing output
    assert call([a, b], 1, x=None) == binding.QTAM_ERR_INVALID_ARG
    assert call([a, b], -1) == binding.QTAM_ERR_INVALID_ARG
    assert L.qtam_forward_sweep(None, 1, d, None, 1, d, ws, None) == binding.QTAM_ERR_INVALID_ARG


def test_unsupported_shapes_report_unsupported_not_invalid():
    """N/2 with an odd factor other than 3 or 5: a valid plan the GPU path
    does not run."""
    gp = host_plan(sample_rate=4096.0, n_samples=2 * 7 * 1024, q=8.0, f_min=20.0, f_max=1000.0, n_rows=62)
    dummy = ctypes.c_void_p(0x1000)
    st_ = binding.lib.qtam_forward(gp._h, dummy, dummy, 1, dummy, 1 << 30, None)
    assert st_ == binding.QTAM_ERR_UNSUPPORTED


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("cap,n_out", [("cover", 0), ("paper", 13677)])
def test_long_chirp_rows_are_supported(precision, cap, n_out):
    """Odd N_out whose chirp-z convolution exceeds one workgroup (the long-
    segment plan's smallest valid N_out, 27353, and the paper's minimal 13677
    under the literal cap): supported, with two rows of the convolution
    length per row and segment in the workspace."""
    kw = dict(sample_rate=8192.0, n_samples=1 << 21, q=12.0, f_min=5.0, f_max=4096.0, n_rows=512,
              cap_mode=cap, precision=precision)
    if n_out == 0:
        n_out = host_plan(**kw).info.max_len
    assert n_out in (27353, 13677)
    gp = host_plan(n_out=n_out, **kw)
    L = 65536 if n_out == 27353 else 32768                 # next power of two >= 2 N_out - 1
    cb = 16 if precision == "fp64" else 8
    assert gp.info.workspace_bytes_per_segment >= 2 * 512 * L * cb
    dummy = ctypes.c_void_p(0x1000)
    # supported shape: a host-only plan fails on the missing device tables, not on the shape
    st_ = binding.lib.qtam_forward(gp._h, dummy, dummy, 1, dummy, 1 << 34, None)
    assert st_ == binding.QTAM_ERR_INVALID_ARG


@pytest.mark.parametrize("n", [24576, 40960, 3 * 65536])
def test_radix_three_and_five_lengths_are_supported(n):
    gp = host_plan(sample_rate=4096.0, n_samples=n, q=8.0, f_min=20.0, f_max=1000.0, n_rows=62)
    dummy = ctypes.c_void_p(0x1000)
    # supported shape: a host-only plan fails on the missing device tables, not on the shape
    st_ = binding.lib.qtam_forward(gp._h, dummy, dummy, 1, dummy, 1 << 30, None)
    assert st_ == binding.QTAM_ERR_INVALID_ARG


COMPOSITES = [
    [(4.0, "bisquare", 0.0), (8.0, "bisquare", 0.0), (16.0, "bisquare", 0.0)],
    [(3.0, "hann", 0.0), (9.0, "kaiser", 6.0), (27.0, "tukey", 0.4), (12.0, "planck", 0.3)],
]


@pytest.mark.parametrize("planes", COMPOSITES)
def test_composite_plan_tables_match_oracle(planes):
    kw = dict(sample_rate=4096.0, n_samples=32768, q=1.0, f_min=16.0, f_max=1800.0, n_rows=40)
    gp = host_plan(planes=planes, **kw)
    op = o.OraclePlan(fs=4096.0, n=32768, q=1.0, f_min=16.0, f_max=1800.0, rows=40,
                      planes=[(q, WINS[w], a) for q, w, a in planes])
    assert gp.planes == len(planes) and gp.rows_per_plane == 40 and gp.R == 40 * len(planes)
    assert np.array_equal(gp.row_q, np.repeat([q for q, _, _ in planes], 40))
    compare_tables(gp, op)


def test_composite_invalid_and_select_without_device():
    with pytest.raises(qt.QtamError):
        host_plan(sample_rate=1024.0, n_samples=4096, q=1.0, f_min=10.0, f_max=400.0, n_rows=16,
                  planes=[(4.0, "bisquare", 0.0), (-2.0, "bisquare", 0.0)])
    gp = host_plan(sample_rate=1024.0, n_samples=4096, q=1.0, f_min=10.0, f_max=400.0, n_rows=16,
                   planes=[(4.0, "bisquare", 0.0), (8.0, "bisquare", 0.0)])
    L = binding.lib
    d = ctypes.c_void_p(0x1000)
    ws = gp.workspace_bytes(1)
    assert L.qtam_forward_metric(gp._h, d, d, None, 1, d, ws, None) == binding.QTAM_ERR_INVALID_ARG
    assert L.qtam_forward_metric(gp._h, d, d, d, 1, d, ws, None) == binding.QTAM_ERR_INVALID_ARG
    assert L.qtam_select_planes(gp._h, d, d, 7, d, d, d, 1, None) == binding.QTAM_ERR_INVALID_ARG
    assert L.qtam_select_planes(gp._h, d, d, 0, d, None, d, 1, None) == binding.QTAM_ERR_INVALID_ARG
    assert L.qtam_select_planes(gp._h, d, d, 0, d, d, d, 1, None) == binding.QTAM_ERR_INVALID_ARG  # host-only
    assert L.qtam_select_planes(gp._h, d, d, 1, None, d, d, 0, None) == binding.QTAM_OK


def test_regularised_plan_tables_match_oracle():
    kw = dict(sample_rate=1024.0, n_samples=4096, q=8.0, f_min=10.0, f_max=400.0, n_rows=16)
    for win, param in (("bisquare", 0.0), ("tukey", 0.5)):
        gp = host_plan(window=win, window_param=param, window_eps=1e-5, **kw)
        op = o.OraclePlan(fs=1024.0, n=4096, q=8.0, f_min=10.0, f_max=400.0, rows=16, window=WINS[win],
                          window_param=param, eps=1e-5)
        compare_tables(gp, op)
        assert gp.info.max_len == 4096 // 2 + 1 and np.all(gp.windows_dense() > 0)
    L = binding.lib
    d = ctypes.c_void_p(0x1000)
    plain = host_plan(**kw)
    assert L.qtam_tile_inverse(plain._h, d, 0, d, 1, d, 1 << 20, None) == binding.QTAM_ERR_INVALID_ARG
    reg = host_plan(window_eps=1e-5, **kw)
    assert L.qtam_tile_inverse(reg._h, d, 16, d, 1, d, 1 << 20, None) == binding.QTAM_ERR_INVALID_ARG
    assert L.qtam_tile_inverse(reg._h, d, 0, d, 0, d, 1 << 20, None) == binding.QTAM_OK
    with pytest.raises(qt.QtamError):
        host_plan(window_eps=-1.0, **kw)


def test_unknown_precision_rejected():
    with pytest.raises(ValueError):
        host_plan(sample_rate=1024.0, n_samples=4096, q=8.0, f_min=10.0, f_max=400.0, n_rows=16, precision="fp16")
    assert host_plan(sample_rate=1024.0, n_samples=4096, q=8.0, f_min=10.0, f_max=400.0, n_rows=16,
                     precision="float64").fp64


def test_output_and_workspace_checks():
    """Caller-supplied outputs and workspaces are checked for exact shape,
    dtype, device and contiguity before any pointer reaches the library (it
    writes the whole expected shape through the base pointer)."""
    import torch
    dev = torch.device("cpu")
    good = torch.empty((2, 3, 8), dtype=torch.complex64)
    assert binding.expect_tensor(good, (2, 3, 8), torch.complex64, dev, "out") is good
    bad = [
        torch.empty((2, 3, 7), dtype=torch.complex64),             # short rows
        torch.empty((1, 3, 8), dtype=torch.complex64),             # short batch
        torch.empty((2, 3, 8), dtype=torch.complex128),            # dtype
        torch.empty((2, 8, 3), dtype=torch.complex64).transpose(1, 2),   # strided
        torch.empty((2, 3, 16), dtype=torch.complex64)[..., ::2],  # strided view
        np.zeros((2, 3, 8), dtype=np.complex64),                   # not a tensor
    ]
    for t in bad:
        with pytest.raises(ValueError):
            binding.expect_tensor(t, (2, 3, 8), torch.complex64, dev, "out")
    with pytest.raises(ValueError):
        binding.expect_tensor(good, (2, 3, 8), torch.complex64, torch.device("cuda", 0), "out")
    ws = torch.empty(1024, dtype=torch.uint8)
    assert binding.expect_workspace(ws, dev) is ws
    with pytest.raises(ValueError):
        binding.expect_workspace(ws, torch.device("cuda", 0))
    with pytest.raises(ValueError):
        binding.expect_workspace(torch.empty(2048, dtype=torch.uint8)[::2], dev)
    with pytest.raises(ValueError):
        binding.expect_workspace(bytearray(16), dev)


def test_noalloc_forward_rejects_plans_beyond_its_workspace():
    """qtam_forward_noalloc checks the plan against its static workspace before
    touching the device: a plan one segment of which needs more (the
    long-segment plan in FP64: two-pass rows) gets QTAM_ERR_WORKSPACE with the
    sizes in qtam_last_error; a plan that fits but has no device tables gets
    QTAM_ERR_INVALID_ARG."""
    big = host_plan(sample_rate=8192.0, n_samples=1 << 21, q=12.0, f_min=5.0, f_max=4096.0, n_rows=512,
                    precision="fp64")
    hdr = open(os.path.join(ROOT, "include", "qtam.h")).read()
    m = re.search(r"#define QTAM_NOALLOC_WORKSPACE_BYTES \(\(size_t\)(\d+) << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == binding.NOALLOC_WORKSPACE_BYTES
    assert big.workspace_bytes(1) > binding.NOALLOC_WORKSPACE_BYTES
    dummy = ctypes.c_void_p(0x1000)
    assert binding.lib.qtam_forward_noalloc(big._h, dummy, dummy, 1, None) == binding.QTAM_ERR_WORKSPACE
    msg = binding.lib.qtam_last_error().decode()
    assert "qtam_forward_noalloc" in msg and str(binding.NOALLOC_WORKSPACE_BYTES) in msg
    small = host_plan(sample_rate=4096.0, n_samples=16384, q=8.0, f_min=20.0, f_max=1000.0, n_rows=64)
    assert small.workspace_bytes(1) <= binding.NOALLOC_WORKSPACE_BYTES
    assert binding.lib.qtam_forward_noalloc(small._h, dummy, dummy, 1, None) == binding.QTAM_ERR_INVALID_ARG
    assert binding.lib.qtam_forward_noalloc(None, dummy, dummy, 1, None) == binding.QTAM_ERR_INVALID_ARG


def test_plan_host_allocation_failure_is_oom():
    """A plan whose host tables cannot be allocated (2^44 samples: the frame
    operator alone would take 64 TiB) returns QTAM_ERR_OOM instead of letting
    the allocation failure cross the C boundary; the host then stays usable.
    Skipped where such an allocation would succeed untouched (a permissive
    overcommit policy), so the test never commits that memory."""
    libc = ctypes.CDLL("libc.so.6")
    libc.malloc.restype = ctypes.c_void_p
    libc.malloc.argtypes = [ctypes.c_size_t]
    libc.free.argtypes = [ctypes.c_void_p]
    probe = libc.malloc(1 << 46)
    if probe:
        libc.free(probe)
        pytest.skip("64 TiB malloc succeeds here (overcommit): not forcing the failure")
    with pytest.raises(qt.QtamError) as e:
        host_plan(sample_rate=float(1 << 40), n_samples=1 << 44, q=8.0, f_min=100.0, f_max=200.0, n_rows=1)
    assert e.value.status == binding.QTAM_ERR_OOM
    assert "host memory" in binding.lib.qtam_last_error().decode()
    assert host_plan(sample_rate=4096.0, n_samples=16384, q=8.0, f_min=20.0, f_max=1000.0, n_rows=64).R == 64


@pytest.mark.parametrize("precision,b", [("fp32", 4), ("fp64", 8)])
def test_mask_entry_points_validate_without_device(precision, b):
    """The denoiser's mask calls: workspace of one real per (segment, row);
    argument checks before any device work (a plan without device tables,
    NULL buffers, negative batches); an empty forward batch is a no-op."""
    gp = host_plan(sample_rate=4096.0, n_samples=32768, q=8.0, f_min=20.0, f_max=2000.0, n_rows=128,
                   precision=precision)
    L = binding.lib
    assert L.qtam_mask_workspace_size(gp._h, 64) == 64 * 128 * b
    assert L.qtam_mask_workspace_size(gp._h, 0) == 0
    assert L.qtam_mask_workspace_size(None, 4) == 0
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: the calls fail validation first
    ws = L.qtam_mask_workspace_size(gp._h, 2)
    inv = binding.QTAM_ERR_INVALID_ARG
    assert L.qtam_mask_forward(gp._h, dummy, dummy, dummy, dummy, 0, None) == binding.QTAM_OK
    assert L.qtam_mask_forward(gp._h, dummy, dummy, dummy, dummy, 2, None) == inv      # no device tables
    assert L.qtam_mask_forward(gp._h, dummy, dummy, dummy, dummy, -1, None) == inv
    assert L.qtam_mask_forward(None, dummy, dummy, dummy, dummy, 2, None) == inv
    args = (dummy, dummy, dummy, dummy, dummy, dummy)
    assert L.qtam_mask_backward(gp._h, *args, 2, dummy, ws, None) == inv               # no device tables
    assert L.qtam_mask_backward(gp._h, *args, -1, dummy, ws, None) == inv
    assert L.qtam_mask_backward(None, *args, 2, dummy, ws, None) == inv
    assert L.qtam_mask_backward(gp._h, dummy, None, dummy, dummy, dummy, dummy, 0, None, 0, None) == inv


def test_masked_inverse_support_and_validation_without_device():
    """The fused mask + inverse calls: supported where rows take one
    workgroup (an empty batch asks), QTAM_ERR_UNSUPPORTED on two-pass rows
    (FP64 rows of 16384 points); workspace = the partial sums (256-aligned)
    + the transform's; argument checks before any device work."""
    L = binding.lib
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: the calls fail validation first
    gp = host_plan(sample_rate=4096.0, n_samples=32768, q=8.0, f_min=20.0, f_max=2000.0, n_rows=128)
    assert gp.masked_inverse_supported
    assert L.qtam_masked_adjoint_workspace_size(gp._h, 3) == (3 * 128 * 4 + 255) // 256 * 256 + gp.workspace_bytes(3)
    assert L.qtam_masked_adjoint_workspace_size(gp._h, 0) == 0
    ws = L.qtam_masked_adjoint_workspace_size(gp._h, 2)
    inv = binding.QTAM_ERR_INVALID_ARG
    assert L.qtam_inverse_masked(gp._h, dummy, dummy, dummy, dummy, 2, dummy, ws, None) == inv   # no device tables
    assert L.qtam_inverse_masked(gp._h, dummy, None, dummy, dummy, 2, dummy, ws, None) == inv
    assert L.qtam_inverse_masked(None, dummy, dummy, dummy, dummy, 2, dummy, ws, None) == inv
    args = (dummy, dummy, dummy, dummy, dummy, dummy)
    assert L.qtam_inverse_masked_adjoint(gp._h, *args, 2, dummy, ws, None) == inv
    assert L.qtam_inverse_masked_adjoint(gp._h, *args, -1, dummy, ws, None) == inv
    assert L.qtam_inverse_masked_adjoint(gp._h, dummy, dummy, dummy, dummy, dummy, None, 2, dummy, ws, None) == inv
    long_rows = host_plan(sample_rate=4096.0, n_samples=24576, q=8.0, f_min=10.0, f_max=2048.0, n_rows=62,
                          precision="fp64", n_out=16384)
    assert not long_rows.masked_inverse_supported
    uns = binding.QTAM_ERR_UNSUPPORTED
    assert L.qtam_inverse_masked(long_rows._h, None, None, None, None, 0, None, 0, None) == uns
    assert L.qtam_inverse_masked_adjoint(long_rows._h, *args, 1, dummy, ws, None) == uns


def test_header_compiles_as_c99_and_cxx17(tmp_path):
    """include/qtam.h is a plain C header: it compiles as strict C99 and as
    C++17, with every entry point referenced."""
    import shutil
    import subprocess
    hdr = open(os.path.join(ROOT, "include", "qtam.h")).read()
    names = sorted(set(re.findall(r"\b(qtam_[a-z0-9_]+)\s*\(", hdr)))
    assert "qtam_inverse_masked_adjoint" in names and "qtam_forward_noalloc" in names
    src = tmp_path / "use.c"
    src.write_text('#include "qtam.h"\ntypedef void (*fn)(void);\nfn table[] = {' +
                   ", ".join("(fn)" + n for n in names) + "};\nint main(void) { return table[0] == 0; }\n")
    for cc, std, lang in (("gcc", "-std=c99", "c"), ("g++", "-std=c++17", "c++")):
        if shutil.which(cc) is None:
            pytest.skip(cc + " not available")
        r = subprocess.run([cc, std, "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only", "-x", lang,
                            "-I" + os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def test_c_caller_without_python_or_gpu(tmp_path):
    """tests/c_abi_host.c, a plain C99 caller linked against libqtam.so, runs
    on a machine without a GPU: host-only plans, their tables (the frame is
    the sum of the squared windows), workspace sizes and status codes."""
    import shutil
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    libdir = os.path.dirname(binding.LIB_PATH)
    exe = tmp_path / "c_abi_host"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "c_abi_host.c"),
                        "-o", str(exe), "-L" + libdir, "-lqtam", "-Wl,-rpath," + libdir, "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.rstrip().endswith("PASSED"), r.stdout + r.stderr


def test_mask_binding_rejects_host_tensors():
    """The mask and masked-inverse methods take device tensors only: host
    tensors raise before any pointer reaches the library."""
    import torch
    gp = host_plan(sample_rate=4096.0, n_samples=32768, q=8.0, f_min=20.0, f_max=2000.0, n_rows=128)
    y = torch.zeros((1, gp.R, gp.N_out), dtype=torch.complex64)
    g = torch.ones(gp.R)
    x = torch.zeros((1, gp.N))
    for call in (lambda: gp.mask_forward(y, g, g), lambda: gp.mask_backward(y, g, g, y),
                 lambda: gp.inverse_masked(y, g, g), lambda: gp.inverse_masked_adjoint(x, y, g, g)):
        with pytest.raises(TypeError):
            call()
