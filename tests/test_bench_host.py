"""Host logic of bench.py (no GPU): the single-GPU guard, the algorithmic byte
counts of the roofline against the sizes of the buffers each kernel reads and
writes, and the reader of the committed counter summary."""
import os
import subprocess
import sys
import types

import numpy as np
import pytest

import paper_2603_29785_amd as qt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("precision,cdt,rdt", [("fp32", np.complex64, np.float32),
                                                ("fp64", np.complex128, np.float64)])
def test_design_bytes_are_buffer_sizes(precision, cdt, rdt):
    """Each kernel's design bytes equal the nbytes of the arrays it reads and
    writes once: signal [B, N], half spectrum [B, N/2], envelopes
    [B, R, N_out], kept slots [B, sum of row supports]."""
    p = qt.Plan(4096.0, 131072, 8.0, 10.0, 2048.0, 256, precision=precision, host_only=True)
    B = 3
    b = np.dtype(rdt).itemsize
    x = np.empty((B, p.N), rdt).nbytes
    half = np.empty((B, p.N // 2), cdt).nbytes
    y = np.empty((B, p.R, p.N_out), cdt).nbytes
    s = np.empty((B, p.info.sum_len), cdt).nbytes
    want = {"fwd_rows": y + half, "inv_rows": y + s, "overlap_add": s + half,
            "spectrum_fft": x + half, "spectrum_twist": 2 * half,
            "spectrum_fft_pass1": x + half, "spectrum_fft_pass2": 2 * half,
            "synthesis_fft": half + x, "synthesis_fft_pass1": 2 * half, "synthesis_fft_pass2": half + x}
    for kind, nbytes in want.items():
        assert bench.design_bytes(kind, p, B, b) == float(nbytes), kind
    assert bench.design_bytes("no_such_kernel", p, B, b) is None


# the kernels one forward + inverse launches, by form of the spectrum and of the rows
PATHS = {
    "four-step spectrum": ["spectrum_fft_pass1", "spectrum_fft_pass2", "fwd_rows", "inv_rows", "overlap_add",
                           "synthesis_fft_pass1", "synthesis_fft_pass2"],
    "one-pass spectrum": ["spectrum_fft", "spectrum_twist", "fwd_rows", "inv_rows", "overlap_add",
                          "synthesis_fft"],
    "decimated spectrum": ["spectrum_permute", "spectrum_fft", "spectrum_radix", "spectrum_twist", "fwd_rows",
                           "inv_rows", "overlap_add", "synthesis_radix", "synthesis_fft", "synthesis_permute"],
    "long rows": ["spectrum_fft_pass1", "spectrum_fft_pass2", "fwd_rows", "fwd_rows_pass2", "inv_rows",
                  "inv_rows_pass2", "overlap_add", "synthesis_fft_pass1", "synthesis_fft_pass2"],
}


@pytest.mark.parametrize("form,plan_args", [
    ("four-step spectrum", (4096.0, 131072, 8.0, 10.0, 2048.0, 256)),
    ("one-pass spectrum", (4096.0, 16384, 8.0, 20.0, 1000.0, 64)),
    ("decimated spectrum", (4096.0, 24576, 8.0, 20.0, 2000.0, 62)),
    ("long rows", (8192.0, 1 << 21, 12.0, 5.0, 4096.0, 512)),
])
@pytest.mark.parametrize("precision,b", [("fp32", 4), ("fp64", 8)])
def test_algorithmic_shares_add_up(form, plan_args, precision, b):
    """The kernels' algorithmic shares of one forward + inverse add up to
    2 b N + 4 b R N_out per segment (read x, write Y, read Y, write x-hat),
    whatever passes the path takes; the roofline's per-launch figure is one
    kernel's share."""
    p = qt.Plan(*plan_args, precision=precision, host_only=True)
    B = 5
    kinds = PATHS[form]
    if form == "long rows" and not bench.long_rows(p):
        kinds = [k for k in kinds if not k.endswith("pass2") or k.startswith(("spectrum", "synthesis"))]
    total = sum(bench.kernel_bytes(k, p, B, b) for k in kinds)
    assert total == float(B * (2 * b * p.N + 4 * b * p.R * p.N_out))
    assert bench.kernel_bytes("inv_rows", p, B, b) == float(B * 2 * b * p.R * p.N_out)
    assert bench.kernel_bytes("overlap_add", p, B, b) == 0.0
    assert bench.kernel_bytes("no_such_kernel", p, B, b) is None


def test_cpu_model_names_the_host():
    m = bench.cpu_model()
    assert isinstance(m, str) and m


def test_measured_traffic_only_for_current_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("inv_rows", 256) is None                  # no summary
    f.write_text("# calibrated\nsource_digest: %s\nbatch: 256\ninv_rows: 1234\n" % bench.source_digest())
    assert bench.measured_traffic("inv_rows", 256) == 1234.0
    assert bench.measured_traffic("inv_rows", 128) is None                  # another batch
    assert bench.measured_traffic("fwd_rows", 256) is None                  # kernel not counted
    f.write_text("source_digest: 0000000000000000\nbatch: 256\ninv_rows: 1234\n")
    assert bench.measured_traffic("inv_rows", 256) is None                  # other sources


def test_source_digest_covers_kernel_sources():
    d = bench.source_digest()
    assert len(d) == 16 and int(d, 16) >= 0
    base = os.path.join(ROOT, "paper_2603_29785_amd", "csrc")
    assert any(n.endswith(".hip") for n in os.listdir(base))
    assert d == bench.source_digest()
