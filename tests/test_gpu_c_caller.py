"""The library called from C on the GPU: tests/c_abi_gpu.c (HIP runtime and
libqtam.so only, no Python or torch in that process) runs qtam_forward and
qtam_inverse on two segments of the one-segment workload's shape; its
envelopes and reconstructions are compared with the oracle on the same
input bits (coefficients, and the reconstruction against the projection
x_M), at the FP32 / FP64 bars."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synthetic
from oracle import oracle as o

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL = {"fp32": 1e-5, "fp64": 1e-12}
FS, N, Q, FMIN, FMAX, R = 4096.0, 16384, 8.0, 20.0, 1000.0, 64


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    from paper_2603_29785_amd import binding
    libdir = os.path.dirname(binding.LIB_PATH)
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    out = tmp_path_factory.mktemp("c_caller") / "c_abi_gpu"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                        "-I" + os.path.join(rocm, "include"), "-I" + os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "c_abi_gpu.c"), "-o", str(out),
                        "-L" + os.path.join(rocm, "lib"), "-lamdhip64", "-L" + libdir, "-lqtam",
                        "-Wl,-rpath," + libdir, "-Wl,-rpath," + os.path.join(rocm, "lib")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def rel_rows(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_c_caller_forward_inverse(exe, tmp_path, precision):
    B = 2
    x = np.stack([synthetic.injected_segment(N, FS, synthetic.rng_for(51, i))[0] for i in range(B)])
    if precision == "fp32":
        x = x.astype(np.float32).astype(np.float64)      # the bits the device sees
    fin, fy, fx = tmp_path / "x.bin", tmp_path / "y.bin", tmp_path / "xr.bin"
    np.ascontiguousarray(x, dtype=np.float64).tofile(fin)
    print(f"c caller {precision}: B={B} N={N} R={R}", flush=True)
    r = subprocess.run([str(exe), str(FS), str(N), str(Q), str(FMIN), str(FMAX), str(R), precision, str(B),
                        str(fin), str(fy), str(fx)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    op = o.OraclePlan(fs=FS, n=N, q=Q, f_min=FMIN, f_max=FMAX, rows=R)
    Y = np.fromfile(fy, dtype=np.float64).view(np.complex128).reshape(B, op.R, op.N_out)
    xr = np.fromfile(fx, dtype=np.float64).reshape(B, N)
    e_y = rel_rows(Y, op.forward(x)).max()
    e_x = rel_rows(xr, np.stack([op.project(x[b]) for b in range(B)])).max()
    print(f"  coef {e_y:.3e}, reconstruction vs x_M {e_x:.3e}", flush=True)
    assert e_y <= TOL[precision] and e_x <= TOL[precision]
