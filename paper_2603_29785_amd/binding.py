"""ctypes binding of libqtam.so (include/qtam.h).

Argument marshalling only: every step of the transform runs in the HIP
kernels of the library. PyTorch provides device memory and streams. There is
no CPU fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("QTAM_LIB") or os.path.join(_HERE, "libqtam.so")

QTAM_OK, QTAM_ERR_INVALID_ARG, QTAM_ERR_UNSUPPORTED, QTAM_ERR_WORKSPACE, QTAM_ERR_OOM, QTAM_ERR_DEVICE = range(6)
FP32, FP64 = 0, 1
CAP = {"cover": 0, "paper": 1, "none": 2, "manual": 3}
NORM = {"unit_energy": 0, "paper_inv_energy": 1, "none": 2}
WINDOW = {"bisquare": 0, "hann": 1, "kaiser": 2, "tukey": 3, "planck": 4}
PLAN_HOST_ONLY = 1
METRIC = {"energy": 0, "peak": 1}


class QtamError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        detail = ""
        if status in (QTAM_ERR_DEVICE, QTAM_ERR_OOM):
            detail = lib.qtam_last_error().decode()
        super().__init__("%s: %s (status %d)%s" % (what, status_string(status), status,
                                                   ": " + detail if detail else ""))


class c_params(ctypes.Structure):
    _fields_ = [
        ("sample_rate", ctypes.c_double),
        ("n_samples", ctypes.c_int64),
        ("q", ctypes.c_double),
        ("f_min", ctypes.c_double),
        ("f_max", ctypes.c_double),
        ("n_rows", ctypes.c_int32),
        ("freqs", ctypes.POINTER(ctypes.c_double)),
        ("window", ctypes.c_int32),
        ("window_param", ctypes.c_double),
        ("cap_mode", ctypes.c_int32),
        ("max_window", ctypes.c_int32),
        ("norm_mode", ctypes.c_int32),
        ("n_out", ctypes.c_int32),
        ("p_floor_rel", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("n_planes", ctypes.c_int32),
        ("plane_q", ctypes.POINTER(ctypes.c_double)),
        ("plane_window", ctypes.POINTER(ctypes.c_int32)),
        ("plane_window_param", ctypes.POINTER(ctypes.c_double)),
        ("window_eps", ctypes.c_double),
    ]


class c_info(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int32),
        ("n_planes", ctypes.c_int32),
        ("rows_per_plane", ctypes.c_int32),
        ("n_out", ctypes.c_int32),
        ("max_len", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("n_samples", ctypes.c_int64),
        ("n_bins", ctypes.c_int64),
        ("sum_len", ctypes.c_int64),
        ("l_max", ctypes.c_int64),
        ("frame_A", ctypes.c_double),
        ("frame_B", ctypes.c_double),
        ("masked_fraction", ctypes.c_double),
        ("workspace_bytes_per_segment", ctypes.c_size_t),
        ("freqs", ctypes.POINTER(ctypes.c_double)),
        ("row_q", ctypes.POINTER(ctypes.c_double)),
        ("centre", ctypes.POINTER(ctypes.c_int32)),
        ("half_width", ctypes.POINTER(ctypes.c_int32)),
        ("lo", ctypes.POINTER(ctypes.c_int32)),
        ("hi", ctypes.POINTER(ctypes.c_int32)),
        ("offset", ctypes.POINTER(ctypes.c_int64)),
        ("window", ctypes.POINTER(ctypes.c_double)),
        ("frame", ctypes.POINTER(ctypes.c_double)),
        ("mask", ctypes.POINTER(ctypes.c_uint8)),
    ]


# Size of the static device workspace of qtam_forward_noalloc (QTAM_NOALLOC_WORKSPACE_BYTES).
NOALLOC_WORKSPACE_BYTES = 64 << 20

EXPORTED = [
    "qtam_plan_create", "qtam_plan_info", "qtam_plan_destroy", "qtam_workspace_size",
    "qtam_forward", "qtam_inverse", "qtam_forward_adjoint", "qtam_inverse_adjoint",
    "qtam_forward_metric", "qtam_select_planes", "qtam_timing_enable", "qtam_timing_collect", "qtam_status_string",
    "qtam_dense", "qtam_dense_workspace_size", "qtam_tile_inverse", "qtam_last_error", "qtam_version",
    "qtam_forward_sweep", "qtam_forward_noalloc", "qtam_mask_forward", "qtam_mask_backward",
    "qtam_mask_workspace_size", "qtam_inverse_masked", "qtam_inverse_masked_adjoint",
    "qtam_masked_adjoint_workspace_size",
]


def _load():
    # PyTorch's HIP runtime first: libqtam.so then binds to that same runtime
    # (its soname is already loaded) instead of bringing a second copy into
    # the process beside the one torch loads for its own tensors and streams.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqtam.so not built at %s: run python paper_2603_29785_amd/build.py" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    L.qtam_plan_create.argtypes = [ctypes.POINTER(c_params), ctypes.POINTER(vp)]
    L.qtam_plan_create.restype = ctypes.c_int
    L.qtam_plan_info.argtypes = [vp, ctypes.POINTER(c_info)]
    L.qtam_plan_info.restype = ctypes.c_int
    L.qtam_plan_destroy.argtypes = [vp]
    L.qtam_plan_destroy.restype = None
    L.qtam_workspace_size.argtypes = [vp, i64]
    L.qtam_workspace_size.restype = sz
    for name in ("qtam_forward", "qtam_inverse", "qtam_forward_adjoint", "qtam_inverse_adjoint"):
        f = getattr(L, name)
        f.argtypes = [vp, vp, vp, i64, vp, sz, vp]
        f.restype = ctypes.c_int
    L.qtam_mask_forward.argtypes = [vp, vp, vp, vp, vp, i64, vp]
    L.qtam_mask_forward.restype = ctypes.c_int
    L.qtam_mask_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, i64, vp, sz, vp]
    L.qtam_mask_backward.restype = ctypes.c_int
    L.qtam_mask_workspace_size.argtypes = [vp, i64]
    L.qtam_mask_workspace_size.restype = sz
    L.qtam_inverse_masked.argtypes = [vp, vp, vp, vp, vp, i64, vp, sz, vp]
    L.qtam_inverse_masked.restype = ctypes.c_int
    L.qtam_inverse_masked_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, i64, vp, sz, vp]
    L.qtam_inverse_masked_adjoint.restype = ctypes.c_int
    L.qtam_masked_adjoint_workspace_size.argtypes = [vp, i64]
    L.qtam_masked_adjoint_workspace_size.restype = sz
    L.qtam_forward_noalloc.argtypes = [vp, vp, vp, i64, vp]
    L.qtam_forward_noalloc.restype = ctypes.c_int
    L.qtam_tile_inverse.argtypes = [vp, vp, ctypes.c_int32, vp, i64, vp, sz, vp]
    L.qtam_tile_inverse.restype = ctypes.c_int
    L.qtam_dense.argtypes = [vp, vp, vp, i64, vp, sz, vp]
    L.qtam_dense.restype = ctypes.c_int
    L.qtam_dense_workspace_size.argtypes = [vp, i64]
    L.qtam_dense_workspace_size.restype = sz
    L.qtam_forward_sweep.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, vp, ctypes.POINTER(vp), i64, vp, sz, vp]
    L.qtam_forward_sweep.restype = ctypes.c_int
    L.qtam_forward_metric.argtypes = [vp, vp, vp, vp, i64, vp, sz, vp]
    L.qtam_forward_metric.restype = ctypes.c_int
    L.qtam_select_planes.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp, vp, i64, vp]
    L.qtam_select_planes.restype = ctypes.c_int
    L.qtam_timing_enable.argtypes = [vp, ctypes.c_int32]
    L.qtam_timing_enable.restype = ctypes.c_int
    L.qtam_timing_collect.argtypes = [vp, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32)]
    L.qtam_timing_collect.restype = ctypes.c_int
    L.qtam_status_string.argtypes = [ctypes.c_int]
    L.qtam_status_string.restype = ctypes.c_char_p
    L.qtam_last_error.argtypes = []
    L.qtam_last_error.restype = ctypes.c_char_p
    L.qtam_version.argtypes = []
    L.qtam_version.restype = ctypes.c_char_p
    return L


lib = _load()


def status_string(s: int) -> str:
    return lib.qtam_status_string(int(s)).decode()


def version() -> str:
    return lib.qtam_version().decode()


def _check(status: int, what: str):
    if status != QTAM_OK:
        raise QtamError(status, what)


def _arr(ptr, n, dtype):
    if n == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def expect_tensor(t, shape, dtype, device, what: str):
    """Raises ValueError unless t is a contiguous tensor of exactly this shape
    and dtype on this device: the library is handed only a base pointer and
    writes every element of the expected shape through it."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a tensor" % what)
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s tensor of shape %s on %s; got %s %s on %s%s" % (
            what, dtype, tuple(shape), device, t.dtype, tuple(t.shape), t.device,
            "" if t.is_contiguous() else " (not contiguous)"))
    return t


def expect_workspace(ws, device):
    """Raises ValueError unless ws is a contiguous tensor on `device` (its
    byte size, numel * element_size, is passed to the library, which checks
    it against what the call needs)."""
    import torch
    if not isinstance(ws, torch.Tensor) or ws.device != device or not ws.is_contiguous():
        raise ValueError("workspace must be a contiguous tensor on %s; got %s" % (
            device, ("%s tensor on %s" % (tuple(ws.shape), ws.device)) if isinstance(ws, torch.Tensor)
            else type(ws).__name__))
    return ws


@dataclass(frozen=True)
class PlanInfo:
    n_rows: int
    n_planes: int
    rows_per_plane: int
    n_out: int
    max_len: int
    precision: int
    n_samples: int
    n_bins: int
    sum_len: int
    l_max: int
    frame_A: float
    frame_B: float
    masked_fraction: float
    workspace_bytes_per_segment: int


class Plan:
    """A QTAM plan (immutable). Tables are built in FP64 on the host and
    uploaded once to the current device unless ``host_only``."""

    def __init__(self, sample_rate: float, n_samples: int, q: float, f_min: float = 0.0,
                 f_max: float = 0.0, n_rows: int = 0, freqs=None, window: str = "bisquare",
                 window_param: float = 0.0, cap_mode: str = "cover", max_window: int = 0,
                 norm_mode: str = "unit_energy", n_out: int = 0, p_floor_rel: float = 1e-6,
                 precision: str = "fp32", host_only: bool = False, planes=None, window_eps: float = 0.0):
        """planes: optional list of (q, window, window_param) for a composite
        bank (rows plane after plane, one shared frame); q, window and
        window_param are then ignored."""
        self._h = ctypes.c_void_p()
        p = c_params()
        p.sample_rate = float(sample_rate)
        p.n_samples = int(n_samples)
        p.q = float(q)
        p.f_min = float(f_min)
        p.f_max = float(f_max)
        self._freqs = None
        if freqs is not None:
            self._freqs = np.ascontiguousarray(freqs, dtype=np.float64)
            p.freqs = self._freqs.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            p.n_rows = int(self._freqs.size)
        else:
            p.n_rows = int(n_rows)
        p.window = WINDOW[window] if isinstance(window, str) else int(window)
        p.window_param = float(window_param)
        p.cap_mode = CAP[cap_mode] if isinstance(cap_mode, str) else int(cap_mode)
        p.max_window = int(max_window)
        p.norm_mode = NORM[norm_mode] if isinstance(norm_mode, str) else int(norm_mode)
        p.n_out = int(n_out)
        p.p_floor_rel = float(p_floor_rel)
        if precision in ("fp64", "float64", FP64):
            p.precision = FP64
        elif precision in ("fp32", "float32", FP32):
            p.precision = FP32
        else:
            raise ValueError("precision must be 'fp32' or 'fp64', got %r" % (precision,))
        p.flags = PLAN_HOST_ONLY if host_only else 0
        p.window_eps = float(window_eps)
        if planes:
            self._pq = np.array([float(t[0]) for t in planes], dtype=np.float64)
            self._pw = np.array([WINDOW[t[1]] if isinstance(t[1], str) else int(t[1]) for t in planes],
                                dtype=np.int32)
            self._pp = np.array([float(t[2]) for t in planes], dtype=np.float64)
            p.n_planes = len(planes)
            p.plane_q = self._pq.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            p.plane_window = self._pw.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            p.plane_window_param = self._pp.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.params = dict(sample_rate=sample_rate, n_samples=n_samples, q=q, f_min=f_min, f_max=f_max,
                           n_rows=p.n_rows, window=window, window_param=window_param, cap_mode=cap_mode,
                           max_window=max_window, norm_mode=norm_mode, n_out=n_out,
                           p_floor_rel=p_floor_rel, precision=precision, planes=planes, window_eps=window_eps)
        _check(lib.qtam_plan_create(ctypes.byref(p), ctypes.byref(self._h)), "qtam_plan_create")
        ci = c_info()
        _check(lib.qtam_plan_info(self._h, ctypes.byref(ci)), "qtam_plan_info")
        self.info = PlanInfo(ci.n_rows, ci.n_planes, ci.rows_per_plane, ci.n_out, ci.max_len, ci.precision, ci.n_samples, ci.n_bins,
                             ci.sum_len, ci.l_max, ci.frame_A, ci.frame_B, ci.masked_fraction,
                             ci.workspace_bytes_per_segment)
        R, nb, sl = ci.n_rows, ci.n_bins, ci.sum_len
        self.freqs = _arr(ci.freqs, R, np.float64)
        self.row_q = _arr(ci.row_q, R, np.float64)
        self.centre = _arr(ci.centre, R, np.int64)
        self.half_width = _arr(ci.half_width, R, np.int64)
        self.lo = _arr(ci.lo, R, np.int64)
        self.hi = _arr(ci.hi, R, np.int64)
        self.offset = _arr(ci.offset, R, np.int64)
        self.window_table = _arr(ci.window, sl, np.float64)
        self.frame = _arr(ci.frame, nb, np.float64)
        self.mask = _arr(ci.mask, nb, np.uint8).astype(bool)
        self.host_only = host_only
        self._ws = None

    def __del__(self, _destroy=lib.qtam_plan_destroy):
        # the library function is bound at definition time: at interpreter exit
        # the module's globals may already be gone when a plan is collected
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _destroy(h)
            h.value = None

    # ------------------------------------------------------------------ sizes
    @property
    def R(self) -> int:
        return self.info.n_rows

    @property
    def N(self) -> int:
        return self.info.n_samples

    @property
    def N_out(self) -> int:
        return self.info.n_out

    @property
    def planes(self) -> int:
        return self.info.n_planes

    @property
    def rows_per_plane(self) -> int:
        return self.info.rows_per_plane

    @property
    def fp64(self) -> bool:
        return self.info.precision == FP64

    def windows_dense(self) -> np.ndarray:
        """W as a dense [R, N/2+1] matrix (host, FP64)."""
        W = np.zeros((self.R, self.info.n_bins))
        for k in range(self.R):
            a, b, o = self.lo[k], self.hi[k], self.offset[k]
            W[k, a:b + 1] = self.window_table[o:o + b - a + 1]
        return W

    def workspace_bytes(self, batch: int) -> int:
        return int(lib.qtam_workspace_size(self._h, int(batch)))

    # ------------------------------------------------------------ transforms
    def _torch(self):
        import torch
        return torch

    def _real_dtype(self):
        torch = self._torch()
        return torch.float64 if self.fp64 else torch.float32

    def _complex_dtype(self):
        torch = self._torch()
        return torch.complex128 if self.fp64 else torch.complex64

    def _workspace(self, batch: int, device, ws=None):
        torch = self._torch()
        need = self.workspace_bytes(batch)
        if ws is not None:
            return expect_workspace(ws, device)
        if self._ws is None or self._ws.numel() < need or self._ws.device != device:
            self._ws = torch.empty(need, dtype=torch.uint8, device=device)
        return self._ws

    def _out(self, out, shape, dtype, device, what="out"):
        """A new output tensor, or the caller's after checking it exactly."""
        if out is None:
            return self._torch().empty(shape, dtype=dtype, device=device)
        return expect_tensor(out, shape, dtype, device, what)

    def _call(self, fn, what, src, dst, batch, ws, stream):
        torch = self._torch()
        if stream is None:
            stream = torch.cuda.current_stream(src.device)
        ws = self._workspace(batch, src.device, ws)
        _check(fn(self._h, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), int(batch),
                  ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * ws.element_size()),
                  ctypes.c_void_p(stream.cuda_stream)), what)

    def _check_signal(self, x):
        torch = self._torch()
        if not (isinstance(x, torch.Tensor) and x.is_cuda):
            raise TypeError("expected a CUDA (HIP) tensor")
        if x.dtype != self._real_dtype() or x.shape[-1] != self.N:
            raise ValueError("expected real %s [..., %d], got %s %s" % (self._real_dtype(), self.N, x.dtype,
                                                                        tuple(x.shape)))
        return x.contiguous()

    def _check_rows(self, y):
        torch = self._torch()
        if not (isinstance(y, torch.Tensor) and y.is_cuda):
            raise TypeError("expected a CUDA (HIP) tensor")
        if y.dtype != self._complex_dtype() or tuple(y.shape[-2:]) != (self.R, self.N_out):
            raise ValueError("expected complex %s [..., %d, %d], got %s %s" % (
                self._complex_dtype(), self.R, self.N_out, y.dtype, tuple(y.shape)))
        return y.contiguous()

    def forward(self, x, out=None, ws=None, stream=None):
        """x [..., N] real -> Y [..., R, N_out] complex (Sec. III forward)."""
        torch = self._torch()
        x = self._check_signal(x)
        lead = x.shape[:-1]
        batch = int(np.prod(lead)) if len(lead) else 1
        y = self._out(out, tuple(lead) + (self.R, self.N_out), self._complex_dtype(), x.device)
        self._call(lib.qtam_forward, "qtam_forward", x, y, batch, ws, stream)
        return y

    def forward_noalloc(self, x, out=None, stream=None):
        """forward() through qtam_forward_noalloc: the library's static device
        workspace instead of a caller workspace (the call itself allocates
        nothing; pass `out` to allocate nothing here either)."""
        torch = self._torch()
        x = self._check_signal(x)
        lead = x.shape[:-1]
        batch = int(np.prod(lead)) if len(lead) else 1
        y = self._out(out, tuple(lead) + (self.R, self.N_out), self._complex_dtype(), x.device)
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        _check(lib.qtam_forward_noalloc(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                        int(batch), ctypes.c_void_p(stream.cuda_stream)), "qtam_forward_noalloc")
        return y

    def _check_row_params(self, t, what, device):
        torch = self._torch()
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.device == device):
            raise TypeError("%s: expected a CUDA (HIP) tensor on %s" % (what, device))
        if t.dtype != self._real_dtype() or tuple(t.shape) != (self.R,):
            raise ValueError("%s: expected real %s [%d], got %s %s" % (what, self._real_dtype(), self.R, t.dtype,
                                                                     tuple(t.shape)))
        return t.contiguous()

    def mask_forward(self, y, gain, thresholds, out=None, stream=None):
        """gain[k] * max(0, 1 - thresholds[k] / |y|) * y on envelopes
        [..., R, N_out] (qtam_mask_forward)."""
        torch = self._torch()
        y = self._check_rows(y)
        gain = self._check_row_params(gain, "gain", y.device)
        thresholds = self._check_row_params(thresholds, "thresholds", y.device)
        lead = y.shape[:-2]
        batch = int(np.prod(lead)) if len(lead) else 1
        o = self._out(out, tuple(y.shape), self._complex_dtype(), y.device)
        if stream is None:
            stream = torch.cuda.current_stream(y.device)
        _check(lib.qtam_mask_forward(self._h, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(gain.data_ptr()),
                                     ctypes.c_void_p(thresholds.data_ptr()), ctypes.c_void_p(o.data_ptr()),
                                     int(batch), ctypes.c_void_p(stream.cuda_stream)), "qtam_mask_forward")
        return o

    def mask_backward(self, y, gain, thresholds, gout, stream=None):
        """(dL/dy, dL/dgain) of mask_forward given gout = dL/dout
        (qtam_mask_backward)."""
        torch = self._torch()
        y = self._check_rows(y)
        gout = self._check_rows(gout)
        if gout.shape != y.shape or gout.device != y.device:
            raise ValueError("gout must match y: %s vs %s" % (tuple(gout.shape), tuple(y.shape)))
        gain = self._check_row_params(gain, "gain", y.device)
        thresholds = self._check_row_params(thresholds, "thresholds", y.device)
        lead = y.shape[:-2]
        batch = int(np.prod(lead)) if len(lead) else 1
        gy = torch.empty_like(y)
        dgain = torch.empty(self.R, dtype=self._real_dtype(), device=y.device)
        wsb = max(int(lib.qtam_mask_workspace_size(self._h, int(batch))), 1)
        ws = torch.empty(wsb, dtype=torch.uint8, device=y.device)
        if stream is None:
            stream = torch.cuda.current_stream(y.device)
        _check(lib.qtam_mask_backward(self._h, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(gain.data_ptr()),
                                      ctypes.c_void_p(thresholds.data_ptr()), ctypes.c_void_p(gout.data_ptr()),
                                      ctypes.c_void_p(gy.data_ptr()), ctypes.c_void_p(dgain.data_ptr()),
                                      int(batch), ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(wsb),
                                      ctypes.c_void_p(stream.cuda_stream)), "qtam_mask_backward")
        return gy, dgain

    @property
    def masked_inverse_supported(self) -> bool:
        """Whether inverse_masked / inverse_masked_adjoint run on this plan
        (rows transformed in one workgroup); asks the library with an empty
        batch."""
        ok = getattr(self, "_masked_ok", None)
        if ok is None:
            st = lib.qtam_inverse_masked(self._h, None, None, None, None, 0, None, 0, None)
            if st not in (QTAM_OK, QTAM_ERR_UNSUPPORTED):
                _check(st, "qtam_inverse_masked")
            ok = self._masked_ok = st == QTAM_OK
        return ok

    def inverse_masked(self, y, gain, thresholds, out=None, ws=None, stream=None):
        """inverse(mask_forward(y, gain, thresholds)) in one pass over y: the
        mask is applied as the inverse rows kernel loads the envelopes
        (qtam_inverse_masked)."""
        torch = self._torch()
        y = self._check_rows(y)
        gain = self._check_row_params(gain, "gain", y.device)
        thresholds = self._check_row_params(thresholds, "thresholds", y.device)
        lead = y.shape[:-2]
        batch = int(np.prod(lead)) if len(lead) else 1
        x = self._out(out, tuple(lead) + (self.N,), self._real_dtype(), y.device)
        if stream is None:
            stream = torch.cuda.current_stream(y.device)
        ws = self._workspace(batch, y.device, ws)
        _check(lib.qtam_inverse_masked(self._h, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(gain.data_ptr()),
                                       ctypes.c_void_p(thresholds.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                       int(batch), ctypes.c_void_p(ws.data_ptr()),
                                       ctypes.c_size_t(ws.numel() * ws.element_size()),
                                       ctypes.c_void_p(stream.cuda_stream)), "qtam_inverse_masked")
        return x

    def inverse_masked_adjoint(self, gx, y, gain, thresholds, ws=None, stream=None):
        """(dL/dy, dL/dgain) of inverse_masked given gx = dL/dx
        (qtam_inverse_masked_adjoint)."""
        torch = self._torch()
        gx = self._check_signal(gx)
        y = self._check_rows(y)
        if tuple(gx.shape[:-1]) != tuple(y.shape[:-2]) or gx.device != y.device:
            raise ValueError("gx %s does not match y %s" % (tuple(gx.shape), tuple(y.shape)))
        gain = self._check_row_params(gain, "gain", y.device)
        thresholds = self._check_row_params(thresholds, "thresholds", y.device)
        lead = y.shape[:-2]
        batch = int(np.prod(lead)) if len(lead) else 1
        gy = torch.empty_like(y)
        dgain = torch.empty(self.R, dtype=self._real_dtype(), device=y.device)
        if stream is None:
            stream = torch.cuda.current_stream(y.device)
        if ws is not None:
            ws = expect_workspace(ws, y.device)
        else:
            need = max(int(lib.qtam_masked_adjoint_workspace_size(self._h, int(batch))), 1)
            if self._ws is None or self._ws.numel() < need or self._ws.device != y.device:
                self._ws = torch.empty(need, dtype=torch.uint8, device=y.device)
            ws = self._ws
        _check(lib.qtam_inverse_masked_adjoint(self._h, ctypes.c_void_p(gx.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                               ctypes.c_void_p(gain.data_ptr()),
                                               ctypes.c_void_p(thresholds.data_ptr()),
                                               ctypes.c_void_p(gy.data_ptr()), ctypes.c_void_p(dgain.data_ptr()),
                                               int(batch), ctypes.c_void_p(ws.data_ptr()),
                                               ctypes.c_size_t(ws.numel() * ws.element_size()),
                                               ctypes.c_void_p(stream.cuda_stream)), "qtam_inverse_masked_adjoint")
        return gy, dgain

    def forward_metric(self, x, out=None, metric=None, ws=None, stream=None):
        """Forward plus per-row statistics: (Y, metric) with metric [..., R]
        complex holding (sum_m |Y_k[m]|^2, max_m |Y_k[m]|^2) of each row."""
        torch = self._torch()
        x = self._check_signal(x)
        lead = x.shape[:-1]
        batch = int(np.prod(lead)) if len(lead) else 1
        y = self._out(out, tuple(lead) + (self.R, self.N_out), self._complex_dtype(), x.device)
        m = self._out(metric, tuple(lead) + (self.R,), self._complex_dtype(), x.device, "metric")
        if stream is None:
            stream = torch.cuda.current_stream(x.device)
        ws = self._workspace(batch, x.device, ws)
        _check(lib.qtam_forward_metric(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       ctypes.c_void_p(m.data_ptr()), int(batch),
                                       ctypes.c_void_p(ws.data_ptr()),
                                       ctypes.c_size_t(ws.numel() * ws.element_size()),
                                       ctypes.c_void_p(stream.cuda_stream)), "qtam_forward_metric")
        return y, m

    def tile_inverse(self, y, row, out=None, ws=None, stream=None):
        """The signal [..., N] from row `row` alone of envelopes [..., R, N_out]
        by spectral division (plans with window_eps > 0)."""
        torch = self._torch()
        y = self._check_rows(y)
        lead = y.shape[:-2]
        batch = int(np.prod(lead)) if len(lead) else 1
        x = self._out(out, tuple(lead) + (self.N,), self._real_dtype(), y.device)
        if stream is None:
            stream = torch.cuda.current_stream(y.device)
        ws = self._workspace(batch, y.device, ws)
        _check(lib.qtam_tile_inverse(self._h, ctypes.c_void_p(y.data_ptr()), int(row), ctypes.c_void_p(x.data_ptr()),
                                     int(batch), ctypes.c_void_p(ws.data_ptr()),
                                     ctypes.c_size_t(ws.numel() * ws.element_size()),
                                     ctypes.c_void_p(stream.cuda_stream)), "qtam_tile_inverse")
        return x

    def dense(self, y, out=None, ws=None, stream=None):
        """Dense full-rate tiles [..., R, N] complex from envelopes [..., R, N_out]
        (each row re-modulated and up-sampled to N samples, App. C)."""
        torch = self._torch()
        y = self._check_rows(y)
        lead = y.shape[:-2]
        batch = int(np.prod(lead)) if len(lead) else 1
        d = self._out(out, tuple(lead) + (self.R, self.N), self._complex_dtype(), y.device)
        if batch == 0:
            return d
        need = int(lib.qtam_dense_workspace_size(self._h, batch))
        if need == 0:
            raise QtamError(QTAM_ERR_UNSUPPORTED, "qtam_dense")
        if ws is None:
            ws = torch.empty(need, dtype=torch.uint8, device=y.device)
        else:
            expect_workspace(ws, y.device)
        if stream is None:
            stream = torch.cuda.current_stream(y.device)
        _check(lib.qtam_dense(self._h, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(d.data_ptr()), int(batch),
                              ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * ws.element_size()),
                              ctypes.c_void_p(stream.cuda_stream)), "qtam_dense")
        return d

    def select_planes(self, y, metric, kind="energy", stream=None):
        """Optimal plane per segment: (score [..., planes], best [...] int32,
        y_best [..., rows_per_plane, N_out])."""
        torch = self._torch()
        y = self._check_rows(y)
        lead = y.shape[:-2]
        batch = int(np.prod(lead)) if len(lead) else 1
        if metric.dtype != self._complex_dtype() or tuple(metric.shape) != tuple(lead) + (self.R,):
            raise ValueError("metric must be complex [..., R] as forward_metric returns it")
        metric = metric.contiguous()
        score = torch.empty(tuple(lead) + (self.planes,), dtype=self._real_dtype(), device=y.device)
        best = torch.empty(tuple(lead), dtype=torch.int32, device=y.device)
        yb = torch.empty(tuple(lead) + (self.rows_per_plane, self.N_out), dtype=self._complex_dtype(),
                         device=y.device)
        if stream is None:
            stream = torch.cuda.current_stream(y.device)
        k = METRIC[kind] if isinstance(kind, str) else int(kind)
        _check(lib.qtam_select_planes(self._h, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(metric.data_ptr()),
                                      k, ctypes.c_void_p(score.data_ptr()), ctypes.c_void_p(best.data_ptr()),
                                      ctypes.c_void_p(yb.data_ptr()), int(batch),
                                      ctypes.c_void_p(stream.cuda_stream)), "qtam_select_planes")
        return score, best, yb

    def inverse(self, y, out=None, ws=None, stream=None):
        """Y [..., R, N_out] complex -> x [..., N] real (canonical dual frame)."""
        torch = self._torch()
        y = self._check_rows(y)
        lead = y.shape[:-2]
        batch = int(np.prod(lead)) if len(lead) else 1
        x = self._out(out, tuple(lead) + (self.N,), self._real_dtype(), y.device)
        self._call(lib.qtam_inverse, "qtam_inverse", y, x, batch, ws, stream)
        return x

    def forward_adjoint(self, gy, out=None, ws=None, stream=None):
        torch = self._torch()
        gy = self._check_rows(gy)
        lead = gy.shape[:-2]
        batch = int(np.prod(lead)) if len(lead) else 1
        gx = self._out(out, tuple(lead) + (self.N,), self._real_dtype(), gy.device)
        self._call(lib.qtam_forward_adjoint, "qtam_forward_adjoint", gy, gx, batch, ws, stream)
        return gx

    def inverse_adjoint(self, gx, out=None, ws=None, stream=None):
        torch = self._torch()
        gx = self._check_signal(gx)
        lead = gx.shape[:-1]
        batch = int(np.prod(lead)) if len(lead) else 1
        gy = self._out(out, tuple(lead) + (self.R, self.N_out), self._complex_dtype(), gx.device)
        self._call(lib.qtam_inverse_adjoint, "qtam_inverse_adjoint", gx, gy, batch, ws, stream)
        return gy

    # ---------------------------------------------------------------- timing
    def timing(self, on: bool):
        _check(lib.qtam_timing_enable(self._h, 1 if on else 0), "qtam_timing_enable")

    def timing_collect(self) -> dict:
        n = 32
        names = (ctypes.c_char_p * n)()
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        got = ctypes.c_int32()
        _check(lib.qtam_timing_collect(self._h, names, ms, cnt, n, ctypes.byref(got)), "qtam_timing_collect")
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(min(n, got.value))}


def forward_sweep(plans, x, outs=None, ws=None, stream=None):
    """Forward transform of x [..., N] under every plan in `plans` (same N and
    precision), with the spectrum of each segment computed once for all of
    them (multi-Q extension, App. A). Returns one Y [..., R_i, N_out_i] per
    plan, identical to ``plans[i].forward(x)``."""
    import torch
    plans = list(plans)
    if not plans:
        raise ValueError("forward_sweep needs at least one plan")
    x = plans[0]._check_signal(x)
    lead = x.shape[:-1]
    batch = int(np.prod(lead)) if len(lead) else 1
    if outs is None:
        outs = [torch.empty(tuple(lead) + (p.R, p.N_out), dtype=p._complex_dtype(), device=x.device)
                for p in plans]
    outs = list(outs)
    if len(outs) != len(plans):
        raise ValueError("one output per plan")
    for i, (p, y) in enumerate(zip(plans, outs)):
        expect_tensor(y, tuple(lead) + (p.R, p.N_out), p._complex_dtype(), x.device, "output %d" % i)
    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    if ws is None:
        need = max(p.workspace_bytes(batch) for p in plans)
        ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    else:
        expect_workspace(ws, x.device)
    n = len(plans)
    hs = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
    ys = (ctypes.c_void_p * n)(*[y.data_ptr() for y in outs])
    _check(lib.qtam_forward_sweep(hs, n, ctypes.c_void_p(x.data_ptr()), ys, int(batch),
                                  ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * ws.element_size()),
                                  ctypes.c_void_p(stream.cuda_stream)), "qtam_forward_sweep")
    return outs
