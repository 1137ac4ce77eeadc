"""ctypes wrapper of the FP64 CPU oracle (qtam_oracle.cpp).

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it to check the GPU library. Nothing on the product path
imports this module, and it imports nothing from the product package.

Arrays are numpy float64 / complex128. Envelopes are ``[batch, R, N_out]``
complex, signals ``[batch, N]`` real, spectra ``[batch, N/2+1]`` complex.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qtam_oracle.cpp")
_LIB = os.environ.get("QTAM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

CAP_COVER, CAP_PAPER, CAP_NONE, CAP_MANUAL = 0, 1, 2, 3
NORM_UNIT_ENERGY, NORM_PAPER_INV_ENERGY, NORM_NONE = 0, 1, 2
WIN_BISQUARE, WIN_HANN, WIN_KAISER, WIN_TUKEY, WIN_PLANCK = 0, 1, 2, 3, 4


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain -O2, no fast-math)."""
    if os.environ.get("QTAM_ORACLE_LIB"):
        return _LIB          # a prebuilt variant (the mutation test builds its own)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.ora_plan_create.restype = ctypes.c_void_p
        L.ora_plan_create.argtypes = [ctypes.c_double, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int32, dp,
                                      ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_double, ctypes.c_int32, dp,
                                      ctypes.POINTER(ctypes.c_int32), dp, ctypes.c_double]
        L.ora_plan_destroy.argtypes = [ctypes.c_void_p]
        L.ora_plan_sizes.argtypes = [ctypes.c_void_p, i64p]
        L.ora_plan_rows.argtypes = [ctypes.c_void_p, dp, i64p, i64p, i64p, i64p]
        L.ora_plan_windows.argtypes = [ctypes.c_void_p, dp]
        L.ora_plan_frame.argtypes = [ctypes.c_void_p, dp, ctypes.POINTER(ctypes.c_ubyte)]
        L.ora_set_force_direct.argtypes = [ctypes.c_int32]
        L.ora_dft.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_int32]
        for name in ("ora_spectrum", "ora_forward", "ora_inverse", "ora_synthesis"):
            getattr(L, name).argtypes = [ctypes.c_void_p, dp, ctypes.c_int64, dp]
        L.ora_forward_rows.argtypes = [ctypes.c_void_p, dp, ctypes.c_int64, i64p, ctypes.c_int64, dp]
        L.ora_forward_rows.restype = ctypes.c_int
        L.ora_dense.argtypes = [ctypes.c_void_p, dp, dp]
        L.ora_tile_inverse.argtypes = [ctypes.c_void_p, dp, ctypes.c_int32, ctypes.c_int64, dp]
        L.ora_tile_inverse.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_force_direct(on: bool) -> None:
    """Use the direct O(n^2) DFT for every transform (tiny inputs only)."""
    lib().ora_set_force_direct(1 if on else 0)


def dft(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unnormalised complex DFT with kernel exp(sign * 2 pi i k n / N)."""
    a = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(a)
    lib().ora_dft(a.size, _dp(a.view(np.float64)), _dp(out.view(np.float64)), int(sign))
    return out


@dataclass
class OraclePlan:
    fs: float
    n: int
    q: float
    f_min: float
    f_max: float
    rows: int
    freqs: np.ndarray | None = None
    window: int = WIN_BISQUARE
    window_param: float = 0.0
    cap_mode: int = CAP_COVER
    max_window: int = 0
    norm_mode: int = NORM_UNIT_ENERGY
    n_out: int = 0
    p_floor_rel: float = 1e-6
    planes: list | None = None     # [(q, window, param), ...]: composite bank, plane after plane
    eps: float = 0.0               # stop-band value of every window (> 0: windows cover the whole band)

    def __post_init__(self):
        L = lib()
        fr = None
        if self.freqs is not None:
            self._freqs = np.ascontiguousarray(self.freqs, dtype=np.float64)
            fr = _dp(self._freqs)
            self.rows = int(self._freqs.size)
        npl, qs, ws, ps = 0, None, None, None
        if self.planes:
            npl = len(self.planes)
            self._qs = np.array([p[0] for p in self.planes], dtype=np.float64)
            self._ws = np.array([p[1] for p in self.planes], dtype=np.int32)
            self._ps = np.array([p[2] for p in self.planes], dtype=np.float64)
            qs, ps = _dp(self._qs), _dp(self._ps)
            ws = self._ws.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        self.n_planes = max(npl, 1)
        self.rows_per_plane = int(self.rows)
        h = L.ora_plan_create(float(self.fs), int(self.n), float(self.q), float(self.f_min),
                              float(self.f_max), int(self.rows), fr, int(self.window),
                              float(self.window_param), int(self.cap_mode), int(self.max_window),
                              int(self.norm_mode), int(self.n_out), float(self.p_floor_rel),
                              int(npl), qs, ws, ps, float(self.eps))
        if not h:
            raise ValueError("oracle rejected the plan parameters")
        self._h = ctypes.c_void_p(h)
        sz = np.zeros(6, dtype=np.int64)
        L.ora_plan_sizes(self._h, sz.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        self.R, self.N_out, self.n_bins, self.l_max, self.max_len, self.sum_len = (int(v) for v in sz)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.ora_plan_destroy(h)
            self._h = None

    # -- tables -------------------------------------------------------------
    def row_table(self):
        R = self.R
        f = np.zeros(R)
        s, hw, lo, hi = (np.zeros(R, dtype=np.int64) for _ in range(4))
        i64 = ctypes.POINTER(ctypes.c_int64)
        lib().ora_plan_rows(self._h, _dp(f), s.ctypes.data_as(i64), hw.ctypes.data_as(i64),
                            lo.ctypes.data_as(i64), hi.ctypes.data_as(i64))
        return dict(freq=f, centre=s, half=hw, lo=lo, hi=hi)

    def windows(self) -> np.ndarray:
        W = np.zeros((self.R, self.n_bins))
        lib().ora_plan_windows(self._h, _dp(W))
        return W

    def frame(self):
        P = np.zeros(self.n_bins)
        M = np.zeros(self.n_bins, dtype=np.uint8)
        lib().ora_plan_frame(self._h, _dp(P), M.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
        return P, M.astype(bool)

    # -- transforms ---------------------------------------------------------
    def _signal(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        return x.reshape(-1, self.n), x.ndim == 1

    def spectrum(self, x):
        x2, one = self._signal(x)
        X = np.zeros((x2.shape[0], self.n_bins), dtype=np.complex128)
        lib().ora_spectrum(self._h, _dp(x2), x2.shape[0], _dp(X.view(np.float64)))
        return X[0] if one else X

    def forward(self, x):
        x2, one = self._signal(x)
        Y = np.zeros((x2.shape[0], self.R, self.N_out), dtype=np.complex128)
        lib().ora_forward(self._h, _dp(x2), x2.shape[0], _dp(Y.view(np.float64)))
        return Y[0] if one else Y

    def forward_rows(self, x, rows):
        """Coefficients of the given rows only, shape [batch, len(rows), N_out]
        (or [len(rows), N_out] for one segment)."""
        x2, one = self._signal(x)
        idx = np.ascontiguousarray(rows, dtype=np.int64)
        Y = np.zeros((x2.shape[0], idx.size, self.N_out), dtype=np.complex128)
        if lib().ora_forward_rows(self._h, _dp(x2), x2.shape[0], idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  idx.size, _dp(Y.view(np.float64))) != 0:
            raise IndexError("row index out of range")
        return Y[0] if one else Y

    def inverse(self, Y):
        Y = np.ascontiguousarray(Y, dtype=np.complex128)
        one = Y.ndim == 2
        Y3 = Y.reshape(-1, self.R, self.N_out)
        x = np.zeros((Y3.shape[0], self.n))
        lib().ora_inverse(self._h, _dp(Y3.view(np.float64)), Y3.shape[0], _dp(x))
        return x[0] if one else x

    def synthesis(self, Xh):
        Xh = np.ascontiguousarray(Xh, dtype=np.complex128)
        one = Xh.ndim == 1
        X2 = Xh.reshape(-1, self.n_bins)
        x = np.zeros((X2.shape[0], self.n))
        lib().ora_synthesis(self._h, _dp(X2.view(np.float64)), X2.shape[0], _dp(x))
        return x[0] if one else x

    def dense(self, x):
        """Dense full-rate tiles T_k[tau], shape [R, N], of one segment."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(self.n)
        T = np.zeros((self.R, self.n), dtype=np.complex128)
        lib().ora_dense(self._h, _dp(x), _dp(T.view(np.float64)))
        return T

    def tile_inverse(self, Y, k):
        """The signal from row k alone by spectral division (regularised
        windows): Y [batch, R, N_out] -> x [batch, N]."""
        Y = np.ascontiguousarray(Y, dtype=np.complex128)
        batch = Y.shape[0] if Y.ndim == 3 else 1
        x = np.zeros((batch, self.n))
        if lib().ora_tile_inverse(self._h, _dp(Y.view(np.float64)), int(k), batch, _dp(x)) != 0:
            raise ValueError("tile inverse needs a window that is non-zero on its kept bins")
        return x if Y.ndim == 3 else x[0]

    def project(self, x):
        """x_M = irfft(M * rfft(x)): what exact reconstruction returns."""
        _, M = self.frame()
        X = self.spectrum(x)
        return self.synthesis(X * M)

    # ------------------------------------------------------- composite banks
    # Multi-Q / multi-window extension (App. A): the bank's planes are
    # consecutive blocks of rows_per_plane rows; each plane is scored by a
    # quality metric, and the optimal-selection mode keeps, for every
    # segment on its own, the plane with the best score.

    def row_stats(self, Y):
        """(energy, peak) per row: sum and max over m of |Y_k[m]|^2."""
        a = np.abs(np.asarray(Y, dtype=np.complex128)) ** 2
        return a.sum(axis=-1), a.max(axis=-1)

    def plane_scores(self, Y, kind: str = "energy"):
        """Score of each plane, shape [..., n_planes]."""
        energy, peak = self.row_stats(Y)
        per = (energy if kind == "energy" else peak)
        per = per.reshape(per.shape[:-1] + (self.n_planes, self.rows_per_plane))
        return per.sum(axis=-1) if kind == "energy" else per.max(axis=-1)

    def select_planes(self, Y, kind: str = "energy"):
        """(score, best, Y_best): the first plane with the largest score."""
        Y = np.asarray(Y)
        score = self.plane_scores(Y, kind)
        best = np.argmax(score, axis=-1)
        Yp = Y.reshape(Y.shape[:-2] + (self.n_planes, self.rows_per_plane, Y.shape[-1]))
        Yb = np.take_along_axis(Yp, best[..., None, None, None], axis=-3)[..., 0, :, :]
        return score, best, Yb
