"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

None of these re-type the oracle's own formulas: each compares it with a
library routine (numpy / scipy), an exact rational evaluation of a printed
formula, a closed form, a brute-force matrix identity, or an invariant the
paper states (Sec. III; App. A; App. C). A plausible slip in the oracle (wrong
DFT sign, dropped sqrt(N_out/N), off-by-one centre or width, missing 1/P, a
transposed index in the roll) breaks at least one of them.
"""
from fractions import Fraction
import json
import math
import os

import numpy as np
import pytest
import scipy.signal
import scipy.special

from oracle import oracle as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# --------------------------------------------------------------------------
# DFT / spectrum / synthesis against numpy (a textbook library), and the
# radix-2 path against the direct O(n^2) sum.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 12, 16, 64, 100, 256, 1024, 4096, 24576, 20480, 997])
def test_dft_matches_numpy(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert rel(o.dft(x, -1), np.fft.fft(x)) < 1e-13
    assert rel(o.dft(x, +1), np.fft.ifft(x) * n) < 1e-13


@pytest.mark.parametrize("n", [16, 128, 512, 12, 96, 105, 1155, 3 * 1024, 2 * 997])
def test_fast_paths_match_direct(n):
    """Radix-2 (powers of two) and the smallest-prime-factor split (other
    composite lengths) against the direct O(n^2) sum."""
    rng = np.random.default_rng(7 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    fast = o.dft(x, -1)
    o.set_force_direct(True)
    try:
        slow = o.dft(x, -1)
    finally:
        o.set_force_direct(False)
    assert rel(fast, slow) < 1e-13


def test_spectrum_and_synthesis_match_numpy():
    p = o.OraclePlan(fs=512.0, n=1024, q=4.0, f_min=10.0, f_max=200.0, rows=8)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 1024))
    assert rel(p.spectrum(x), np.fft.rfft(x, axis=-1)) < 1e-13
    # irfft convention: imaginary parts of DC and Nyquist are ignored
    Xh = rng.standard_normal((3, 513)) + 1j * rng.standard_normal((3, 513))
    assert rel(p.synthesis(Xh), np.fft.irfft(Xh, n=1024, axis=-1)) < 1e-13


# --------------------------------------------------------------------------
# Windows: exact rational evaluation of the printed bisquare formula (Sec. II
# window equation) and library special cases of the other shapes (App. A).
# --------------------------------------------------------------------------
def _single_row(window=o.WIN_BISQUARE, param=0.0, norm=o.NORM_UNIT_ENERGY, q=2.0):
    # T = 1 s, f = 16 Hz -> centre bin 16; Q = 2 -> full width 8 bins -> h = 4
    return o.OraclePlan(fs=64.0, n=64, q=q, f_min=16.0, f_max=16.0, rows=1,
                        freqs=np.array([16.0]), window=window, window_param=param,
                        cap_mode=o.CAP_NONE, norm_mode=norm)


def test_bisquare_exact_rational():
    p = _single_row()
    t = p.row_table()
    assert t["centre"][0] == 16 and t["half"][0] == 4
    W = p.windows()[0]
    h = 4
    shape = {j: (1 - Fraction(j * j, h * h)) ** 2 for j in range(-h, h + 1)}
    energy = sum(v * v for v in shape.values())
    assert energy == Fraction(213060, 65536)
    for j, v in shape.items():
        assert W[16 + j] == pytest.approx(float(v) / math.sqrt(float(energy)), rel=1e-15, abs=1e-300)
    assert np.count_nonzero(W) == 7          # the two edge bins are exact zeros
    assert np.sum(W ** 2) == pytest.approx(1.0, rel=1e-15)
    # literal printed normalisation C = 1 / sum W'^2
    Wp = _single_row(norm=o.NORM_PAPER_INV_ENERGY).windows()[0]
    assert Wp[16] == pytest.approx(float(1 / energy), rel=1e-15)
    Wn = _single_row(norm=o.NORM_NONE).windows()[0]
    assert Wn[17] == pytest.approx(float(shape[1]), rel=1e-15)


@pytest.mark.parametrize("kind,param,ref", [
    (o.WIN_HANN, 0.0, lambda m, a: scipy.signal.windows.hann(m, sym=True)),
    (o.WIN_KAISER, 6.0, lambda m, a: scipy.signal.windows.kaiser(m, a, sym=True)),
    (o.WIN_TUKEY, 0.5, lambda m, a: scipy.signal.windows.tukey(m, a, sym=True)),
    (o.WIN_TUKEY, 0.25, lambda m, a: scipy.signal.windows.tukey(m, a, sym=True)),
])
def test_window_family_matches_scipy(kind, param, ref):
    W = _single_row(window=kind, param=param, norm=o.NORM_NONE).windows()[0]
    expect = ref(9, param)
    assert np.allclose(W[12:21], expect, rtol=1e-13, atol=1e-15)


def test_planck_taper_points():
    # h = 4, alpha = 0.5: taper on 2 <= |j| <= 4; u = (1-|x|)/alpha
    W = _single_row(window=o.WIN_PLANCK, param=0.5, norm=o.NORM_NONE).windows()[0]
    assert W[16] == 1.0 and W[17] == 1.0 and W[18] == 1.0     # |x| <= 1 - alpha
    assert W[20] == 0.0 and W[12] == 0.0                       # edge
    assert W[19] == pytest.approx(0.5, abs=1e-15)             # u = 1/2 -> z = 0
    # 1/(e^z+1) with z(1-u) = -z(u): finer grid, W(u) + W(1-u) = 1
    p = o.OraclePlan(fs=256.0, n=256, q=1.0, f_min=64.0, f_max=64.0, rows=1,
                     freqs=np.array([64.0]), window=o.WIN_PLANCK, window_param=0.5,
                     cap_mode=o.CAP_NONE, norm_mode=o.NORM_NONE)
    h = int(p.row_table()["half"][0])
    assert h == 32
    Wf = p.windows()[0]
    s = 64
    # |x| = 1 - alpha*u ; u and 1-u map to offsets j and j' with j + j' = h*(2-alpha) = 1.5h
    for j in range(h // 2 + 1, h):
        jp = int(round(1.5 * h)) - j
        if h // 2 < jp < h:
            assert Wf[s + j] + Wf[s + jp] == pytest.approx(1.0, abs=1e-14)


# --------------------------------------------------------------------------
# Grid, cap and sizes (App. A formulas; Sec. III minimal length).
# --------------------------------------------------------------------------
def test_cap_and_width_integers():
    # T = 1 s, rows at 100 and 200 Hz: largest gap 100 Hz -> g = 100 bins.
    kw = dict(fs=1024.0, n=1024, q=1.0, f_min=100.0, f_max=200.0, rows=2)
    cover = o.OraclePlan(cap_mode=o.CAP_COVER, **kw)
    paper = o.OraclePlan(cap_mode=o.CAP_PAPER, **kw)
    none = o.OraclePlan(cap_mode=o.CAP_NONE, **kw)
    assert cover.l_max == 201 and paper.l_max == 101 and none.l_max == -1
    assert list(cover.row_table()["half"]) == [50, 100]
    assert list(paper.row_table()["half"]) == [50, 50]
    assert list(cover.row_table()["centre"]) == [100, 200]
    assert cover.N_out == 256 and paper.N_out == 128
    # the paper's minimal length n = ceil(N_t df_max) + 1 holds the clamped supports
    n_min = math.ceil(1.0 * 100.0) + 1
    assert paper.max_len <= n_min
    assert o.OraclePlan(cap_mode=o.CAP_PAPER, n_out=n_min, **kw).N_out == n_min
    with pytest.raises(ValueError):
        o.OraclePlan(cap_mode=o.CAP_COVER, n_out=200, **kw)
    man = o.OraclePlan(cap_mode=o.CAP_MANUAL, max_window=41, **kw)
    assert list(man.row_table()["half"]) == [20, 20]


def test_geometric_grid_and_floor():
    p = o.OraclePlan(fs=4096.0, n=16384, q=8.0, f_min=20.0, f_max=1000.0, rows=64)
    f = p.row_table()["freq"]
    assert f[0] == 20.0 and f[-1] == pytest.approx(1000.0, rel=1e-15)
    ratio = f[1:] / f[:-1]
    assert np.allclose(ratio, (1000.0 / 20.0) ** (1.0 / 63.0), rtol=1e-14)
    t = p.row_table()
    # centre: nearest bin to f*T; T = 4 s
    assert np.all(np.abs(t["centre"] - f * 4.0) <= 0.5)
    # narrow low rows: the floor h >= 1 (Q = 32 at 5 Hz, T = 1 s: f*T/Q < 1)
    low = o.OraclePlan(fs=4096.0, n=4096, q=32.0, f_min=5.0, f_max=50.0, rows=4)
    assert low.row_table()["half"][0] == 1


def test_paper_printed_sizes():
    """Sizes the paper prints (App. B: 62 x 12289 standard and 62 x 669
    minimal outputs of 6 s segments at 4096 Hz; Sec. IV: a 64 x 410 dense
    tile of 0.2 s at 4096 Hz) against the oracle's own plans and outputs.

    * The standard width is the one-sided spectrum of the segment: the
      oracle's spectrum of a 24576-sample segment has 12289 bins, and a
      62-row plan has 62 rows.
    * The minimal width n = ceil(N_t df_max) + 1 (App. A) is lossless: under
      the printed cap the oracle's widest support fits in n, n itself is an
      accepted output length whose round trip returns the projection x_M to
      machine precision (P1), and an output shorter than the widest support
      is rejected. The paper gives no frequency range for its glitch tensor;
      the 10-2048 Hz band is a reading, so the printed 669 itself stays
      unpinned and only the formula is checked.
    * 0.2 s at 4096 Hz is 819.2 samples; with the even length 818 the
      oracle's one-sided spectrum has the printed 410 bins."""
    with open(os.path.join(GOLDEN, "paper_printed.json")) as fh:
        g = json.load(fh)
    std = g["standard_output_6s"]
    fs, n, rows = float(std["fs"]), int(std["n_samples"]), int(std["rows"])
    T = n / fs
    kw = dict(fs=fs, n=n, q=8.0, f_min=10.0, f_max=fs / 2, rows=rows)
    paper = o.OraclePlan(cap_mode=o.CAP_PAPER, **kw)
    rng = np.random.default_rng(17)
    x = rng.standard_normal(n)
    X = paper.spectrum(x)
    assert paper.R == rows and X.shape == (std["cols"],) and paper.n_bins == std["cols"]
    assert np.abs(X - np.fft.rfft(x)).max() <= 1e-9 * np.abs(X).max()
    f = paper.row_table()["freq"]
    gap = int(math.ceil(T * float(np.max(np.diff(f)))))
    n_min = gap + 1
    assert paper.l_max == 2 * (gap // 2) + 1
    assert paper.max_len <= n_min
    minimal = o.OraclePlan(cap_mode=o.CAP_PAPER, n_out=n_min, **kw)
    assert minimal.N_out == n_min
    Y = minimal.forward(x)
    assert Y.shape == (rows, n_min)
    xm = minimal.project(x)
    assert np.linalg.norm(minimal.inverse(Y) - xm) <= 1e-12 * np.linalg.norm(xm)
    with pytest.raises(ValueError):
        o.OraclePlan(cap_mode=o.CAP_PAPER, n_out=paper.max_len - 1, **kw)
    gw = g["gw150914_demo"]
    n_gw = int(gw["duration_s"] * gw["fs"]) // 2 * 2
    demo = o.OraclePlan(fs=float(gw["fs"]), n=n_gw, q=8.0, f_min=30.0, f_max=500.0, rows=gw["rows"])
    assert demo.n_bins == gw["cols_dense"] and demo.spectrum(rng.standard_normal(n_gw)).shape == (gw["cols_dense"],)
    assert demo.R == gw["rows"]


# --------------------------------------------------------------------------
# Invariants of Sec. III and App. C on tiny and config-1 sized plans.
# --------------------------------------------------------------------------
def small_plan(**kw):
    base = dict(fs=256.0, n=256, q=4.0, f_min=10.0, f_max=100.0, rows=6)
    base.update(kw)
    return o.OraclePlan(**base)


def test_remodulated_envelope_equals_dense_row():
    p = small_plan()
    rng = np.random.default_rng(11)
    x = rng.standard_normal(p.n)
    T = p.dense(x)               # plain definition, direct summation
    Y = p.forward(x)
    s = p.row_table()["centre"]
    N, M = p.n, p.N_out
    assert N % M == 0
    m = np.arange(M)
    for k in range(p.R):
        carrier = np.exp(2j * np.pi * s[k] * m / M)
        assert rel(T[k, m * (N // M)], math.sqrt(M / N) * carrier * Y[k]) < 1e-12
    # full-rate restoration of every sample: DFT_Nout, sqrt(N/N_out), re-place at s+j
    t = p.row_table()
    for k in range(p.R):
        Yt = np.fft.fft(Y[k]) * math.sqrt(N / M)
        F = np.zeros(N, dtype=complex)
        for c in range(t["lo"][k], t["hi"][k] + 1):
            F[c] = Yt[(c - s[k]) % M]
        assert rel(np.fft.ifft(F), T[k]) < 1e-12


def test_energy_per_row():
    p = small_plan(q=6.0, rows=5)
    x = np.random.default_rng(5).standard_normal(p.n)
    T = p.dense(x)
    Y = p.forward(x)
    eT = np.sum(np.abs(T) ** 2, axis=1)
    eY = np.sum(np.abs(Y) ** 2, axis=1)
    assert np.allclose(eY, eT, rtol=1e-13, atol=0)


def test_dense_row_flat_window_is_half_analytic_signal():
    # flat (Tukey alpha = 0) window on bins 1..N/2-1: centre 16, h = 15, N = 64
    p = o.OraclePlan(fs=64.0, n=64, q=16.0 / 30.5, f_min=16.0, f_max=16.0, rows=1,
                     freqs=np.array([16.0]), window=o.WIN_TUKEY, window_param=0.0,
                     cap_mode=o.CAP_NONE, norm_mode=o.NORM_NONE)
    assert p.row_table()["half"][0] == 15
    x = np.random.default_rng(2).standard_normal(64)
    z = scipy.signal.hilbert(x)
    X = np.fft.rfft(x)
    tau = np.arange(64)
    expect = 0.5 * (z - (X[0] + X[32] * (-1.0) ** tau) / 64)
    assert rel(p.dense(x)[0], expect) < 1e-13


def test_frame_operator_is_diagonal_in_fourier():
    """S = Re(A^H A) from dense tiles equals irfft(c P rfft(.)), c = 1/2 inside."""
    p = small_plan(n=32, fs=32.0, f_min=3.0, f_max=14.0, rows=4, q=2.0)
    N = p.n
    A = np.stack([p.dense(e).ravel() for e in np.eye(N)], axis=1)    # [R*N, N]
    S = np.real(A.conj().T @ A)
    P, _ = p.frame()
    c = np.full(N // 2 + 1, 0.5)
    c[0] = c[-1] = 1.0
    S_ref = np.stack([np.fft.irfft(c * P * np.fft.rfft(e), n=N) for e in np.eye(N)], axis=1)
    assert np.abs(S - S_ref).max() < 1e-13 * np.abs(S_ref).max()
    assert np.allclose(S, S.T, atol=1e-15)


def _matrices(p):
    N, R, M = p.n, p.R, p.N_out
    F = np.stack([p.forward(e).ravel() for e in np.eye(N)], axis=1)        # [R*M, N] complex
    Freal = np.concatenate([F.real, F.imag], axis=0)                        # [2RM, N]
    cols = []
    for i in range(R * M):
        y = np.zeros(R * M, dtype=complex)
        y[i] = 1.0
        cols.append(p.inverse(y.reshape(R, M)))
    Gre = np.stack(cols, axis=1)
    cols = []
    for i in range(R * M):
        y = np.zeros(R * M, dtype=complex)
        y[i] = 1.0j
        cols.append(p.inverse(y.reshape(R, M)))
    Gim = np.stack(cols, axis=1)
    G = np.concatenate([Gre, Gim], axis=1)                                  # [N, 2RM]
    return Freal, G


def test_inverse_is_canonical_dual_pseudoinverse():
    # windows wide enough that every bin 0..N/2 is covered (P > 0 everywhere)
    p = o.OraclePlan(fs=32.0, n=32, q=0.25, f_min=2.0, f_max=16.0, rows=5,
                     freqs=np.array([2.0, 5.0, 9.0, 13.0, 16.0]), cap_mode=o.CAP_NONE,
                     p_floor_rel=0.0)
    P, Mk = p.frame()
    assert Mk.all()
    F, G = _matrices(p)
    assert np.abs(G @ F - np.eye(p.n)).max() < 1e-12
    assert np.abs(G - np.linalg.pinv(F)).max() < 1e-10 * np.abs(G).max()


def test_inverse_projects_onto_mask():
    p = small_plan(n=64, fs=64.0, f_min=6.0, f_max=20.0, rows=4, q=3.0)
    _, Mk = p.frame()
    assert not Mk.all()
    F, G = _matrices(p)
    Pi = G @ F
    Pi_ref = np.stack([np.fft.irfft(Mk * np.fft.rfft(e), n=p.n) for e in np.eye(p.n)], axis=1)
    assert np.abs(Pi - Pi_ref).max() < 1e-12
    assert np.abs(Pi @ Pi - Pi).max() < 1e-12
    assert np.abs(Pi - Pi.T).max() < 1e-12


@pytest.mark.parametrize("kw", [
    dict(fs=4096.0, n=16384, q=8.0, f_min=20.0, f_max=1000.0, rows=64),             # config-1 plan
    dict(fs=4096.0, n=16384, q=8.0, f_min=20.0, f_max=1000.0, rows=64, cap_mode=o.CAP_PAPER),
    dict(fs=1024.0, n=4096, q=4.0, f_min=10.0, f_max=512.0, rows=48),               # band to Nyquist
    dict(fs=1024.0, n=4096, q=16.0, f_min=10.0, f_max=500.0, rows=40, n_out=301),   # non-pow2 N_out
])
def test_exact_reconstruction(kw):
    p = o.OraclePlan(**kw)
    rng = np.random.default_rng(17)
    x = rng.standard_normal((2, p.n))
    xm = p.project(x)
    assert rel(p.inverse(p.forward(x)), xm) < 1e-12
    # band-limited to the mask: reconstruction is the identity
    assert rel(p.inverse(p.forward(xm)), xm) < 1e-12


def test_linearity():
    p = small_plan(n=512, fs=512.0, rows=9)
    rng = np.random.default_rng(23)
    x1, x2 = rng.standard_normal((2, p.n))
    a, b = 1.7, -0.3
    assert rel(p.forward(a * x1 + b * x2), a * p.forward(x1) + b * p.forward(x2)) < 1e-13
    Y1 = rng.standard_normal((p.R, p.N_out)) + 1j * rng.standard_normal((p.R, p.N_out))
    Y2 = rng.standard_normal((p.R, p.N_out)) + 1j * rng.standard_normal((p.R, p.N_out))
    assert rel(p.inverse(a * Y1 + b * Y2), a * p.inverse(Y1) + b * p.inverse(Y2)) < 1e-13


def test_shift_covariance():
    p = small_plan(n=512, fs=512.0, rows=7)
    N, M = p.n, p.N_out
    x = np.random.default_rng(29).standard_normal(N)
    s = p.row_table()["centre"]
    # dense tiles: integer shift d moves every tile by d
    d = 37
    assert rel(p.dense(np.roll(x, d)), np.roll(p.dense(x), d, axis=1)) < 1e-12
    # envelopes: a shift by q output samples (d = q N/N_out) is a roll times a phase
    qs = 3
    Y0 = p.forward(x)
    Y1 = p.forward(np.roll(x, qs * (N // M)))
    phase = np.exp(-2j * np.pi * s * qs / M)[:, None]
    assert rel(Y1, phase * np.roll(Y0, qs, axis=1)) < 1e-12


def test_pure_sinusoid_closed_form():
    p = o.OraclePlan(fs=1024.0, n=4096, q=8.0, f_min=20.0, f_max=400.0, rows=24)
    t = p.row_table()
    W = p.windows()
    N, M = p.n, p.N_out
    k0 = 15
    b0 = int(t["centre"][k0])
    assert b0 not in set(np.delete(t["centre"], k0))
    x = np.cos(2 * np.pi * b0 * np.arange(N) / N)
    Y = p.forward(x)
    amp = 0.5 * math.sqrt(N / M) * W[:, b0]
    assert np.allclose(np.abs(Y), amp[:, None], rtol=1e-12, atol=1e-13)
    assert int(np.argmax(np.abs(Y).max(axis=1))) == k0
    # the carrier offset is removed: row k0 is constant in time, phase 0
    assert np.allclose(Y[k0], amp[k0], rtol=1e-12, atol=1e-13)


# --------------------------------------------------------------------------
# Composite multi-Q / multi-window banks (App. A extension): planes are
# independent analyses of one spectrum, the frame is their sum, and the
# plane metrics follow from Parseval and from a pure tone.
# --------------------------------------------------------------------------
COMPOSITE = [(4.0, o.WIN_BISQUARE, 0.0), (8.0, o.WIN_HANN, 0.0), (16.0, o.WIN_TUKEY, 0.5)]


def composite_plan(**kw):
    base = dict(fs=1024.0, n=4096, q=1.0, f_min=20.0, f_max=400.0, rows=24, planes=COMPOSITE)
    base.update(kw)
    return o.OraclePlan(**base)


def test_composite_planes_are_single_plans():
    pc = composite_plan()
    assert pc.R == 3 * 24 and pc.n_planes == 3 and pc.rows_per_plane == 24
    x = np.random.default_rng(31).standard_normal(pc.n)
    Yc = pc.forward(x)
    P_sum = np.zeros(pc.n // 2 + 1)
    for i, (q, w, a) in enumerate(COMPOSITE):
        ps = o.OraclePlan(fs=1024.0, n=4096, q=q, f_min=20.0, f_max=400.0, rows=24, window=w, window_param=a,
                          n_out=pc.N_out)
        # forward rows do not see the other planes
        assert np.array_equal(Yc[24 * i:24 * (i + 1)], ps.forward(x))
        P_sum += ps.frame()[0]
    # the bank's frame operator is the sum of the planes' ones
    assert rel(pc.frame()[0], P_sum) < 1e-14


def test_composite_exact_reconstruction():
    pc = composite_plan()
    x = np.random.default_rng(32).standard_normal(pc.n)
    xm = pc.project(x)
    assert rel(pc.inverse(pc.forward(x)), xm) < 1e-12
    # the bank covers more bins than its narrowest plane
    ps = o.OraclePlan(fs=1024.0, n=4096, q=16.0, f_min=20.0, f_max=400.0, rows=24, window=o.WIN_TUKEY,
                      window_param=0.5)
    assert pc.frame()[1].sum() >= ps.frame()[1].sum()


def test_row_energy_is_parseval_of_windowed_spectrum():
    pc = composite_plan()
    x = np.random.default_rng(33).standard_normal(pc.n)
    energy, _ = pc.row_stats(pc.forward(x))
    X = np.fft.rfft(x)                       # numpy, not the oracle's spectrum
    W = pc.windows()
    expect = np.sum(np.abs(W * X[None, :]) ** 2, axis=1) / pc.n
    assert rel(energy, expect) < 1e-12


def test_plane_scores_of_a_pure_tone():
    """A tone at bin b0 gives |Y_k[m]|^2 = (sqrt(N/N_out) W_k[b0] / 2)^2 for
    every m, so the peak score of plane p is max_k of that and the energy
    score is N/4 times the plane's frame operator at b0."""
    pc = composite_plan()
    N, M = pc.n, pc.N_out
    b0 = 300
    x = np.cos(2 * np.pi * b0 * np.arange(N) / N)
    Y = pc.forward(x)
    W = pc.windows()[:, b0].reshape(3, 24)
    peak = pc.plane_scores(Y, "peak")
    energy = pc.plane_scores(Y, "energy")
    assert np.allclose(peak, (0.5 * math.sqrt(N / M) * W.max(axis=1)) ** 2, rtol=1e-12)
    assert np.allclose(energy, N / 4.0 * np.sum(W ** 2, axis=1), rtol=1e-12)
    _, best, Yb = pc.select_planes(Y, "energy")
    assert best == int(np.argmax(np.sum(W ** 2, axis=1)))
    assert np.array_equal(Yb, Y[24 * best:24 * (best + 1)])


def test_selection_is_per_segment():
    """A long steady tone favours the highest-Q plane under the peak metric;
    a short click favours the lowest-Q plane; in one batch each segment
    keeps its own plane."""
    pc = composite_plan(planes=[(2.0, o.WIN_BISQUARE, 0.0), (32.0, o.WIN_BISQUARE, 0.0)])
    N = pc.n
    b0 = int(pc.row_table()["centre"][10])       # on a row centre, where the Q = 32 plane has no hole
    tone = np.cos(2 * np.pi * (b0 + 0.25) * np.arange(N) / N)
    click = np.zeros(N)
    click[N // 2] = 50.0
    Y = pc.forward(np.stack([tone, click]))
    _, best, Yb = pc.select_planes(Y, "peak")
    assert list(best) == [1, 0]
    R = pc.rows_per_plane
    assert np.array_equal(Yb[0], Y[0, R:2 * R]) and np.array_equal(Yb[1], Y[1, :R])


# --------------------------------------------------------------------------
# Regularised stop band (Sec. III; App. A): windows non-zero on every bin,
# so the signal comes back from any single tile by spectral division.
# --------------------------------------------------------------------------
def test_regularised_windows_and_single_tile_recovery():
    kw = dict(fs=256.0, n=1024, q=4.0, f_min=10.0, f_max=100.0, rows=8)
    eps = 1e-4
    p = o.OraclePlan(eps=eps, **kw)
    p0 = o.OraclePlan(**kw)
    W, W0 = p.windows(), p0.windows()
    assert np.all(W > 0) and p.N_out >= p.n // 2 + 1
    # where the shape is at least eps it is the plain window up to the
    # normalisation; elsewhere (the stop band, the support's end points and
    # the tails below eps) the value is eps times that factor
    for k in range(p.R):
        on = W0[k] >= eps * W0[k].max()
        assert (~on).sum() > p.n // 2 - (p.row_table()["hi"][k] - p.row_table()["lo"][k])   # tails included
        ratio = W[k, on] / W0[k, on]
        assert np.allclose(ratio, ratio[0], rtol=1e-13)
        # the bisquare shape peaks at 1, so the plain window's peak is 1/||shape||
        assert np.allclose(W[k, ~on], eps * ratio[0] * W0[k].max(), rtol=1e-12)
    x = np.random.default_rng(41).standard_normal((2, p.n))
    Y = p.forward(x)
    for k in (0, 3, p.R - 1):
        assert rel(p.tile_inverse(Y, k), x) < 1e-10
    # the plain windows vanish at their support ends: no division possible
    with pytest.raises(ValueError):
        p0.tile_inverse(p0.forward(x), 2)


def test_regularised_taper_tails_floored():
    """A Planck taper falls far below any eps inside its support (down to
    underflow near the ends). With eps read as a floor every window is at
    least eps times its peak, so the single-tile inverse amplifies rounding
    by at most about 1/eps: FP64 recovery of the signal from each of several
    tiles within 1e-15/eps, on rows whose plain taper has values below
    eps/10 of its peak (with only the zeros replaced, row 11's smallest value,
    6e-9 of its peak, would amplify rounding about 200 times more)."""
    kw = dict(fs=256.0, n=2048, q=6.0, f_min=8.0, f_max=120.0, rows=12, window=o.WIN_PLANCK, window_param=0.25)
    eps = 1e-5
    p = o.OraclePlan(eps=eps, **kw)
    p0 = o.OraclePlan(**kw)
    W, W0 = p.windows(), p0.windows()
    for k in range(p.R):
        assert W[k].min() >= eps * W[k].max() * (1 - 1e-12)
    tiny = [k for k in range(p.R) if np.any((W0[k] > 0) & (W0[k] < 0.1 * eps * W0[k].max()))]
    assert tiny, "no row with a taper tail far below eps"
    x = np.random.default_rng(43).standard_normal((2, p.n))
    Y = p.forward(x)
    for k in tiny + [0]:
        assert rel(p.tile_inverse(Y, k), x) < 1e-15 / eps, k


@pytest.mark.parametrize("n,f_min,f_max", [(256, 8.0, 50.0), (384, 5.0, 60.0), (640, 3.0, 62.0)])
def test_regularised_forward_matches_dense_definition(n, f_min, f_max):
    """With eps the dense tile of the definition still equals the re-modulated
    envelope (the full band is one kept support). N = 384 and 640 (N/2 = 3 and
    5 times a power of two) give N_out = 256 and 512, shorter than N: a row's
    band 0..N/2 then reaches further than N_out/2 on one side of its centre,
    and the wrap of slots (c - s) mod N_out is what places it."""
    p = o.OraclePlan(fs=128.0, n=n, q=4.0, f_min=f_min, f_max=f_max, rows=5, eps=1e-3)
    assert p.N_out >= p.n // 2 + 1
    t0 = p.row_table()
    if n != 256:
        assert p.N_out < p.n
        off_centre = (t0["centre"] - t0["lo"] > p.N_out // 2) | (t0["hi"] - t0["centre"] >= p.N_out // 2)
        assert off_centre.any()
    x = np.random.default_rng(42).standard_normal(p.n)
    xs = np.stack([x, np.roll(x, 7)])
    assert rel(p.inverse(p.forward(xs)), p.project(xs)) < 1e-12
    for k in (0, p.R - 1):
        assert rel(p.tile_inverse(p.forward(xs), k), xs) < 1e-9
    T = p.dense(x)
    Y = p.forward(x)
    t = p.row_table()
    N, M = p.n, p.N_out
    for k in range(p.R):
        F = np.zeros(N, dtype=complex)
        Yt = np.fft.fft(Y[k]) * np.sqrt(N / M)
        for c in range(t["lo"][k], t["hi"][k] + 1):
            F[c] = Yt[(c - t["centre"][k]) % M]
        assert rel(np.fft.ifft(F), T[k]) < 1e-12


def test_sampled_rows_are_the_full_forward_rows():
    """forward_rows (the forward for chosen rows only, used where the oracle's
    every-row transform is too slow) returns exactly those rows of forward."""
    p = o.OraclePlan(fs=1024.0, n=4096, q=8.0, f_min=10.0, f_max=400.0, rows=16, n_out=201)
    x = np.random.default_rng(43).standard_normal((2, p.n))
    Y = p.forward(x)
    assert np.array_equal(p.forward_rows(x, [3, 0, 15]), Y[:, [3, 0, 15]])
    assert np.array_equal(p.forward_rows(x[1], [7]), Y[1, [7]])
    with pytest.raises(IndexError):
        p.forward_rows(x, [16])
