"""Seeded synthetic detector-like inputs.

This module only draws input signals. It holds none of the transform's
arithmetic, imports neither the library nor the oracle, and is the one piece of
code that both sides' tests and the benchmark share.

Every draw uses ``numpy.random.Generator(PCG64(seed))`` with
``seed = 1000 * workload + segment``, so a segment is reproducible on its own.

Signal models (stand-ins for the paper's LIGO/Virgo strain and glitch data,
which are not available here):

* white Gaussian noise, sigma = 1;
* coloured Gaussian noise: white noise shaped in the frequency domain by
  sqrt(S(f)) with S(f) = (20 Hz / f)^4 for 1 <= f < 20 Hz, S(1 Hz) below 1 Hz,
  0 at DC, 1 for f >= 20 Hz (a steep low-frequency wall, flat above; the flat
  level has unit variance per sample);
* sine-Gaussian glitch A exp(-(t-t0)^2/tau^2) sin(2 pi f0 (t-t0)),
  tau = Q / (sqrt(2) pi f0);
* inspiral-like chirp f(t) = 30 Hz (1 - t/tc)^(-3/8), tc = d / (1 - 10^(-8/3)),
  rising from 30 Hz to 300 Hz over its duration d, with 0.1 s cosine tapers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def rng_for(workload: int, segment: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * int(workload) + int(segment)))


def white(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.standard_normal(n)


def coloured(n: int, fs: float, rng: np.random.Generator) -> np.ndarray:
    w = rng.standard_normal(n)
    W = np.fft.rfft(w)
    f = np.fft.rfftfreq(n, d=1.0 / fs)
    S = np.ones_like(f)
    low = f < 20.0
    S[low] = (20.0 / np.maximum(f[low], 1.0)) ** 4
    S[0] = 0.0
    return np.fft.irfft(W * np.sqrt(S), n=n)


def sine_gaussian(n: int, fs: float, f0: float, q: float, t0: float) -> np.ndarray:
    t = np.arange(n) / fs
    tau = q / (math.sqrt(2.0) * math.pi * f0)
    return np.exp(-((t - t0) / tau) ** 2) * np.sin(2.0 * math.pi * f0 * (t - t0))


def chirp(n: int, fs: float, start: float, duration: float, f_lo: float = 30.0,
          f_hi: float = 300.0, taper: float = 0.1) -> np.ndarray:
    t = np.arange(n) / fs - start
    ratio = (f_hi / f_lo) ** (-8.0 / 3.0)
    tc = duration / (1.0 - ratio)
    inside = (t >= 0.0) & (t <= duration)
    u = np.clip(1.0 - t / tc, ratio, 1.0)
    phase = 2.0 * math.pi * f_lo * tc * (8.0 / 5.0) * (1.0 - u ** (5.0 / 8.0))
    y = np.where(inside, np.sin(phase), 0.0)
    if taper > 0.0:
        ramp_in = np.clip(t / taper, 0.0, 1.0)
        ramp_out = np.clip((duration - t) / taper, 0.0, 1.0)
        y *= 0.5 * (1.0 - np.cos(math.pi * ramp_in)) * 0.5 * (1.0 - np.cos(math.pi * ramp_out))
    return y


@dataclass
class Injection:
    kind: str
    params: dict = field(default_factory=dict)


def injected_segment(n: int, fs: float, rng: np.random.Generator, noise: str = "coloured",
                     n_glitch: int = 2, with_chirp: bool = True, amp_sigma: float = 5.0):
    """Noise plus one chirp (d ~ U[2, 8] s, amplitude 5 sigma) and sine-Gaussian
    glitches (f0 ~ U[50, 1500] Hz, Q ~ U[4, 20], t0 ~ U[0, T], peak 5 sigma).
    Returns (noisy, clean, injections)."""
    T = n / fs
    x = coloured(n, fs, rng) if noise == "coloured" else white(n, rng)
    clean = np.zeros(n)
    inj = []
    if with_chirp:
        d = float(rng.uniform(2.0, 8.0))
        d = min(d, 0.9 * T)
        st = float(rng.uniform(0.0, max(T - d, 0.0)))
        c = amp_sigma * chirp(n, fs, st, d)
        clean += c
        inj.append(Injection("chirp", dict(start=st, duration=d)))
    for _ in range(n_glitch):
        f0 = float(rng.uniform(min(50.0, 0.2 * fs), min(1500.0, 0.45 * fs)))   # low rates: below 0.45 fs
        q = float(rng.uniform(4.0, 20.0))
        t0 = float(rng.uniform(0.0, T))
        g = sine_gaussian(n, fs, f0, q, t0)
        peak = np.max(np.abs(g))
        if peak > 0:
            g *= amp_sigma / peak
        clean += g
        inj.append(Injection("sine_gaussian", dict(f0=f0, q=q, t0=t0)))
    return x + clean, clean, inj


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
def single_segment(seed_segment: int = 0):
    """4 s at 4096 Hz: white noise (sigma 1) plus one sine-Gaussian with
    f0 = 100 Hz, Q = 8, t0 = 2 s, scaled to ||h||_2 = 20 (matched-filter SNR
    in unit white noise)."""
    n, fs = 16384, 4096.0
    rng = rng_for(1, seed_segment)
    h = sine_gaussian(n, fs, 100.0, 8.0, 2.0)
    h *= 20.0 / np.linalg.norm(h)
    return white(n, rng) + h


def batched_segments(batch: int = 256, n: int = 131072, fs: float = 4096.0, workload: int = 2,
                     first: int = 0, dtype=np.float32) -> np.ndarray:
    """Coloured noise with one chirp and two sine-Gaussian glitches per segment."""
    out = np.empty((batch, n), dtype=dtype)
    for i in range(batch):
        out[i] = injected_segment(n, fs, rng_for(workload, first + i))[0]
    return out


def differentiable_pairs(batch: int = 64, n: int = 32768, fs: float = 4096.0, first: int = 0,
                         dtype=np.float32):
    """(noisy, clean) pairs: clean = chirp + sine-Gaussians, noisy = clean +
    coloured noise."""
    noisy = np.empty((batch, n), dtype=dtype)
    clean = np.empty((batch, n), dtype=dtype)
    for i in range(batch):
        a, c, _ = injected_segment(n, fs, rng_for(5, first + i))
        noisy[i], clean[i] = a, c
    return noisy, clean


@dataclass
class Request:
    arrival: float          # seconds since the start of the stream
    fs: float
    n: int
    q: float
    rows: int
    seed: int


def serving_stream(rate: float = 200.0, duration: float = 60.0, seed: int = 3000,
                   seconds=(1, 4, 16, 64), rates=(4096.0, 16384.0), qs=(4.0, 8.0, 16.0, 32.0),
                   rows=(64, 128, 256, 512)):
    """Poisson arrivals (exponential gaps) of requests whose duration, sample
    rate, Q and row count are drawn uniformly from the given sets."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    i = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration:
            break
        sec = int(rng.choice(seconds))
        fs = float(rng.choice(rates))
        out.append(Request(arrival=t, fs=fs, n=int(sec * fs), q=float(rng.choice(qs)),
                           rows=int(rng.choice(rows)), seed=3000 + i))
        i += 1
    return out


def request_signal(req: Request, dtype=np.float32) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(req.seed))
    return injected_segment(req.n, req.fs, rng)[0].astype(dtype)
