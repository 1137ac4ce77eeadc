// QTAM oracle: a plain, slow, FP64 CPU implementation of the forward and
// inverse Q-transform with amplitude demodulation (Asprea et al., "QTAM:
// Q-Transform Amplitude Modulation", arXiv 2603.29785).
//
// THIS IS TEST INFRASTRUCTURE. It exists only to check the GPU library. It
// shares no code, header, table or constant generator with the library under
// paper_2603_29785_amd/, and nothing on the product path may load it. Only the
// tests, the smoke check and the CPU-baseline leg of the benchmark call it.
//
// Everything is double precision and written for clarity, not speed:
//   * the spectrum is the full N-point complex DFT of the real input, of which
//     bins 0..N/2 are kept (no real-FFT packing tricks);
//   * transforms use an iterative radix-2 Cooley-Tukey FFT for power-of-two
//     lengths, a recursive split by the smallest prime factor for other
//     composite lengths, and a direct O(n^2) DFT for primes (or when asked);
//   * every twiddle is cos/sin of its own angle, never a recurrence.
//
// Readings of points the paper leaves open are listed beside the step that
// takes them. Parity of the absolute scale of the windows (Q constant, width
// rounding, normalisation) is pinned only by the paper's formulas as read
// here, not by any number the paper prints.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <vector>

namespace {

using cd = std::complex<double>;
const double kPi = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------------------
// Discrete Fourier transforms. sign = -1: X[k] = sum_n x[n] e^{-2 pi i kn/n}
// (the paper's forward DFT, App. C); sign = +1: the unnormalised inverse kernel
// e^{+2 pi i kn/n}. No 1/n factor is applied here.
// ---------------------------------------------------------------------------

void dft_direct(int64_t n, const cd* in, cd* out, int sign) {
  std::vector<cd> tmp(static_cast<size_t>(n));
  for (int64_t k = 0; k < n; ++k) {
    cd acc(0.0, 0.0);
    for (int64_t t = 0; t < n; ++t) {
      // reduce k*t mod n exactly in integers before forming the angle
      const int64_t m = static_cast<int64_t>((static_cast<__int128>(k) * t) % n);
      const double ang = sign * 2.0 * kPi * static_cast<double>(m) / static_cast<double>(n);
      acc += in[t] * cd(std::cos(ang), std::sin(ang));
    }
    tmp[static_cast<size_t>(k)] = acc;
  }
  std::copy(tmp.begin(), tmp.end(), out);
}

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

// Iterative radix-2 decimation-in-time FFT (bit-reversal permutation, then
// log2(n) butterfly stages). Twiddle w^j of a stage of length len is computed
// as cos/sin of 2*pi*j/len directly.
void fft_radix2(int64_t n, const cd* in, cd* out, int sign) {
  std::vector<cd> a(in, in + n);
  int bits = 0;
  while ((int64_t(1) << bits) < n) ++bits;
  for (int64_t i = 0; i < n; ++i) {
    int64_t r = 0;
    for (int b = 0; b < bits; ++b)
      if (i & (int64_t(1) << b)) r |= int64_t(1) << (bits - 1 - b);
    if (r > i) std::swap(a[static_cast<size_t>(i)], a[static_cast<size_t>(r)]);
  }
  for (int64_t len = 2; len <= n; len <<= 1) {
    const int64_t half = len / 2;
    std::vector<cd> w(static_cast<size_t>(half));
    for (int64_t j = 0; j < half; ++j) {
      const double ang = sign * 2.0 * kPi * static_cast<double>(j) / static_cast<double>(len);
      w[static_cast<size_t>(j)] = cd(std::cos(ang), std::sin(ang));
    }
    for (int64_t base = 0; base < n; base += len) {
      for (int64_t j = 0; j < half; ++j) {
        const cd u = a[static_cast<size_t>(base + j)];
        const cd v = a[static_cast<size_t>(base + j + half)] * w[static_cast<size_t>(j)];
        a[static_cast<size_t>(base + j)] = u + v;
        a[static_cast<size_t>(base + j + half)] = u - v;
      }
    }
  }
  std::copy(a.begin(), a.end(), out);
}

bool g_force_direct = false;

void dft(int64_t n, const cd* in, cd* out, int sign);

// Cooley-Tukey split of a composite length n = p * m, p its smallest prime
// factor: the p decimated sequences x[q + p t] are transformed (length m)
// and combined, X[k] = sum_q w^(q k) F_q[k mod m], w = e^(sign 2 pi i / n),
// every w^(qk) again from its own angle with qk reduced mod n in integers.
void fft_split(int64_t n, int64_t p, const cd* in, cd* out, int sign) {
  const int64_t m = n / p;
  std::vector<cd> sub(static_cast<size_t>(m)), f(static_cast<size_t>(n));
  for (int64_t q = 0; q < p; ++q) {
    for (int64_t t = 0; t < m; ++t) sub[static_cast<size_t>(t)] = in[q + p * t];
    dft(m, sub.data(), f.data() + q * m, sign);
  }
  std::vector<cd> tmp(static_cast<size_t>(n));
  for (int64_t k = 0; k < n; ++k) {
    cd acc(0.0, 0.0);
    for (int64_t q = 0; q < p; ++q) {
      const int64_t e = (q * k) % n;
      const double ang = sign * 2.0 * kPi * static_cast<double>(e) / static_cast<double>(n);
      acc += f[static_cast<size_t>(q * m + k % m)] * cd(std::cos(ang), std::sin(ang));
    }
    tmp[static_cast<size_t>(k)] = acc;
  }
  std::copy(tmp.begin(), tmp.end(), out);
}

int64_t smallest_factor(int64_t n) {
  for (int64_t p = 2; p * p <= n; ++p)
    if (n % p == 0) return p;
  return n;
}

// Power-of-two lengths: radix-2; other composite lengths: split by their
// smallest prime factor; primes (or when forced): the direct sum.
void dft(int64_t n, const cd* in, cd* out, int sign) {
  if (g_force_direct || n <= 1) {
    dft_direct(n, in, out, sign);
  } else if (is_pow2(n)) {
    fft_radix2(n, in, out, sign);
  } else {
    const int64_t p = smallest_factor(n);
    if (p == n)
      dft_direct(n, in, out, sign);
    else
      fft_split(n, p, in, out, sign);
  }
}

// ---------------------------------------------------------------------------
// Plan: the frequency grid, centres, widths, windows and frame (App. A;
// Sec. II window equations; App. C frame operator).
// ---------------------------------------------------------------------------

enum { CAP_COVER = 0, CAP_PAPER = 1, CAP_NONE = 2, CAP_MANUAL = 3 };
enum { NORM_UNIT_ENERGY = 0, NORM_PAPER_INV_ENERGY = 1, NORM_NONE = 2 };
enum { WIN_BISQUARE = 0, WIN_HANN = 1, WIN_KAISER = 2, WIN_TUKEY = 3, WIN_PLANCK = 4 };

struct Row {
  double f;                 // nominal centre frequency f_k (Hz)
  int64_t s;                // centre bin s_k
  int64_t h;                // half width h_k (support |j| <= h_k)
  int64_t lo, hi;           // kept bins [lo, hi] after clipping to [0, N/2]
  std::vector<double> w;    // W_k at bins lo..hi
};

struct Plan {
  double fs = 0.0;
  int64_t n = 0;            // samples per segment N
  double q = 0.0;
  int64_t nbins = 0;        // N/2 + 1
  int64_t l_max = -1;       // cap on L_k (odd), -1 = no cap
  int64_t n_out = 0;
  double tau = 0.0;         // mask threshold relative to max P
  double eps = 0.0;         // stop-band value (> 0: every row keeps the whole band)
  std::vector<Row> rows;
  std::vector<double> P;    // frame operator diagonal, per bin
  std::vector<unsigned char> M;  // reconstruction mask, per bin
};

// Zeroth-order modified Bessel function of the first kind by its power
// series sum_k ((x/2)^k / k!)^2 (used only by the Kaiser window).
double bessel_i0(double x) {
  double term = 1.0, sum = 1.0;
  const double y = 0.25 * x * x;
  for (int k = 1; k < 500; ++k) {
    term *= y / (static_cast<double>(k) * static_cast<double>(k));
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

// Window shape at relative offset x = j / h in [-1, 1] (App. A). The
// Planck-taper exponent is read as 1/u - 1/(1-u) with u = (1-|x|)/alpha the
// position inside the taper: the printed sum of the two terms would vanish
// at both ends of the taper, the sign makes it rise from 0 to 1.
double window_shape(int kind, double x, double param) {
  const double ax = std::fabs(x);
  if (ax > 1.0) return 0.0;
  switch (kind) {
    case WIN_BISQUARE: {
      const double t = 1.0 - x * x;
      return t * t;
    }
    case WIN_HANN:
      return 0.5 * (1.0 + std::cos(kPi * x));
    case WIN_KAISER:
      return bessel_i0(param * std::sqrt(std::max(0.0, 1.0 - x * x))) / bessel_i0(param);
    case WIN_TUKEY: {
      const double a = param;
      if (a <= 0.0) return 1.0;
      if (ax <= 1.0 - a) return 1.0;
      return 0.5 * (1.0 + std::cos(kPi * (ax - (1.0 - a)) / a));
    }
    case WIN_PLANCK: {
      const double a = param;
      if (a <= 0.0) return ax < 1.0 ? 1.0 : 0.0;
      if (ax <= 1.0 - a) return 1.0;
      if (ax >= 1.0) return 0.0;
      const double u = (1.0 - ax) / a;
      const double z = 1.0 / u - 1.0 / (1.0 - u);
      if (z > 700.0) return 0.0;
      return 1.0 / (std::exp(z) + 1.0);
    }
  }
  return 0.0;
}

int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// One plane of a composite bank: its quality factor and window (App. A,
// multi-Q / multi-window extension). A plain plan has one plane.
struct PlaneSpec {
  double q;
  int32_t window;
  double param;
};

// Returns 0 on success, 1 on invalid parameters. Rows are plane after plane,
// each plane over the same frequency grid.
// eps > 0: every window takes the value eps on the bins of the one-sided
// band where its shape is below eps (Sec. III regularised stop band; App. A:
// the stop band, the support's end points and the tails of a taper below
// eps), before the normalisation, so that it is at least eps times its peak
// on all bins 0..N/2 and a single tile is invertible with rounding amplified
// by at most about 1/eps.
int build_plan(Plan& pl, double fs, int64_t n, const std::vector<PlaneSpec>& planes, double fmin,
               double fmax, int32_t nrows, const double* freqs, int32_t cap_mode, int32_t max_window,
               int32_t norm_mode, int32_t n_out, double tau, double eps) {
  if (!(eps >= 0.0)) return 1;
  pl.eps = eps;
  if (!(fs > 0.0) || n < 4 || (n % 2) != 0 || nrows < 1 || planes.empty()) return 1;
  for (const PlaneSpec& ps : planes)
    if (!(ps.q > 0.0)) return 1;
  pl.q = planes[0].q;
  pl.fs = fs;
  pl.n = n;
  pl.nbins = n / 2 + 1;
  pl.tau = tau;
  const double T = static_cast<double>(n) / fs;   // segment duration N_t

  // O1 grid: geometric spacing of R rows over [f_min, f_max], both ends
  // included (App. A builds f_min * 2^(k/B); a row count replaces B here), or
  // the caller's explicit list.
  std::vector<double> f(static_cast<size_t>(nrows));
  for (int32_t k = 0; k < nrows; ++k) {
    if (freqs) {
      f[static_cast<size_t>(k)] = freqs[k];
    } else if (nrows == 1) {
      f[0] = fmin;
    } else {
      f[static_cast<size_t>(k)] =
          fmin * std::pow(fmax / fmin, static_cast<double>(k) / static_cast<double>(nrows - 1));
    }
  }
  for (int32_t k = 0; k < nrows; ++k) {
    const double fk = f[static_cast<size_t>(k)];
    if (!(fk > 0.0) || fk > fs / 2.0) return 1;
    if (k > 0 && fk < f[static_cast<size_t>(k - 1)]) return 1;
  }

  // O3 cap (App. A, max_window_size): the largest gap between consecutive
  // centres, rounded up to whole bins, g = ceil(N_t * df_max).
  pl.l_max = -1;
  if (cap_mode == CAP_MANUAL) {
    if (max_window < 1) return 1;
    pl.l_max = max_window;
  } else if (cap_mode != CAP_NONE && nrows >= 2) {
    double dfmax = 0.0;
    for (int32_t k = 0; k + 1 < nrows; ++k)
      dfmax = std::max(dfmax, f[static_cast<size_t>(k + 1)] - f[static_cast<size_t>(k)]);
    const int64_t g = static_cast<int64_t>(std::ceil(T * dfmax));
    if (cap_mode == CAP_COVER)
      pl.l_max = 2 * g + 1;              // each clamped window reaches its neighbours' centres
    else if (cap_mode == CAP_PAPER)
      pl.l_max = 2 * (g / 2) + 1;        // the formula as printed in App. A
    else
      return 1;
  } else if (cap_mode != CAP_NONE && cap_mode != CAP_COVER && cap_mode != CAP_PAPER) {
    return 1;
  }

  pl.rows.clear();
  const int64_t half_bins = n / 2;
  int64_t max_len = 0;
  for (size_t plane = 0; plane < planes.size(); ++plane)
  for (int32_t k = 0; k < nrows; ++k) {
    const double q = planes[plane].q;
    const int32_t window = planes[plane].window;
    const double window_param = planes[plane].param;
    Row r;
    r.f = f[static_cast<size_t>(k)];
    // O2 centre bin: k_c = f * N_t (Sec. II), rounded to the nearest integer
    // bin so that the baseband shift is a circular roll by whole bins.
    r.s = static_cast<int64_t>(std::floor(r.f * T + 0.5));
    // O4 width: ideal full width f*N_t/Q bins (Q = f/df), made odd as in
    // the cap formula, then clamped to the cap; at least one bin each side.
    int64_t h = static_cast<int64_t>(std::ceil(r.f * T / q)) / 2;
    if (h < 1) h = 1;
    if (pl.l_max > 0) h = std::min(h, pl.l_max / 2);
    if (h < 1) h = 1;
    r.h = h;
    max_len = std::max(max_len, 2 * h + 1);
    // O5 window on the support |j| <= h, clipped to the one-sided band
    // 0 <= s+j <= N/2 (no wrap into negative frequencies); with a stop-band
    // value eps the kept bins are the whole band.
    r.lo = eps > 0.0 ? 0 : std::max<int64_t>(0, r.s - h);
    r.hi = eps > 0.0 ? half_bins : std::min<int64_t>(half_bins, r.s + h);
    if (r.lo > r.hi) return 1;
    if (eps > 0.0) max_len = std::max(max_len, half_bins + 1);
    r.w.assign(static_cast<size_t>(r.hi - r.lo + 1), 0.0);
    double energy = 0.0;
    for (int64_t c = r.lo; c <= r.hi; ++c) {
      // eps is a floor: every bin where the shape is below it (the stop band,
      // the support's own end points where the bisquare is zero, the tails
      // of a taper that fall below eps) takes the value eps
      const bool inside = c >= r.s - h && c <= r.s + h;
      const double x = static_cast<double>(c - r.s) / static_cast<double>(h);
      double v = inside ? window_shape(window, x, window_param) : 0.0;
      if (eps > 0.0 && v < eps) v = eps;
      r.w[static_cast<size_t>(c - r.lo)] = v;
      energy += v * v;
    }
    if (!(energy > 0.0)) return 1;
    // Normalisation (Sec. II): unit energy per tile by default; the literal
    // printed constant 1/sum(W'^2) on request; or none.
    double scale = 1.0;
    if (norm_mode == NORM_UNIT_ENERGY)
      scale = 1.0 / std::sqrt(energy);
    else if (norm_mode == NORM_PAPER_INV_ENERGY)
      scale = 1.0 / energy;
    else if (norm_mode != NORM_NONE)
      return 1;
    for (double& v : r.w) v *= scale;
    pl.rows.push_back(std::move(r));
  }

  // O6 output length: any N_out >= max L_k holds every support without
  // aliasing; automatic choice is the next power of two.
  if (n_out == 0)
    pl.n_out = next_pow2(max_len);
  else if (n_out >= max_len)
    pl.n_out = n_out;
  else
    return 1;

  // O9 frame operator P[b] = sum_k |W_k[b]|^2 (App. C) and the mask of bins
  // where it is usable, M[b] = [P[b] >= tau * max P] (tau = 0: P > 0).
  pl.P.assign(static_cast<size_t>(pl.nbins), 0.0);
  for (const Row& r : pl.rows)
    for (int64_t c = r.lo; c <= r.hi; ++c) {
      const double v = r.w[static_cast<size_t>(c - r.lo)];
      pl.P[static_cast<size_t>(c)] += v * v;
    }
  double pmax = 0.0;
  for (double v : pl.P) pmax = std::max(pmax, v);
  pl.M.assign(static_cast<size_t>(pl.nbins), 0);
  for (int64_t b = 0; b < pl.nbins; ++b) {
    const double v = pl.P[static_cast<size_t>(b)];
    pl.M[static_cast<size_t>(b)] = (v > 0.0 && v >= tau * pmax) ? 1 : 0;
  }
  return 0;
}

// O7 spectrum: X[b] = sum_n x[n] e^{-2 pi i bn/N}, b = 0..N/2 (App. C), from
// the full complex N-point DFT of the real input.
void spectrum(const Plan& pl, const double* x, std::vector<cd>& X) {
  const int64_t n = pl.n;
  std::vector<cd> a(static_cast<size_t>(n)), A(static_cast<size_t>(n));
  for (int64_t t = 0; t < n; ++t) a[static_cast<size_t>(t)] = cd(x[t], 0.0);
  dft(n, a.data(), A.data(), -1);
  X.assign(A.begin(), A.begin() + pl.nbins);
}

// O12 back to time: x[n] = (1/N) sum over the full Hermitian spectrum, built
// from bins 0..N/2 with the real parts of DC and Nyquist (irfft convention).
void synthesis_real(const Plan& pl, const std::vector<cd>& Xh, double* x) {
  const int64_t n = pl.n;
  std::vector<cd> F(static_cast<size_t>(n)), a(static_cast<size_t>(n));
  F[0] = cd(Xh[0].real(), 0.0);
  F[static_cast<size_t>(n / 2)] = cd(Xh[static_cast<size_t>(n / 2)].real(), 0.0);
  for (int64_t b = 1; b < n / 2; ++b) {
    F[static_cast<size_t>(b)] = Xh[static_cast<size_t>(b)];
    F[static_cast<size_t>(n - b)] = std::conj(Xh[static_cast<size_t>(b)]);
  }
  dft(n, F.data(), a.data(), +1);
  for (int64_t t = 0; t < n; ++t) x[t] = a[static_cast<size_t>(t)].real() / static_cast<double>(n);
}

int64_t wrap(int64_t j, int64_t m) {
  int64_t r = j % m;
  return r < 0 ? r + m : r;
}

// O8 forward, one segment: filter by W_k, roll the band to baseband (bin s_k
// to slot 0, offset j to slot j mod N_out), zero-pad to N_out and take the
// short inverse DFT with the renormalisation sqrt(N_out/N) (Sec. III; App. A;
// App. C, demodulation equations; N_in read as N).
// Rows idx[0..count) of the segment, in that order (every row: idx = 0..R-1).
void forward_rows(const Plan& pl, const double* x, const int64_t* idx, int64_t count, cd* Y) {
  std::vector<cd> X;
  spectrum(pl, x, X);
  const int64_t m = pl.n_out;
  const double norm = std::sqrt(static_cast<double>(m) / static_cast<double>(pl.n)) / static_cast<double>(m);
  std::vector<cd> Z(static_cast<size_t>(m)), y(static_cast<size_t>(m));
  for (int64_t i = 0; i < count; ++i) {
    const Row& r = pl.rows[static_cast<size_t>(idx[i])];
    std::fill(Z.begin(), Z.end(), cd(0.0, 0.0));
    for (int64_t c = r.lo; c <= r.hi; ++c)
      Z[static_cast<size_t>(wrap(c - r.s, m))] += X[static_cast<size_t>(c)] * r.w[static_cast<size_t>(c - r.lo)];
    dft(m, Z.data(), y.data(), +1);
    for (int64_t t = 0; t < m; ++t) Y[i * m + t] = y[static_cast<size_t>(t)] * norm;
  }
}

void forward_one(const Plan& pl, const double* x, cd* Y) {
  std::vector<int64_t> all(pl.rows.size());
  for (size_t k = 0; k < all.size(); ++k) all[k] = static_cast<int64_t>(k);
  forward_rows(pl, x, all.data(), static_cast<int64_t>(all.size()), Y);
}

// O10-O12 inverse, one segment: DFT each row, re-modulate it to its carrier
// with sqrt(N/N_out), weight by W_k, overlap-add, divide by the frame
// operator P on the mask M, and go back to time (Sec. III canonical dual
// frame; App. C).
void inverse_one(const Plan& pl, const cd* Y, double* x) {
  const int64_t m = pl.n_out;
  const double scale = std::sqrt(static_cast<double>(pl.n) / static_cast<double>(m));
  std::vector<cd> acc(static_cast<size_t>(pl.nbins), cd(0.0, 0.0));
  std::vector<cd> y(static_cast<size_t>(m)), Yt(static_cast<size_t>(m));
  for (size_t k = 0; k < pl.rows.size(); ++k) {
    const Row& r = pl.rows[k];
    for (int64_t t = 0; t < m; ++t) y[static_cast<size_t>(t)] = Y[static_cast<int64_t>(k) * m + t];
    dft(m, y.data(), Yt.data(), -1);
    for (int64_t c = r.lo; c <= r.hi; ++c) {
      const cd tile = scale * Yt[static_cast<size_t>(wrap(c - r.s, m))];
      acc[static_cast<size_t>(c)] += tile * r.w[static_cast<size_t>(c - r.lo)];
    }
  }
  std::vector<cd> Xh(static_cast<size_t>(pl.nbins), cd(0.0, 0.0));
  for (int64_t b = 0; b < pl.nbins; ++b)
    if (pl.M[static_cast<size_t>(b)]) Xh[static_cast<size_t>(b)] = acc[static_cast<size_t>(b)] / pl.P[static_cast<size_t>(b)];
  synthesis_real(pl, Xh, x);
}

// The plain definition of a dense (full-rate) tile, App. C:
// T_k[tau] = (1/N) sum_b X[b] W_k[b] e^{+2 pi i b tau/N} over the one-sided
// spectrum, tau = 0..N-1, computed by direct summation of its support.
void dense_one(const Plan& pl, const double* x, cd* T) {
  std::vector<cd> X;
  spectrum(pl, x, X);
  const int64_t n = pl.n;
  for (size_t k = 0; k < pl.rows.size(); ++k) {
    const Row& r = pl.rows[k];
    for (int64_t t = 0; t < n; ++t) {
      cd acc(0.0, 0.0);
      for (int64_t c = r.lo; c <= r.hi; ++c) {
        const int64_t e = static_cast<int64_t>((static_cast<__int128>(c) * t) % n);
        const double ang = 2.0 * kPi * static_cast<double>(e) / static_cast<double>(n);
        acc += X[static_cast<size_t>(c)] * r.w[static_cast<size_t>(c - r.lo)] * cd(std::cos(ang), std::sin(ang));
      }
      T[static_cast<int64_t>(k) * n + t] = acc / static_cast<double>(n);
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface, loaded by the tests through ctypes. Complex arrays are
// interleaved (re, im) doubles. Envelopes are [batch, R, N_out]; dense tiles
// [R, N]; signals [batch, N].
// ---------------------------------------------------------------------------
extern "C" {

// n_planes > 0: plane p has quality factor qs[p], window windows[p] with
// parameter params[p]; otherwise one plane (q, window, window_param).
void* ora_plan_create(double fs, int64_t n, double q, double fmin, double fmax, int32_t nrows,
                      const double* freqs, int32_t window, double window_param, int32_t cap_mode,
                      int32_t max_window, int32_t norm_mode, int32_t n_out, double tau,
                      int32_t n_planes, const double* qs, const int32_t* windows, const double* params,
                      double eps) {
  std::vector<PlaneSpec> planes;
  if (n_planes > 0)
    for (int32_t p = 0; p < n_planes; ++p) planes.push_back(PlaneSpec{qs[p], windows[p], params[p]});
  else
    planes.push_back(PlaneSpec{q, window, window_param});
  Plan* pl = new Plan();
  if (build_plan(*pl, fs, n, planes, fmin, fmax, nrows, freqs, cap_mode, max_window, norm_mode, n_out,
                 tau, eps) != 0) {
    delete pl;
    return nullptr;
  }
  return pl;
}

void ora_plan_destroy(void* h) { delete static_cast<Plan*>(h); }

// sizes[0] = R, [1] = N_out, [2] = N/2+1, [3] = L_max (-1: none), [4] = max L_k,
// [5] = sum of kept support lengths
void ora_plan_sizes(void* h, int64_t* sizes) {
  const Plan& pl = *static_cast<Plan*>(h);
  int64_t mx = 0, sum = 0;
  for (const Row& r : pl.rows) {
    // longest row: its window's support, or the whole band with a stop band
    mx = std::max(mx, pl.eps > 0.0 ? pl.nbins : 2 * r.h + 1);
    sum += r.hi - r.lo + 1;
  }
  sizes[0] = static_cast<int64_t>(pl.rows.size());
  sizes[1] = pl.n_out;
  sizes[2] = pl.nbins;
  sizes[3] = pl.l_max;
  sizes[4] = mx;
  sizes[5] = sum;
}

// Per row: freq, centre, half width, lo, hi.
void ora_plan_rows(void* h, double* freq, int64_t* centre, int64_t* half, int64_t* lo, int64_t* hi) {
  const Plan& pl = *static_cast<Plan*>(h);
  for (size_t k = 0; k < pl.rows.size(); ++k) {
    freq[k] = pl.rows[k].f;
    centre[k] = pl.rows[k].s;
    half[k] = pl.rows[k].h;
    lo[k] = pl.rows[k].lo;
    hi[k] = pl.rows[k].hi;
  }
}

// Dense window matrix W[R][N/2+1] (zeros off the support).
void ora_plan_windows(void* h, double* W) {
  const Plan& pl = *static_cast<Plan*>(h);
  std::memset(W, 0, sizeof(double) * pl.rows.size() * static_cast<size_t>(pl.nbins));
  for (size_t k = 0; k < pl.rows.size(); ++k) {
    const Row& r = pl.rows[k];
    for (int64_t c = r.lo; c <= r.hi; ++c)
      W[k * static_cast<size_t>(pl.nbins) + static_cast<size_t>(c)] = r.w[static_cast<size_t>(c - r.lo)];
  }
}

void ora_plan_frame(void* h, double* P, unsigned char* M) {
  const Plan& pl = *static_cast<Plan*>(h);
  std::copy(pl.P.begin(), pl.P.end(), P);
  std::copy(pl.M.begin(), pl.M.end(), M);
}

void ora_set_force_direct(int32_t on) { g_force_direct = on != 0; }

// Complex DFT of length n: sign -1 forward, +1 unnormalised inverse kernel.
void ora_dft(int64_t n, const double* in, double* out, int32_t sign) {
  dft(n, reinterpret_cast<const cd*>(in), reinterpret_cast<cd*>(out), sign);
}

void ora_spectrum(void* h, const double* x, int64_t batch, double* X) {
  const Plan& pl = *static_cast<Plan*>(h);
  std::vector<cd> s;
  for (int64_t b = 0; b < batch; ++b) {
    spectrum(pl, x + b * pl.n, s);
    std::copy(s.begin(), s.end(), reinterpret_cast<cd*>(X) + b * pl.nbins);
  }
}

void ora_forward(void* h, const double* x, int64_t batch, double* Y) {
  const Plan& pl = *static_cast<Plan*>(h);
  const int64_t per = static_cast<int64_t>(pl.rows.size()) * pl.n_out;
  for (int64_t b = 0; b < batch; ++b)
    forward_one(pl, x + b * pl.n, reinterpret_cast<cd*>(Y) + b * per);
}

// Forward coefficients of the rows idx[0..count) only (sampled rows of
// plans too large for every row): Y [batch, count, N_out]. Returns 1 if an
// index is out of range.
int ora_forward_rows(void* h, const double* x, int64_t batch, const int64_t* idx, int64_t count, double* Y) {
  const Plan& pl = *static_cast<Plan*>(h);
  for (int64_t i = 0; i < count; ++i)
    if (idx[i] < 0 || idx[i] >= static_cast<int64_t>(pl.rows.size())) return 1;
  for (int64_t b = 0; b < batch; ++b)
    forward_rows(pl, x + b * pl.n, idx, count, reinterpret_cast<cd*>(Y) + b * count * pl.n_out);
  return 0;
}

void ora_inverse(void* h, const double* Y, int64_t batch, double* x) {
  const Plan& pl = *static_cast<Plan*>(h);
  const int64_t per = static_cast<int64_t>(pl.rows.size()) * pl.n_out;
  for (int64_t b = 0; b < batch; ++b)
    inverse_one(pl, reinterpret_cast<const cd*>(Y) + b * per, x + b * pl.n);
}

void ora_dense(void* h, const double* x, double* T) {
  dense_one(*static_cast<Plan*>(h), x, reinterpret_cast<cd*>(T));
}

// Recovery of the signal from the single tile k by spectral division
// (Sec. III, regularised windows): the row's kept slots give
// X[c] W_k[c] = sqrt(N/N_out) DFT_{N_out}(Y_k)[(c - s_k) mod N_out]; divide by
// W_k[c] on every kept bin (zero elsewhere) and return to the time domain.
// Y: [batch, R, N_out]; x: [batch, N]. Returns 1 if a kept W_k[c] is 0.
int ora_tile_inverse(void* h, const double* Y, int32_t k, int64_t batch, double* x) {
  const Plan& pl = *static_cast<Plan*>(h);
  const int64_t R = static_cast<int64_t>(pl.rows.size()), M = pl.n_out;
  if (k < 0 || k >= R) return 1;
  const Row& r = pl.rows[static_cast<size_t>(k)];
  const cd* Yc = reinterpret_cast<const cd*>(Y);
  const double amp = std::sqrt(static_cast<double>(pl.n) / static_cast<double>(M));
  std::vector<cd> F(static_cast<size_t>(M));
  for (int64_t b = 0; b < batch; ++b) {
    dft(M, Yc + (b * R + k) * M, F.data(), -1);
    std::vector<cd> Xh(static_cast<size_t>(pl.nbins), cd(0.0, 0.0));
    for (int64_t c = r.lo; c <= r.hi; ++c) {
      const double w = r.w[static_cast<size_t>(c - r.lo)];
      if (w == 0.0) return 1;
      const int64_t u = ((c - r.s) % M + M) % M;
      Xh[static_cast<size_t>(c)] = amp * F[static_cast<size_t>(u)] / w;
    }
    synthesis_real(pl, Xh, x + b * pl.n);
  }
  return 0;
}

// Real-signal synthesis from a one-sided spectrum (irfft convention).
void ora_synthesis(void* h, const double* Xh, int64_t batch, double* x) {
  const Plan& pl = *static_cast<Plan*>(h);
  for (int64_t b = 0; b < batch; ++b) {
    std::vector<cd> s(reinterpret_cast<const cd*>(Xh) + b * pl.nbins,
                      reinterpret_cast<const cd*>(Xh) + (b + 1) * pl.nbins);
    synthesis_real(pl, s, x + b * pl.n);
  }
}

}  // extern "C"
