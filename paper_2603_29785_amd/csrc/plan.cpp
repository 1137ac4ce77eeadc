// Host construction of the QTAM plan tables in FP64.
//
// Grid, centre, width and cap follow App. A of the paper; windows and their
// normalisation follow the window equations of Sec. II and App. A; the frame
// operator P and the canonical dual follow App. C. The integer parts (centre
// bins, half widths, cap) are evaluated with the same floating-point
// expressions the reference definition uses, so that every implementation of
// the method lands on the same integers:
//   T = N / fs;  f_k = f_min * (f_max/f_min)^(k/(R-1));  s_k = floor(f_k T + 1/2);
//   g = ceil(T * max_k(f_{k+1} - f_k));  h_k = floor(ceil(f_k T / Q) / 2).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace qtam {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Window value at relative position x = j/h in [-1, 1].
double shape(int32_t kind, double x, double a) {
  const double ax = std::fabs(x);
  if (ax > 1.0) return 0.0;
  if (kind == QTAM_WIN_BISQUARE) {
    const double u = (1.0 - ax) * (1.0 + ax);
    return u * u;
  }
  if (kind == QTAM_WIN_HANN) return 0.5 + 0.5 * std::cos(0.5 * kTwoPi * x);
  if (kind == QTAM_WIN_KAISER) {
    // I0(beta) once per beta (every bin of a plane shares it)
    thread_local double beta = std::numeric_limits<double>::quiet_NaN(), i0_beta = 1.0;
    if (!(a == beta)) {
      beta = a;
      i0_beta = std::cyl_bessel_i(0.0, a);
    }
    const double r = std::sqrt(std::max(0.0, (1.0 - ax) * (1.0 + ax)));
    return std::cyl_bessel_i(0.0, a * r) / i0_beta;
  }
  if (kind == QTAM_WIN_TUKEY) {
    const double flat = 1.0 - a;
    if (a <= 0.0 || ax <= flat) return 1.0;
    return 0.5 + 0.5 * std::cos(0.5 * kTwoPi * (ax - flat) / a);
  }
  if (kind == QTAM_WIN_PLANCK) {
    // logistic taper 1/(1+e^z), z = 1/u - 1/(1-u), u = (1-|x|)/alpha the
    // depth into the taper: 0 at the window edge, 1 where the flat top starts
    if (ax >= 1.0) return 0.0;
    const double flat = 1.0 - a;
    if (a <= 0.0 || ax <= flat) return 1.0;
    const double u = (1.0 - ax) / a;
    const double z = 1.0 / u - 1.0 / (1.0 - u);
    return z > 700.0 ? 0.0 : 1.0 / (1.0 + std::exp(z));
  }
  return 0.0;
}

int64_t pow2_at_least(int64_t v) {
  int64_t p = 1;
  while (p < v) p *= 2;
  return p;
}

}  // namespace

qtam_status build_host_plan(const qtam_params& p, HostPlan& hp) {
  const int64_t n = p.n_samples;
  if (!(p.sample_rate > 0.0) || n < 16 || (n & 1) || p.n_rows < 1 || p.n_planes < 0)
    return QTAM_ERR_INVALID_ARG;
  // planes of the bank: (Q, window, parameter)
  struct Plane {
    double q;
    int32_t window;
    double param;
  };
  std::vector<Plane> planes;
  if (p.n_planes == 0) {
    planes.push_back(Plane{p.q, p.window, p.window_param});
  } else {
    if (!p.plane_q || !p.plane_window || !p.plane_window_param) return QTAM_ERR_INVALID_ARG;
    for (int32_t i = 0; i < p.n_planes; ++i)
      planes.push_back(Plane{p.plane_q[i], p.plane_window[i], p.plane_window_param[i]});
  }
  if (int64_t(planes.size()) * p.n_rows > std::numeric_limits<int32_t>::max()) return QTAM_ERR_INVALID_ARG;
  for (const Plane& pl : planes) {
    if (!(pl.q > 0.0)) return QTAM_ERR_INVALID_ARG;
    if (pl.window < QTAM_WIN_BISQUARE || pl.window > QTAM_WIN_PLANCK) return QTAM_ERR_INVALID_ARG;
  }
  if (p.precision != QTAM_FP32 && p.precision != QTAM_FP64) return QTAM_ERR_INVALID_ARG;
  if (p.n_out < 0 || !(p.p_floor_rel >= 0.0) || p.p_floor_rel > 1.0) return QTAM_ERR_INVALID_ARG;
  if (!(p.window_eps >= 0.0)) return QTAM_ERR_INVALID_ARG;

  hp = HostPlan();
  hp.fs = p.sample_rate;
  hp.q = planes[0].q;
  hp.f_min = p.f_min;
  hp.f_max = p.f_max;
  hp.p_floor_rel = p.p_floor_rel;
  hp.window = planes[0].window;
  hp.window_param = planes[0].param;
  hp.eps = p.window_eps;
  for (const Plane& pl : planes) hp.all_bisquare = hp.all_bisquare && pl.window == QTAM_WIN_BISQUARE;
  hp.n = n;
  hp.half = n / 2;
  hp.n_bins = n / 2 + 1;
  hp.planes = static_cast<int32_t>(planes.size());
  hp.rows_per_plane = p.n_rows;
  hp.rows = hp.planes * p.n_rows;
  hp.precision = p.precision;
  const int32_t R = p.n_rows;      // rows of one plane
  const double T = static_cast<double>(n) / p.sample_rate;

  // Frequency grid.
  hp.freq.resize(R);
  if (p.freqs) {
    std::copy(p.freqs, p.freqs + R, hp.freq.begin());
  } else {
    if (!(p.f_min > 0.0) || !(p.f_max >= p.f_min)) return QTAM_ERR_INVALID_ARG;
    const double ratio = p.f_max / p.f_min;
    for (int32_t k = 0; k < R; ++k)
      hp.freq[k] = R == 1 ? p.f_min
                          : p.f_min * std::pow(ratio, static_cast<double>(k) / static_cast<double>(R - 1));
  }
  for (int32_t k = 0; k < R; ++k) {
    if (!(hp.freq[k] > 0.0) || hp.freq[k] > 0.5 * p.sample_rate) return QTAM_ERR_INVALID_ARG;
    if (k && hp.freq[k] < hp.freq[k - 1]) return QTAM_ERR_INVALID_ARG;
  }

  // Cap on window length.
  switch (p.cap_mode) {
    case QTAM_CAP_NONE: hp.l_max = -1; break;
    case QTAM_CAP_MANUAL:
      if (p.max_window < 1) return QTAM_ERR_INVALID_ARG;
      hp.l_max = p.max_window;
      break;
    case QTAM_CAP_COVER:
    case QTAM_CAP_PAPER: {
      if (R < 2) { hp.l_max = -1; break; }
      double gap = 0.0;
      for (int32_t k = 1; k < R; ++k) gap = std::max(gap, hp.freq[k] - hp.freq[k - 1]);
      const int64_t g = static_cast<int64_t>(std::ceil(T * gap));
      hp.l_max = p.cap_mode == QTAM_CAP_COVER ? 2 * g + 1 : 2 * (g / 2) + 1;
      break;
    }
    default: return QTAM_ERR_INVALID_ARG;
  }

  // Rows of every plane: centre, width, kept support, packed window.
  const int32_t RT = hp.rows;
  hp.freq.resize(RT);
  for (int32_t k = R; k < RT; ++k) hp.freq[k] = hp.freq[k % R];
  hp.row_q.resize(RT);
  hp.centre.resize(RT);
  hp.half_width.resize(RT);
  hp.lo.resize(RT);
  hp.hi.resize(RT);
  hp.offset.resize(RT);
  int64_t longest = 0;
  for (int32_t k = 0; k < RT; ++k) {
    const Plane& plane = planes[k / R];
    hp.row_q[k] = plane.q;
    const double f = hp.freq[k];
    const int64_t s = static_cast<int64_t>(std::floor(f * T + 0.5));
    int64_t h = std::max<int64_t>(1, static_cast<int64_t>(std::ceil(f * T / plane.q)) / 2);
    if (hp.l_max > 0) h = std::max<int64_t>(1, std::min<int64_t>(h, hp.l_max / 2));
    // kept bins: the support clipped to 0..N/2, or the whole band with a stop band
    const int64_t a = hp.eps > 0.0 ? 0 : std::max<int64_t>(0, s - h);
    const int64_t b = hp.eps > 0.0 ? hp.half : std::min<int64_t>(hp.half, s + h);
    if (a > b || h > std::numeric_limits<int32_t>::max() / 4) return QTAM_ERR_INVALID_ARG;
    hp.centre[k] = static_cast<int32_t>(s);
    hp.half_width[k] = static_cast<int32_t>(h);
    hp.lo[k] = static_cast<int32_t>(a);
    hp.hi[k] = static_cast<int32_t>(b);
    hp.offset[k] = hp.sum_len;
    hp.sum_len += b - a + 1;
    longest = std::max(longest, hp.eps > 0.0 ? hp.half + 1 : 2 * h + 1);

    double e2 = 0.0;
    const size_t base = hp.win.size();
    // every shape depends on |x| only: each offset |c - s| is evaluated once
    // (x = -j/h and j/h give the same |x| bits)
    std::vector<double> at(static_cast<size_t>(h) + 1, -1.0);
    for (int64_t c = a; c <= b; ++c) {
      const bool inside = c >= s - h && c <= s + h;
      double w = 0.0;
      if (inside) {
        const size_t j = static_cast<size_t>(c >= s ? c - s : s - c);
        if (at[j] < 0.0) at[j] = shape(plane.window, static_cast<double>(j) / static_cast<double>(h), plane.param);
        w = at[j];
      }
      if (hp.eps > 0.0 && w < hp.eps) w = hp.eps;   // floor: the stop band, end points, tails below eps
      hp.win.push_back(w);
      e2 += w * w;
    }
    if (!(e2 > 0.0)) return QTAM_ERR_INVALID_ARG;   // the row keeps no energy
    double norm;
    switch (p.norm_mode) {
      case QTAM_NORM_UNIT_ENERGY: norm = 1.0 / std::sqrt(e2); break;
      case QTAM_NORM_PAPER_INV_ENERGY: norm = 1.0 / e2; break;
      case QTAM_NORM_NONE: norm = 1.0; break;
      default: return QTAM_ERR_INVALID_ARG;
    }
    for (size_t i = base; i < hp.win.size(); ++i) hp.win[i] *= norm;
  }
  if (hp.sum_len >= (int64_t(1) << 31)) return QTAM_ERR_INVALID_ARG;
  hp.max_len = static_cast<int32_t>(longest);

  // Envelope length.
  if (p.n_out == 0) {
    hp.n_out = static_cast<int32_t>(pow2_at_least(longest));
  } else {
    if (p.n_out < longest) return QTAM_ERR_INVALID_ARG;
    hp.n_out = p.n_out;
  }

  // Frame operator and mask.
  hp.P.assign(hp.n_bins, 0.0);
  for (int32_t k = 0; k < RT; ++k)
    for (int64_t c = hp.lo[k]; c <= hp.hi[k]; ++c) {
      const double w = hp.win[hp.offset[k] + (c - hp.lo[k])];
      hp.P[c] += w * w;
    }
  const double pmax = *std::max_element(hp.P.begin(), hp.P.end());
  const double floor_abs = p.p_floor_rel * pmax;
  hp.M.assign(hp.n_bins, 0);
  hp.frame_A = std::numeric_limits<double>::infinity();
  hp.frame_B = 0.0;
  int64_t masked = 0;
  for (int64_t b = 0; b < hp.n_bins; ++b) {
    const bool keep = hp.P[b] > 0.0 && hp.P[b] >= floor_abs;
    hp.M[b] = keep ? 1 : 0;
    if (keep) {
      hp.frame_A = std::min(hp.frame_A, hp.P[b]);
      hp.frame_B = std::max(hp.frame_B, hp.P[b]);
    } else {
      ++masked;
    }
  }
  if (!(hp.frame_B > 0.0)) hp.frame_A = 0.0;
  hp.masked_fraction = static_cast<double>(masked) / static_cast<double>(hp.n_bins);

  // Per-entry scale tables.
  const double nn = static_cast<double>(n), no = static_cast<double>(hp.n_out);
  const double fwd_scale = std::sqrt(no / nn) / no;
  const double inv_scale = std::sqrt(nn / no);
  hp.fwd_tab.resize(hp.sum_len);
  hp.dual_tab.resize(hp.sum_len);
  hp.afwd_tab.resize(hp.sum_len);
  hp.ainv_tab.resize(hp.sum_len);
  hp.tile_tab.assign(hp.sum_len, 0.0);
  for (int32_t k = 0; k < RT; ++k)
    for (int64_t c = hp.lo[k]; c <= hp.hi[k]; ++c) {
      const int64_t e = hp.offset[k] + (c - hp.lo[k]);
      const double w = hp.win[e];
      const bool edge = (c == 0 || c == hp.half);
      const double dual = hp.M[c] ? inv_scale * w / hp.P[c] : 0.0;
      hp.fwd_tab[e] = w * fwd_scale;
      hp.dual_tab[e] = dual / nn;
      hp.afwd_tab[e] = w * fwd_scale * (edge ? 1.0 : 0.5);
      hp.ainv_tab[e] = dual * (edge ? 1.0 : 2.0) / nn;
      if (hp.eps > 0.0) hp.tile_tab[e] = inv_scale / (w * nn);
    }
  return QTAM_OK;
}

}  // namespace qtam
