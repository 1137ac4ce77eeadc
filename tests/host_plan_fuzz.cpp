// Host plan builder under AddressSanitizer and UndefinedBehaviorSanitizer:
// builds the FP64 plan tables (paper_2603_29785_amd/csrc/plan.cpp, host code
// only) for the workload plans, edge cases and seeded random parameter sets,
// and checks the invariants every device launch relies on. Compiled and run
// by tests/test_host_sanitizers.py with g++ (no device code is involved).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "plan.hpp"

namespace {

int g_failures = 0;

void expect(bool ok, const char* what, int64_t id) {
  if (!ok) {
    std::printf("FAIL case %lld: %s\n", static_cast<long long>(id), what);
    ++g_failures;
  }
}

qtam_params base(double fs, int64_t n, double q, double fmin, double fmax, int32_t rows) {
  qtam_params p{};
  p.sample_rate = fs;
  p.n_samples = n;
  p.q = q;
  p.f_min = fmin;
  p.f_max = fmax;
  p.n_rows = rows;
  p.p_floor_rel = 1e-6;
  return p;
}

// Structural invariants of a built plan (the kernels index with them).
void check(const qtam_params& p, int64_t id) {
  qtam::HostPlan hp;
  const qtam_status st = qtam::build_host_plan(p, hp);
  if (st != QTAM_OK) return;   // rejected parameters: nothing to check
  expect(hp.n_bins == hp.half + 1, "bins", id);
  expect(static_cast<int64_t>(hp.centre.size()) == hp.rows, "rows", id);
  int64_t off = 0, longest = 0;
  for (int32_t k = 0; k < hp.rows; ++k) {
    expect(hp.lo[k] >= 0 && hp.lo[k] <= hp.hi[k] && hp.hi[k] <= hp.half, "support in 0..N/2", id);
    expect(hp.offset[k] == off, "packed offsets", id);
    off += hp.hi[k] - hp.lo[k] + 1;
    longest = std::max<int64_t>(longest, hp.hi[k] - hp.lo[k] + 1);
  }
  expect(off == hp.sum_len, "sum of supports", id);
  expect(longest <= hp.n_out, "support fits N_out", id);
  expect(static_cast<int64_t>(hp.win.size()) == hp.sum_len && static_cast<int64_t>(hp.dual_tab.size()) == hp.sum_len,
         "table sizes", id);
  for (int64_t e = 0; e < hp.sum_len; ++e)
    expect(std::isfinite(hp.fwd_tab[e]) && std::isfinite(hp.dual_tab[e]) && std::isfinite(hp.afwd_tab[e]) &&
               std::isfinite(hp.ainv_tab[e]) && std::isfinite(hp.tile_tab[e]),
           "finite tables", id);
  expect(static_cast<int64_t>(hp.P.size()) == hp.n_bins && static_cast<int64_t>(hp.M.size()) == hp.n_bins,
         "frame sizes", id);
}

}  // namespace

int main() {
  int64_t id = 0;
  // the workload plans
  check(base(4096.0, 16384, 8.0, 20.0, 1000.0, 64), id++);
  for (double q : {4.0, 8.0, 16.0}) check(base(4096.0, 131072, q, 10.0, 2048.0, 256), id++);
  check(base(8192.0, 1 << 21, 12.0, 5.0, 4096.0, 512), id++);
  check(base(4096.0, 32768, 8.0, 20.0, 2000.0, 128), id++);
  // edge cases: one row, tiny N, band at DC and Nyquist, duplicate centres,
  // literal and manual caps, no cap, odd N_out, regularised windows, banks
  check(base(256.0, 16, 2.0, 1.0, 128.0, 1), id++);
  check(base(256.0, 16, 2.0, 16.0, 128.0, 7), id++);
  check(base(1.0, 64, 32.0, 0.01, 0.02, 40), id++);
  {
    qtam_params p = base(4096.0, 24576, 8.0, 20.0, 2000.0, 62);
    p.cap_mode = QTAM_CAP_PAPER;
    check(p, id++);
    p.n_out = 669;
    check(p, id++);
    p.cap_mode = QTAM_CAP_MANUAL;
    p.max_window = 7;
    p.n_out = 0;
    check(p, id++);
    p.cap_mode = QTAM_CAP_NONE;
    check(p, id++);
    p.cap_mode = QTAM_CAP_COVER;
    p.window_eps = 1e-3;
    check(p, id++);
  }
  {
    const double qs[3] = {4.0, 8.0, 16.0};
    const int32_t ws[3] = {QTAM_WIN_BISQUARE, QTAM_WIN_KAISER, QTAM_WIN_PLANCK};
    const double ps[3] = {0.0, 5.0, 0.25};
    qtam_params p = base(4096.0, 32768, 1.0, 20.0, 2000.0, 24);
    p.n_planes = 3;
    p.plane_q = qs;
    p.plane_window = ws;
    p.plane_window_param = ps;
    check(p, id++);
  }
  {
    const double fr[5] = {10.0, 10.0, 10.1, 200.0, 2048.0};
    qtam_params p = base(4096.0, 8192, 4.0, 10.0, 2048.0, 5);
    p.freqs = fr;
    check(p, id++);
  }
  // invalid parameters are rejected without touching anything
  check(base(0.0, 1024, 8.0, 10.0, 100.0, 8), id++);
  check(base(1024.0, 1023, 8.0, 10.0, 100.0, 8), id++);
  check(base(1024.0, 1024, -1.0, 10.0, 100.0, 8), id++);
  // seeded random parameter sets
  std::mt19937_64 rng(2026);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  for (int i = 0; i < 400; ++i) {
    const int r = (i % 3 == 0) ? 1 : (i % 3 == 1 ? 3 : 5);
    const int64_t n = r * (int64_t(1) << (4 + rng() % 13));
    const double fs = 256.0 * (1 << (rng() % 5));
    const double nyq = fs / 2;
    const double fmin = (0.001 + 0.3 * u(rng)) * nyq;
    const double fmax = fmin + (nyq - fmin) * u(rng);
    qtam_params p = base(fs, n, 0.5 + 40.0 * u(rng), fmin, fmax, 1 + int32_t(rng() % 300));
    p.window = int32_t(rng() % 5);
    p.window_param = p.window == QTAM_WIN_KAISER ? 8.0 * u(rng) : u(rng);
    p.cap_mode = int32_t(rng() % 3);
    p.norm_mode = int32_t(rng() % 3);
    if (rng() % 4 == 0) p.window_eps = 1e-4;
    if (rng() % 3 == 0) {
      qtam::HostPlan probe;
      if (qtam::build_host_plan(p, probe) == QTAM_OK) p.n_out = probe.max_len + int32_t(rng() % 7);
    }
    p.precision = int32_t(rng() % 2);
    check(p, id++);
  }
  std::printf("%lld plans checked, %d failures\n", static_cast<long long>(id), g_failures);
  return g_failures == 0 ? 0 : 1;
}
