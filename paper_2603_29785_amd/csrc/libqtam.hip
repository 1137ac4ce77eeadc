// libqtam: QTAM forward / inverse transform on gfx950 (MI355X), host side.
// Plan upload, workspace layout, kernel dispatch and the C ABI of qtam.h; the
// kernels themselves are in spectrum_kernels.hpp, row_kernels.hpp and
// ola_kernels.hpp.
//
// Forward (Sec. III; App. A):
//   1. spectrum: the N real samples of a segment, read as N/2 complex pairs
//      z[m] = x[2m] + i x[2m+1], go through an N/2-point complex FFT
//      (one LDS pass when N/2 fits a workgroup, else two passes of the
//      four-step factorisation N/2 = N1 * N2 through the workspace), and the
//      real-signal twist gives X[0..N/2] (fused into the second pass);
//   2. rows: one fused kernel per (segment, row) gathers X over the row's
//      kept support, multiplies by the window, drops each bin at its baseband
//      slot (c - s_k) mod N_out (roll to baseband, crop, zero pad) and runs
//      the N_out-point inverse FFT in registers and LDS, storing the envelope
//      row coalesced.
// Inverse (Sec. III canonical dual; App. C):
//   1. rows: N_out-point FFT of each envelope row; the kept slots, weighted
//      by the dual table sqrt(N/N_out) W M / P / N, go to a packed buffer;
//   2. overlap-add: each wave sums the covering rows of its bins and their
//      mirrors N/2 - b in fixed row order (no atomics) and applies the
//      real-signal pre-twist, giving the N/2-point half-size spectrum;
//   3. synthesis: N/2-point inverse FFT whose complex output, read as pairs
//      of reals, is the time series.
// The adjoints reuse the same kernels with other tables (App. C: the
// adjoint of analysis is synthesis).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <string>
#include <new>
#include <vector>

#include "mask_kernels.hpp"
#include "ola_kernels.hpp"
#include "plan.hpp"
#include "qtam.h"
#include "row_kernels.hpp"
#include "spectrum_kernels.hpp"

// ===========================================================================
// Host side: plan object, dispatch, C ABI
// ===========================================================================
using namespace qtam;

namespace {

enum Kind { K_SPEC = 0, K_SPEC1, K_SPEC2, K_TWIST, K_FWD_ROWS, K_FWD_ROWS2, K_INV_ROWS, K_INV_ROWS2, K_OLA,
            K_SYN, K_SYN1, K_SYN2, K_ROW_STATS, K_PLANE_BEST, K_GATHER, K_SPEC_PERM, K_SPEC_RADIX, K_SYN_RADIX,
            K_SYN_PERM, K_DENSE_PLACE, K_DENSE_FFT, K_DENSE_FFT1, K_DENSE_FFT2, K_DENSE_RADIX, K_DENSE_PERM,
            K_MASK_FWD, K_MASK_BWD, K_NUM };
const char* const kKindName[K_NUM] = {"spectrum_fft", "spectrum_fft_pass1", "spectrum_fft_pass2",
                                       "spectrum_twist", "fwd_rows", "fwd_rows_pass2", "inv_rows",
                                       "inv_rows_pass2", "overlap_add", "synthesis_fft",
                                       "synthesis_fft_pass1", "synthesis_fft_pass2", "row_stats",
                                       "plane_best", "gather_plane", "spectrum_permute", "spectrum_radix",
                                       "synthesis_radix", "synthesis_permute", "dense_place", "dense_fft",
                                       "dense_fft_pass1", "dense_fft_pass2", "dense_radix", "dense_permute",
                                       "mask_forward", "mask_backward"};

enum Table { T_FWD = 0, T_DUAL = 1, T_AFWD = 2, T_AINV = 3, T_DENSE = 4, T_TILE = 5 };

constexpr int kMaxLog2Single32 = 14;   // LDS-resident FFT up to 16384 points (FP32)
constexpr int kMaxLog2Single64 = 13;   // and 8192 points (FP64)
// Envelope rows in one workgroup: up to 32768 points in FP32 (1024 threads x
// 32 values, exchanges through LDS in two halves), 8192 in FP64.
constexpr int kMaxLog2Rows32 = 15;
constexpr int kMaxLog2Rows64 = 13;
// Values per thread of the second four-step pass of the spectrum and
// synthesis transforms (its twiddle table, d_tw_n1, is built for it).
constexpr int kPass2E = 8;
// Columns per workgroup of the first four-step pass, and rows per workgroup
// of the second, where the LDS and the 1024-thread limit allow it (else 16):
// longer contiguous runs per access. Measured: 32 columns faster than 16 in
// the first pass of the spectrum and synthesis transforms, 64 slower; 32
// rows faster in the spectrum's fused twist pass and the row passes with
// sixteen (FP32) or eight (FP64) values per thread, slower in the synthesis
// second pass with eight values per thread in FP32, which keeps 16.
constexpr int kColWide = 32;
constexpr int kRowWide = 32;

int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Text of the last HIP failure seen on this thread (qtam_last_error).
thread_local std::string g_last_error;

// Set while qtam_forward_noalloc runs on this thread: its launches are not
// timed (timing may create events).
thread_local bool g_untimed = false;

qtam_status hip_failed(hipError_t e, const char* what, qtam_status st = QTAM_ERR_DEVICE) {
  g_last_error = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  (void)hipGetLastError();
  return st;
}

}  // namespace

struct qtam_plan_s {
  HostPlan hp;
  bool device = false;
  int device_id = -1;
  char* dmem = nullptr;         // one allocation holding every device table
  // device table pointers (precision of the plan)
  RowMeta* d_rows = nullptr;
  void* d_roww = nullptr;       // per row (scale, 1/h) of the analytic forward weight
  int* d_ola_start = nullptr;   // [2 * ola_waves + 1] start of each overlap-add wave side's row list
  OlaRow* d_ola_rows = nullptr; // rows meeting each wave side's bins, ascending
  int ola_waves = 0;            // waves of 64 bins covering p = 0 .. N/4
  int* d_one_start = nullptr;   // overlap-add lists of a single row over all bins
  OlaRow* d_one_rows = nullptr;
  void* d_tab[6] = {};
  void* d_tw_out = nullptr;     // N_out, TW_MIXED layout (the row kernels)
  void* d_tw_half = nullptr;    // M2 (single pass) or nullptr
  void* d_tw_n1 = nullptr;      // N1 (four-step, second pass length)
  void* d_tw_n2 = nullptr;      // N2 (four-step, first pass length)
  void* d_tw2_fine = nullptr;
  void* d_tw2_coarse = nullptr;
  int tw2_bits = 0;
  bool four_step = false;       // the length-M2 transforms run as two passes
  int64_t n1 = 0, n2 = 0;       // M2 = n1 * n2 when four_step
  bool dense_ok = false;        // dense tiles available
  int64_t dense_md = 0;         // N = radix_r * dense_md: power-of-two part of the N-point transforms
  bool dense_four_step = false; // dense_md-point transforms in two passes, dense_md = dn1 * dn2
  int64_t dn1 = 0, dn2 = 0;
  void* d_tw_dense = nullptr;   // Stockham twiddles of dense_md (single pass)
  void* d_tw_dn1 = nullptr;
  void* d_tw_dn2 = nullptr;
  bool bluestein = false;       // N_out not a power of two: chirp-z rows of length bs_len
  int64_t bs_len = 0;
  void* d_bs_chirp = nullptr;   // [N_out] e^{+pi i v^2 / N_out}
  void* d_bs_bf = nullptr;      // [bs_len] FFT of the wrapped conjugate chirp / bs_len (forward rows)
  void* d_bs_bi = nullptr;      // [bs_len] FFT of the wrapped chirp / bs_len (inverse rows)
  void* d_bs_tw = nullptr;      // Stockham twiddles of bs_len
  int radix_r = 1;              // N/2 = radix_r * m2
  int64_t m2 = 0;               // power-of-two transform length of the spectrum
  bool big_rows = false;        // N_out beyond one workgroup: four-step rows through the workspace
  bool bs_long = false;         // chirp-z rows whose bs_len exceeds one workgroup: element passes
                                // around four-step transforms through the workspace
  int64_t r1 = 0, r2 = 0;       // N_out = r1 * r2 (big_rows), bs_len = r1 * r2 (bs_long)
  void* d_tw_r1 = nullptr;
  void* d_tw_r2 = nullptr;
  void* d_twr_fine = nullptr;   // two-level exp(-2 pi i m / N_out)
  void* d_twr_coarse = nullptr;
  int twr_bits = 0;
  bool gpu_supported = false;
  bool analytic_fwd = false;    // bisquare: forward weights computed in the kernel
  int num_cus = 0;
  qtam_status unsupported_reason = QTAM_OK;
  size_t seg_bytes = 0;         // workspace per segment (max over operations)
  // host info arrays
  std::vector<int64_t> info_offset;
  // timing
  std::mutex mu;
  bool timing = false;
  struct Pending { int kind; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[K_NUM] = {};
  int64_t launches[K_NUM] = {};
};

namespace {

// ---------------------------------------------------------------------------
// Table construction for the device
// ---------------------------------------------------------------------------
// In-place forward DFT (e^{-2 pi i k n / L}) of a power-of-two length in
// FP64 on the host: bit reversal, then butterflies with every twiddle from
// its own angle.
void host_fft(std::vector<std::complex<double>>& a) {
  const int64_t n = static_cast<int64_t>(a.size());
  for (int64_t i = 1, j = 0; i < n; ++i) {
    int64_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (int64_t len = 2; len <= n; len <<= 1)
    for (int64_t i = 0; i < n; i += len)
      for (int64_t k = 0; k < len / 2; ++k) {
        const std::complex<double> w = std::polar(1.0, -2.0 * M_PI * static_cast<double>(k) / static_cast<double>(len));
        const std::complex<double> u = a[i + k], t = a[i + k + len / 2] * w;
        a[i + k] = u + t;
        a[i + k + len / 2] = u - t;
      }
}

// exp(-2 pi i m / L) for m = first, first + step, ... (count values),
// interleaved, evaluated in FP64 and rounded once to T.
template <typename T>
void twiddles_strided(std::vector<T>& out, int64_t count, int64_t step, int64_t L) {
  out.resize(2 * count);
  for (int64_t m = 0; m < count; ++m) {
    const double a = -2.0 * M_PI * static_cast<double>(m * step) / static_cast<double>(L);
    out[2 * m] = static_cast<T>(std::cos(a));
    out[2 * m + 1] = static_cast<T>(std::sin(a));
  }
}

// Per-pass twiddle table of the block FFT of length L with e values per
// thread, in the order the engine reads it (see BlockFft::tw_offset): for
// each pass with stride ns > 1 and radix R, exp(-2 pi i r k / (ns R)),
// k in [0, ns), for r = 1, 2, 4, 8 (< R) or for every r in [1, R), as
// tw_full_pass(mode, ns) says.
template <typename T>
void stockham_twiddles(std::vector<T>& out, int64_t L, int64_t e, int mode) {
  out.clear();
  const int64_t rmax = std::min<int64_t>(e, 16);   // butterflies of at most radix 16
  auto radix = [&](int64_t ns) { return (L / ns >= rmax) ? rmax : L / ns; };
  for (int64_t ns = 1; ns < L; ns *= radix(ns)) {
    const int64_t R = radix(ns);
    if (ns == 1) continue;
    const bool full = tw_full_pass(mode, static_cast<int>(ns));
    for (int64_t r = 1; r < R; r = full ? r + 1 : 2 * r)
      for (int64_t k = 0; k < ns; ++k) {
        const double a = -2.0 * M_PI * static_cast<double>(r * k) / static_cast<double>(ns * R);
        out.push_back(static_cast<T>(std::cos(a)));
        out.push_back(static_cast<T>(std::sin(a)));
      }
  }
  if (out.empty()) out.assign(2, T(0));
}

// Values per thread of a length-L block transform (as RowGeom: at most 1024
// threads per transform).
int64_t engine_e(int64_t L, bool f64) {
  const int64_t e = std::min<int64_t>(L, f64 ? 8 : 16);
  return L / e > 1024 ? L / 1024 : e;
}

struct Blob {
  std::vector<char> bytes;
  size_t add(const void* p, size_t n) {
    const size_t off = align256(bytes.size());
    bytes.resize(off + n);
    if (n) std::memcpy(bytes.data() + off, p, n);
    return off;
  }
};

template <typename T>
qtam_status upload(qtam_plan_s* pl) {
  HostPlan& hp = pl->hp;
  Blob blob;
  std::vector<RowMeta> rm(hp.rows);
  for (int k = 0; k < hp.rows; ++k)
    rm[k] = RowMeta{hp.centre[k], hp.lo[k], hp.hi[k], static_cast<int>(hp.offset[k])};
  const size_t o_rows = blob.add(rm.data(), rm.size() * sizeof(RowMeta));
  // overlap-add: per wave of 64 bins p (p <= N/4) and its mirror side q = N/2 - p,
  // the rows whose kept support meets those bins, ascending
  const int64_t quarter = hp.half / 2;
  const int nw = static_cast<int>(quarter / 64 + 1);
  std::vector<std::vector<OlaRow>> side(2 * size_t(nw));
  for (int k = 0; k < hp.rows; ++k) {
    const OlaRow r{hp.lo[k], hp.hi[k] - hp.lo[k], static_cast<int>(hp.offset[k]) - hp.lo[k], 0};
    const int64_t pa = std::max<int64_t>(0, hp.lo[k]), pb = std::min<int64_t>(quarter, hp.hi[k]);
    for (int64_t w = pa / 64; pa <= pb && w <= pb / 64; ++w) side[2 * w].push_back(r);
    const int64_t qa = std::max<int64_t>(0, hp.half - hp.hi[k]), qb = std::min<int64_t>(quarter, hp.half - hp.lo[k]);
    for (int64_t w = qa / 64; qa <= qb && w <= qb / 64; ++w) side[2 * w + 1].push_back(r);
  }
  std::vector<int> ola_start(2 * size_t(nw) + 1, 0);
  std::vector<OlaRow> ola_rows;
  for (size_t i = 0; i < side.size(); ++i) {
    ola_start[i] = static_cast<int>(ola_rows.size());
    ola_rows.insert(ola_rows.end(), side[i].begin(), side[i].end());
  }
  ola_start[side.size()] = static_cast<int>(ola_rows.size());
  if (ola_rows.empty()) ola_rows.push_back(OlaRow{0, -1, 0, 0});
  pl->ola_waves = nw;
  const size_t o_bstart = blob.add(ola_start.data(), ola_start.size() * sizeof(int));
  const size_t o_bent = blob.add(ola_rows.data(), ola_rows.size() * sizeof(OlaRow));
  // the same lists for one row holding every bin in order (single-tile recovery)
  std::vector<int> one_start(2 * size_t(nw) + 1);
  for (size_t i = 0; i < one_start.size(); ++i) one_start[i] = static_cast<int>(i);
  const std::vector<OlaRow> one_rows(2 * size_t(nw), OlaRow{0, static_cast<int>(hp.half), 0, 0});
  const size_t o_one_start = blob.add(one_start.data(), one_start.size() * sizeof(int));
  const size_t o_one_rows = blob.add(one_rows.data(), one_rows.size() * sizeof(OlaRow));
  size_t o_tab[6];
  // dense tiles: Z = sqrt(N/N_out) DFT_{N_out}(Y) at the kept bins, and the
  // 1/N of the N-point inverse DFT, one constant per entry
  const std::vector<double> dense_tab(
      hp.sum_len, std::sqrt(static_cast<double>(hp.n) / static_cast<double>(hp.n_out)) / static_cast<double>(hp.n));
  const std::vector<double>* src[6] = {&hp.fwd_tab, &hp.dual_tab, &hp.afwd_tab, &hp.ainv_tab, &dense_tab,
                                       &hp.tile_tab};
  for (int i = 0; i < 6; ++i) {
    std::vector<T> v(src[i]->begin(), src[i]->end());
    o_tab[i] = blob.add(v.data(), v.size() * sizeof(T));
  }
  // per row (scale_k, 1/h_k): the forward weight at offset j is
  // scale_k (1 - (j/h_k)^2)^2 for the bisquare window
  std::vector<T> rw(2 * hp.rows);
  for (int k = 0; k < hp.rows; ++k) {
    rw[2 * k] = static_cast<T>(hp.fwd_tab[hp.offset[k] + (hp.centre[k] - hp.lo[k])]);
    rw[2 * k + 1] = static_cast<T>(1.0 / static_cast<double>(hp.half_width[k]));
  }
  const size_t o_rw = blob.add(rw.data(), rw.size() * sizeof(T));
  const bool f64 = sizeof(T) == 8;
  std::vector<T> tw;
  if (pl->bluestein) tw.assign(2, T(0));
  else stockham_twiddles(tw, hp.n_out, engine_e(hp.n_out, f64), TW_MIXED);
  const size_t o_out = blob.add(tw.data(), tw.size() * sizeof(T));
  size_t o_half = 0, o_n1 = 0, o_n2 = 0;
  if (!pl->four_step) {
    stockham_twiddles(tw, pl->m2, engine_e(pl->m2, f64), TW_POW);
    o_half = blob.add(tw.data(), tw.size() * sizeof(T));
  } else {
    stockham_twiddles(tw, pl->n1, std::min<int64_t>(pl->n1, kPass2E), TW_POW);
    o_n1 = blob.add(tw.data(), tw.size() * sizeof(T));
    stockham_twiddles(tw, pl->n2, engine_e(pl->n2, f64), TW_POW);
    o_n2 = blob.add(tw.data(), tw.size() * sizeof(T));
  }
  size_t o_r1 = 0, o_r2 = 0, o_rf = 0, o_rc = 0;
  if (pl->big_rows || pl->bs_long) {
    const int64_t lr = pl->big_rows ? int64_t(hp.n_out) : pl->bs_len;   // r1 * r2
    stockham_twiddles(tw, pl->r1, engine_e(pl->r1, f64), TW_POW);
    o_r1 = blob.add(tw.data(), tw.size() * sizeof(T));
    stockham_twiddles(tw, pl->r2, engine_e(pl->r2, f64), TW_POW);
    o_r2 = blob.add(tw.data(), tw.size() * sizeof(T));
    const int nbr = ilog2(lr);
    pl->twr_bits = (nbr + 1) / 2;
    const int64_t nf = int64_t(1) << pl->twr_bits, ncs = lr >> pl->twr_bits;
    twiddles_strided(tw, nf, 1, lr);
    o_rf = blob.add(tw.data(), tw.size() * sizeof(T));
    twiddles_strided(tw, ncs, nf, lr);
    o_rc = blob.add(tw.data(), tw.size() * sizeof(T));
  }
  size_t o_bsc = 0, o_bsf = 0, o_bsi = 0, o_bstw = 0;
  if (pl->bluestein) {
    const int64_t M = hp.n_out, Lb = pl->bs_len;
    std::vector<std::complex<double>> a(M), bf(Lb), bi(Lb);
    for (int64_t v = 0; v < M; ++v) {
      const int64_t e = (v * v) % (2 * M);   // exact v^2 mod 2M
      a[v] = std::polar(1.0, M_PI * static_cast<double>(e) / static_cast<double>(M));
    }
    for (int64_t v = 0; v < M; ++v) {
      bf[v] = std::conj(a[v]);
      bi[v] = a[v];
      if (v > 0) {
        bf[Lb - v] = std::conj(a[v]);
        bi[Lb - v] = a[v];
      }
    }
    host_fft(bf);
    host_fft(bi);
    std::vector<T> ta(2 * M), tf(2 * Lb), ti(2 * Lb);
    for (int64_t v = 0; v < M; ++v) {
      ta[2 * v] = static_cast<T>(a[v].real());
      ta[2 * v + 1] = static_cast<T>(a[v].imag());
    }
    for (int64_t k = 0; k < Lb; ++k) {
      tf[2 * k] = static_cast<T>(bf[k].real() / static_cast<double>(Lb));
      tf[2 * k + 1] = static_cast<T>(bf[k].imag() / static_cast<double>(Lb));
      ti[2 * k] = static_cast<T>(bi[k].real() / static_cast<double>(Lb));
      ti[2 * k + 1] = static_cast<T>(bi[k].imag() / static_cast<double>(Lb));
    }
    o_bsc = blob.add(ta.data(), ta.size() * sizeof(T));
    o_bsf = blob.add(tf.data(), tf.size() * sizeof(T));
    o_bsi = blob.add(ti.data(), ti.size() * sizeof(T));
    if (!pl->bs_long) {   // one-workgroup rows: Stockham twiddles of the whole length
      stockham_twiddles(tw, Lb, engine_e(Lb, f64), TW_POW);
      o_bstw = blob.add(tw.data(), tw.size() * sizeof(T));
    }
  }
  size_t o_dt = 0, o_dn1 = 0, o_dn2 = 0;
  if (pl->dense_ok) {
    if (!pl->dense_four_step) {
      stockham_twiddles(tw, pl->dense_md, engine_e(pl->dense_md, f64), TW_POW);
      o_dt = blob.add(tw.data(), tw.size() * sizeof(T));
    } else {
      stockham_twiddles(tw, pl->dn1, engine_e(pl->dn1, f64), TW_POW);
      o_dn1 = blob.add(tw.data(), tw.size() * sizeof(T));
      stockham_twiddles(tw, pl->dn2, engine_e(pl->dn2, f64), TW_POW);
      o_dn2 = blob.add(tw.data(), tw.size() * sizeof(T));
    }
  }
  // two-level table of exp(-2 pi i m / N)
  const int nb = ilog2(hp.n);
  pl->tw2_bits = (nb + 1) / 2;
  const int64_t nfine = int64_t(1) << pl->tw2_bits, ncoarse = (hp.n + nfine - 1) >> pl->tw2_bits;
  twiddles_strided(tw, nfine, 1, hp.n);
  const size_t o_f = blob.add(tw.data(), tw.size() * sizeof(T));
  twiddles_strided(tw, ncoarse, nfine, hp.n);
  const size_t o_c = blob.add(tw.data(), tw.size() * sizeof(T));

  hipError_t e = hipMalloc(reinterpret_cast<void**>(&pl->dmem), blob.bytes.size());
  if (e != hipSuccess) {
    pl->dmem = nullptr;
    return hip_failed(e, "hipMalloc of the plan tables", QTAM_ERR_OOM);
  }
  e = hipMemcpy(pl->dmem, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_failed(e, "hipMemcpy of the plan tables");
  char* d = pl->dmem;
  pl->d_rows = reinterpret_cast<RowMeta*>(d + o_rows);
  pl->d_roww = d + o_rw;
  pl->d_ola_start = reinterpret_cast<int*>(d + o_bstart);
  pl->d_ola_rows = reinterpret_cast<OlaRow*>(d + o_bent);
  pl->d_one_start = reinterpret_cast<int*>(d + o_one_start);
  pl->d_one_rows = reinterpret_cast<OlaRow*>(d + o_one_rows);
  for (int i = 0; i < 6; ++i) pl->d_tab[i] = d + o_tab[i];
  pl->d_tw_out = d + o_out;
  if (pl->dense_ok) {
    pl->d_tw_dense = pl->dense_four_step ? nullptr : d + o_dt;
    pl->d_tw_dn1 = pl->dense_four_step ? d + o_dn1 : nullptr;
    pl->d_tw_dn2 = pl->dense_four_step ? d + o_dn2 : nullptr;
  }
  if (pl->bluestein) {
    pl->d_bs_chirp = d + o_bsc;
    pl->d_bs_bf = d + o_bsf;
    pl->d_bs_bi = d + o_bsi;
    pl->d_bs_tw = pl->bs_long ? nullptr : d + o_bstw;
  }
  pl->d_tw_half = pl->four_step ? nullptr : d + o_half;
  pl->d_tw_n1 = pl->four_step ? d + o_n1 : nullptr;
  pl->d_tw_n2 = pl->four_step ? d + o_n2 : nullptr;
  if (pl->big_rows || pl->bs_long) {
    pl->d_tw_r1 = d + o_r1;
    pl->d_tw_r2 = d + o_r2;
    pl->d_twr_fine = d + o_rf;
    pl->d_twr_coarse = d + o_rc;
  }
  pl->d_tw2_fine = d + o_f;
  pl->d_tw2_coarse = d + o_c;
  return QTAM_OK;
}

// ---------------------------------------------------------------------------
// Timing hooks
// ---------------------------------------------------------------------------
struct Timed {
  qtam_plan_s* pl;
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(qtam_plan_s* p, int k, hipStream_t st) : pl(p), kind(k), s(st) {
    if (!pl->timing || g_untimed) return;
    std::lock_guard<std::mutex> g(pl->mu);
    for (hipEvent_t* e : {&a, &b}) {
      if (!pl->pool.empty()) {
        *e = pl->pool.back();
        pl->pool.pop_back();
      } else if (hipEventCreate(e) != hipSuccess) {
        *e = nullptr;
      }
    }
    if (a) (void)hipEventRecord(a, s);
  }
  ~Timed() {
    if (!a || !b) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> g(pl->mu);
    try {
      pl->pending.push_back({kind, a, b});
    } catch (const std::bad_alloc&) {   // no room to keep the record: the launch goes untimed
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  }
};

// ---------------------------------------------------------------------------
// Dispatch over compile-time sizes
// ---------------------------------------------------------------------------
#define QTAM_POW2_CASES(X) \
  X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15)

template <typename T, int S>
bool launch_fft_rows(int log2l, const void* in, void* out, int64_t count, int64_t stride, const void* tw,
                     hipStream_t st) {
  using C = typename Complex<T>::type;
  switch (log2l) {
#define X(LG)                                                                                      \
  case LG:                                                                                         \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Single32 : kMaxLog2Single64)) {               \
      using Geo = RowGeom<T, (1 << LG)>;                                                           \
      const int64_t blocks = (count + Geo::G - 1) / Geo::G;                                        \
      hipLaunchKernelGGL((k_fft_rows<T, (1 << LG), S>), dim3(unsigned(blocks)), dim3(Geo::NT), 0, st, \
                         static_cast<const C*>(in), static_cast<C*>(out), count, stride,            \
                         static_cast<const C*>(tw));                                               \
      return true;                                                                                 \
    }                                                                                              \
    return false;
    QTAM_POW2_CASES(X)
#undef X
    default: return false;
  }
}

#define QTAM_COL_CASES(X) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)
constexpr int kMaxLog2Col32 = 12;   // four-step sub-FFTs up to 4096 points (FP32)
constexpr int kMaxLog2Col64 = 11;   // and 2048 points (FP64)

template <typename T, int S>
bool launch_fft_cols(int log2l, const void* in, void* out, int64_t n1, int64_t segs, int64_t seg_stride,
                     const void* tw, Twiddle2<typename Complex<T>::type> tw2, hipStream_t st, int tw_mul = 2) {
  using C = typename Complex<T>::type;
  switch (log2l) {
#define X(LG)                                                                                     \
  case LG:                                                                                        \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Col32 : kMaxLog2Col64)) {                     \
      using GeoW = ColGeom<T, (1 << LG), 0, kColWide>;                                            \
      if (n1 % GeoW::CC == 0) {                                                                   \
        hipLaunchKernelGGL((k_fft_cols<T, (1 << LG), S, kColWide>), dim3(unsigned(n1 / GeoW::CC), unsigned(segs)), \
                           dim3(GeoW::NT), 0, st, static_cast<const C*>(in), static_cast<C*>(out), n1, \
                           seg_stride, static_cast<const C*>(tw), tw2, tw_mul);                   \
        return true;                                                                              \
      }                                                                                           \
      using Geo = ColGeom<T, (1 << LG)>;                                                          \
      if (n1 % Geo::CC) return false;                                                             \
      hipLaunchKernelGGL((k_fft_cols<T, (1 << LG), S>), dim3(unsigned(n1 / Geo::CC), unsigned(segs)), \
                         dim3(Geo::NT), 0, st, static_cast<const C*>(in), static_cast<C*>(out), n1, \
                         seg_stride, static_cast<const C*>(tw), tw2, tw_mul);                     \
      return true;                                                                                \
    }                                                                                             \
    return false;
    QTAM_COL_CASES(X)
#undef X
    default: return false;
  }
}

template <typename T, int S, int EP = 0>
bool launch_fft_rows_t(int log2l, const void* in, void* out, int64_t n2, int64_t segs, int64_t seg_stride,
                       const void* tw, hipStream_t st) {
  using C = typename Complex<T>::type;
  switch (log2l) {
#define X(LG)                                                                                       \
  case LG:                                                                                          \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Col32 : kMaxLog2Col64)) {                       \
      constexpr int CW = EP == 0 ? kRowWide : 0;                                                    \
      using GeoW = ColGeom<T, (1 << LG), EP, CW>;                                                   \
      if (n2 % GeoW::CC == 0) {                                                                     \
        hipLaunchKernelGGL((k_fft_rows_t<T, (1 << LG), S, EP, CW>), dim3(unsigned(n2 / GeoW::CC), unsigned(segs)), \
                           dim3(GeoW::NT), 0, st, static_cast<const C*>(in), static_cast<C*>(out), n2, \
                           seg_stride, static_cast<const C*>(tw));                                  \
        return true;                                                                                \
      }                                                                                             \
      using Geo = ColGeom<T, (1 << LG), EP>;                                                        \
      if (n2 % Geo::CC) return false;                                                               \
      hipLaunchKernelGGL((k_fft_rows_t<T, (1 << LG), S, EP>), dim3(unsigned(n2 / Geo::CC), unsigned(segs)), \
                         dim3(Geo::NT), 0, st, static_cast<const C*>(in), static_cast<C*>(out), n2,  \
                         seg_stride, static_cast<const C*>(tw));                                    \
      return true;                                                                                  \
    }                                                                                               \
    return false;
    QTAM_COL_CASES(X)
#undef X
    default: return false;
  }
}

template <typename T>
bool launch_spec_rows_twist(int log2l, const void* in, void* out, int64_t n2, int64_t segs, int64_t seg_stride,
                            const void* tw, Twiddle2<typename Complex<T>::type> tw2, hipStream_t st) {
  using C = typename Complex<T>::type;
  switch (log2l) {
#define X(LG)                                                                                       \
  case LG:                                                                                          \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Col32 : kMaxLog2Col64)) {                       \
      using GeoW = ColGeom<T, (1 << LG), kPass2E, kRowWide>;                                        \
      if (n2 % GeoW::CC == 0) {                                                                     \
        hipLaunchKernelGGL((k_spec_rows_twist<T, (1 << LG), kPass2E, kRowWide>), dim3(unsigned(n2 / GeoW::CC), unsigned(segs)), \
                           dim3(GeoW::NT), 0, st, static_cast<const C*>(in), static_cast<C*>(out), n2, \
                           seg_stride, static_cast<const C*>(tw), tw2);                             \
        return true;                                                                                \
      }                                                                                             \
      using Geo = ColGeom<T, (1 << LG), kPass2E>;                                                   \
      if (n2 % Geo::CC) return false;                                                               \
      hipLaunchKernelGGL((k_spec_rows_twist<T, (1 << LG), kPass2E>), dim3(unsigned(n2 / Geo::CC), unsigned(segs)), \
                         dim3(Geo::NT), 0, st, static_cast<const C*>(in), static_cast<C*>(out), n2,  \
                         seg_stride, static_cast<const C*>(tw), tw2);                               \
      return true;                                                                                  \
    }                                                                                               \
    return false;
    QTAM_COL_CASES(X)
#undef X
    default: return false;
  }
}

// The denoiser's mask fused into the row kernels of a masked inverse (gain,
// lam) and of its adjoint (y: the unmasked envelopes; part: one partial sum
// of the gain gradient per row of the chunk).
struct MaskArgs {
  const void* y;
  const void* gain;
  const void* lam;
  void* part;
};

template <typename T>
bool launch_rows(bool forward, bool analytic, int log2l, const void* in, void* out, const RowMeta* rows,
                 const void* roww, const void* tab, int R, int64_t total_rows, int64_t half, int64_t sum_len,
                 const void* tw, hipStream_t st, void* stats = nullptr, const MaskArgs* mk = nullptr) {
  using C = typename Complex<T>::type;
  const C* my = mk ? static_cast<const C*>(mk->y) : nullptr;
  const T* mg = mk ? static_cast<const T*>(mk->gain) : nullptr;
  const T* ml = mk ? static_cast<const T*>(mk->lam) : nullptr;
  T* mp = mk ? static_cast<T*>(mk->part) : nullptr;
  switch (log2l) {
#define X(LG)                                                                                          \
  case LG:                                                                                             \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Rows32 : kMaxLog2Rows64)) {                        \
      using Geo = RowGeom<T, (1 << LG)>;                                                               \
      const int blocks = static_cast<int>((total_rows + Geo::G - 1) / Geo::G);                         \
      if (forward) {                                                                                   \
        auto kern = mk ? k_fwd_rows<T, (1 << LG), false, false, true>                                  \
                       : stats ? (analytic ? k_fwd_rows<T, (1 << LG), true, true>                      \
                                           : k_fwd_rows<T, (1 << LG), false, true>)                    \
                               : (analytic ? k_fwd_rows<T, (1 << LG), true, false>                     \
                                           : k_fwd_rows<T, (1 << LG), false, false>);                  \
        hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(Geo::NT), 0, st, static_cast<const C*>(in), \
                           static_cast<C*>(out), rows, static_cast<const C*>(roww),                    \
                           static_cast<const T*>(tab), R, int(total_rows), int(half), int(sum_len),    \
                           (total_rows / R) * half, static_cast<const C*>(tw), blocks,                 \
                           static_cast<C*>(stats), my, mg, ml, mp);                                    \
      } else {                                                                                         \
        auto kern = mk ? k_inv_rows<T, (1 << LG), true> : k_inv_rows<T, (1 << LG), false>;            \
        hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(Geo::NT), 0, st,                         \
                           static_cast<const C*>(in), static_cast<C*>(out), rows,                      \
                           static_cast<const T*>(tab), R, int(total_rows), int(sum_len),               \
                           int(total_rows / R), static_cast<const C*>(tw), mg, ml);                   \
      }                                                                                                \
      return true;                                                                                     \
    }                                                                                                  \
    return false;
    QTAM_POW2_CASES(X)
#undef X
    default: return false;
  }
}

template <typename T>
bool launch_rows_bs(bool forward, int log2l, const void* in, void* out, const RowMeta* rows, const void* tab, int R,
                    int64_t total_rows, int64_t half, int64_t sum_len, int M, const void* chirp, const void* bhat,
                    const void* tw, hipStream_t st) {
  using C = typename Complex<T>::type;
  switch (log2l) {
#define X(LG)                                                                                          \
  case LG:                                                                                             \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Single32 : kMaxLog2Single64)) {                    \
      using Geo = RowGeom<T, (1 << LG)>;                                                               \
      const int blocks = static_cast<int>((total_rows + Geo::G - 1) / Geo::G);                         \
      if (forward)                                                                                     \
        hipLaunchKernelGGL((k_fwd_rows_bs<T, (1 << LG)>), dim3(unsigned(blocks)), dim3(Geo::NT), 0, st,  \
                           static_cast<const C*>(in), static_cast<C*>(out), rows, static_cast<const T*>(tab), \
                           R, int(total_rows), int(half), int(sum_len), (total_rows / R) * half, M,    \
                           static_cast<const C*>(chirp), static_cast<const C*>(bhat), static_cast<const C*>(tw)); \
      else                                                                                             \
        hipLaunchKernelGGL((k_inv_rows_bs<T, (1 << LG)>), dim3(unsigned(blocks)), dim3(Geo::NT), 0, st,  \
                           static_cast<const C*>(in), static_cast<C*>(out), rows, static_cast<const T*>(tab), \
                           R, int(total_rows), int(sum_len), M, static_cast<const C*>(chirp),          \
                           static_cast<const C*>(bhat), static_cast<const C*>(tw));                    \
      return true;                                                                                     \
    }                                                                                                  \
    return false;
    QTAM_POW2_CASES(X)
#undef X
    default: return false;
  }
}

template <typename T>
bool launch_fwd_rows_cols(int log2l2, const void* spec, void* A, const RowMeta* rows, const void* tab, int R,
                          int64_t total_rows, int64_t half, int64_t n_out, int64_t l1, const void* tw,
                          Twiddle2<typename Complex<T>::type> tw2, hipStream_t st) {
  using C = typename Complex<T>::type;
  switch (log2l2) {
#define X(LG)                                                                                          \
  case LG:                                                                                             \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Col32 : kMaxLog2Col64)) {                          \
      using Geo = ColGeom<T, (1 << LG)>;                                                               \
      if (l1 % Geo::CC) return false;                                                                  \
      hipLaunchKernelGGL((k_fwd_rows_cols<T, (1 << LG)>), dim3(unsigned(l1 / Geo::CC), unsigned(total_rows)), \
                         dim3(Geo::NT), 0, st, static_cast<const C*>(spec), static_cast<C*>(A), rows,  \
                         static_cast<const T*>(tab), R, int(half), n_out, l1, static_cast<const C*>(tw), tw2); \
      return true;                                                                                     \
    }                                                                                                  \
    return false;
    QTAM_COL_CASES(X)
#undef X
    default: return false;
  }
}

template <typename T>
bool launch_inv_rows_rowst(int log2l1, const void* A, void* S, const RowMeta* rows, const void* tab, int R,
                           int64_t total_rows, int64_t sum_len, int64_t n_out, int64_t l2, const void* tw,
                           hipStream_t st) {
  using C = typename Complex<T>::type;
  switch (log2l1) {
#define X(LG)                                                                                          \
  case LG:                                                                                             \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Col32 : kMaxLog2Col64)) {                          \
      using Geo = ColGeom<T, (1 << LG)>;                                                               \
      if (l2 % Geo::CC) return false;                                                                  \
      hipLaunchKernelGGL((k_inv_rows_rowst<T, (1 << LG)>), dim3(unsigned(l2 / Geo::CC), unsigned(total_rows)), \
                         dim3(Geo::NT), 0, st, static_cast<const C*>(A), static_cast<C*>(S), rows,     \
                         static_cast<const T*>(tab), R, sum_len, n_out, l2, static_cast<const C*>(tw)); \
      return true;                                                                                     \
    }                                                                                                  \
    return false;
    QTAM_COL_CASES(X)
#undef X
    default: return false;
  }
}

// ---------------------------------------------------------------------------
// Workspace layout for a chunk of segments
// ---------------------------------------------------------------------------
struct WsLayout {
  size_t spec = 0, tmp = 0, tmp2 = 0, pack = 0, rows = 0, total = 0;
};

WsLayout layout_for(const qtam_plan_s* pl, int64_t segs) {
  const size_t cb = (pl->hp.precision == QTAM_FP64 ? 16 : 8);
  WsLayout w;
  size_t off = 0;
  w.spec = off;
  off = align256(off + size_t(segs) * size_t(pl->hp.half) * cb);
  w.tmp = off;
  if (pl->four_step || pl->radix_r > 1) off = align256(off + size_t(segs) * size_t(pl->hp.half) * cb);
  w.tmp2 = off;
  if (pl->radix_r > 1) off = align256(off + size_t(segs) * size_t(pl->hp.half) * cb);
  w.pack = off;
  off = align256(off + size_t(segs) * size_t(pl->hp.sum_len) * cb);
  w.rows = off;
  if (pl->big_rows) off = align256(off + size_t(segs) * size_t(pl->hp.rows) * size_t(pl->hp.n_out) * cb);
  if (pl->bs_long) off = align256(off + 2 * size_t(segs) * size_t(pl->hp.rows) * size_t(pl->bs_len) * cb);
  w.total = off;
  return w;
}

// Largest number of segments whose signal, envelope and workspace regions each
// stay below 2 GiB (kernels address them with 32-bit byte offsets).
int64_t chunk_cap(const qtam_plan_s* pl) {
  const HostPlan& hp = pl->hp;
  const size_t rb = hp.precision == QTAM_FP64 ? 8 : 4;
  const size_t per = std::max({size_t(hp.n) * rb, size_t(hp.rows) * size_t(hp.n_out) * 2 * rb,
                               size_t(hp.sum_len) * 2 * rb});
  const size_t lim = size_t(1) << 31;
  int64_t cap = per > lim ? 0 : int64_t(lim / per);
  if (pl->big_rows || pl->bs_long) cap = std::min<int64_t>(cap, 65535 / hp.rows);   // rows of a chunk index grid.y
  cap = std::min<int64_t>(cap, 65535 / pl->radix_r);                  // decimated rows index grid.y
  return cap;
}

int64_t chunk_for(const qtam_plan_s* pl, int64_t batch, size_t ws_bytes) {
  if (layout_for(pl, 1).total > ws_bytes) return 0;
  int64_t lo = 1, hi = std::min(batch, chunk_cap(pl));
  if (hi < 1) return 0;
  while (lo < hi) {   // largest chunk whose layout fits
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (layout_for(pl, mid).total <= ws_bytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// The two halves of the path, for one chunk
// ---------------------------------------------------------------------------
template <typename T>
Twiddle2<typename Complex<T>::type> tw2_of(const qtam_plan_s* pl) {
  using C = typename Complex<T>::type;
  return Twiddle2<C>{static_cast<const C*>(pl->d_tw2_fine), static_cast<const C*>(pl->d_tw2_coarse),
                     pl->tw2_bits};
}

// count length-M2 transforms (sign S) of consecutive M2-element blocks: one
// LDS pass, or two passes through `tmp` (then `tmp` must differ from both).
template <typename T, int S>
bool transform_m2(qtam_plan_s* pl, const void* in, void* out, void* tmp, int64_t count, hipStream_t st, int k_one,
                  int k_pass1, int k_pass2) {
  const int64_t m2 = pl->m2;
  if (!pl->four_step) {
    Timed tm(pl, k_one, st);
    return launch_fft_rows<T, S>(ilog2(m2), in, out, count, m2, pl->d_tw_half, st);
  }
  bool ok;
  {
    Timed tm(pl, k_pass1, st);
    ok = launch_fft_cols<T, S>(ilog2(pl->n2), in, tmp, pl->n1, count, m2, pl->d_tw_n2, tw2_of<T>(pl), st,
                               static_cast<int>(2 * pl->radix_r));
  }
  if (!ok) return false;
  Timed tm(pl, k_pass2, st);
  return launch_fft_rows_t<T, S, kPass2E>(ilog2(pl->n1), tmp, out, pl->n2, count, m2, pl->d_tw_n1, st);
}

// Radix-r combination of the decimated transforms (S = -1, analysis) or its
// inverse (S = +1, synthesis), over segs segments.
template <typename T, int S>
bool launch_radix(qtam_plan_s* pl, const void* in, void* out, int64_t segs, hipStream_t st) {
  using C = typename Complex<T>::type;
  Timed tm(pl, S < 0 ? K_SPEC_RADIX : K_SYN_RADIX, st);
  const dim3 grid(unsigned((pl->m2 + 255) / 256), unsigned(segs));
  if (pl->radix_r == 3)
    hipLaunchKernelGGL((k_radix<T, 3, S>), grid, dim3(256), 0, st, static_cast<const C*>(in), static_cast<C*>(out),
                       pl->m2, tw2_of<T>(pl));
  else if (pl->radix_r == 5)
    hipLaunchKernelGGL((k_radix<T, 5, S>), grid, dim3(256), 0, st, static_cast<const C*>(in), static_cast<C*>(out),
                       pl->m2, tw2_of<T>(pl));
  else
    return false;
  return true;
}

// analysis, first half: real signal x -> its spectrum in ws + lay.spec (bins
// 0 .. N/2 - 1 of the N/2-point half-size transform after the real-signal twist).
// Depends on N and the precision only, so plans that share both share it.
template <typename T>
bool analysis_spectrum(qtam_plan_s* pl, const void* x, int64_t segs, char* ws, const WsLayout& lay,
                       hipStream_t st) {
  const HostPlan& hp = pl->hp;
  const int64_t half = hp.half;
  void* spec = ws + lay.spec;
  bool ok;
  bool twisted = false;
  if (pl->radix_r == 1 && pl->four_step) {
    // first pass, then the second pass with the real-signal twist folded in
    void* tmp = ws + lay.tmp;
    {
      Timed tm(pl, K_SPEC1, st);
      ok = launch_fft_cols<T, -1>(ilog2(pl->n2), x, tmp, pl->n1, segs, half, pl->d_tw_n2, tw2_of<T>(pl), st, 2);
    }
    if (ok) {
      Timed tm(pl, K_SPEC2, st);
      ok = launch_spec_rows_twist<T>(ilog2(pl->n1), tmp, spec, pl->n2, segs, half, pl->d_tw_n1, tw2_of<T>(pl), st);
    }
    twisted = true;
  } else if (pl->radix_r == 1) {
    ok = transform_m2<T, -1>(pl, x, spec, ws + lay.tmp, segs, st, K_SPEC, K_SPEC1, K_SPEC2);
  } else {
    using C = typename Complex<T>::type;
    void* tmp = ws + lay.tmp;
    void* tmp2 = ws + lay.tmp2;
    {
      Timed tm(pl, K_SPEC_PERM, st);
      hipLaunchKernelGGL((k_permute<T, true>), dim3(unsigned((half + 255) / 256), unsigned(segs)), dim3(256), 0, st,
                         static_cast<const C*>(x), static_cast<C*>(tmp2), pl->radix_r, pl->m2);
    }
    // single pass: tmp2 -> tmp; four-step: tmp2 -> tmp -> tmp2
    void* f = pl->four_step ? tmp2 : tmp;
    ok = transform_m2<T, -1>(pl, tmp2, f, tmp, segs * pl->radix_r, st, K_SPEC, K_SPEC1, K_SPEC2);
    if (ok) ok = launch_radix<T, -1>(pl, f, spec, segs, st);
  }
  if (!ok) return false;
  if (!twisted) {
    using C = typename Complex<T>::type;
    Timed tm(pl, K_TWIST, st);
    hipLaunchKernelGGL((k_twist<T>), dim3(unsigned((half / 2 + 1 + 255) / 256), unsigned(segs)), dim3(256), 0, st,
                       static_cast<C*>(spec), half, tw2_of<T>(pl));
  }
  return true;
}

// Chirp-z rows beyond one workgroup, for one chunk: the length-L cyclic
// convolution of each row (L = bs_len = r1 * r2) as a forward and an inverse
// four-step transform through two workspace buffers A and B of
// segs * R * L values (ws + lay.rows), between element passes:
//   forward:  prep (gather x table x chirp) -> B, FFT B -> B (via A),
//             B *= Bhat_f, IFFT B -> B (via A), y = B x chirp;
//   inverse:  prep (y x conj chirp) -> B, FFT, B *= Bhat_i, IFFT,
//             kept slots x conj chirp x table -> packed.
template <typename T>
bool chirp_rows_long(qtam_plan_s* pl, bool forward, int table, const void* in, void* out, int64_t segs, char* ws,
                     const WsLayout& lay, hipStream_t st) {
  using C = typename Complex<T>::type;
  const HostPlan& hp = pl->hp;
  const int64_t L = pl->bs_len, count = segs * hp.rows;
  const int M = hp.n_out;
  C* A = reinterpret_cast<C*>(ws + lay.rows);
  C* B = A + count * L;
  const Twiddle2<C> twr{static_cast<const C*>(pl->d_twr_fine), static_cast<const C*>(pl->d_twr_coarse),
                        pl->twr_bits};
  const C* chirp = static_cast<const C*>(pl->d_bs_chirp);
  const dim3 gl(unsigned((L + 255) / 256), unsigned(count)), gm(unsigned((M + 255) / 256), unsigned(count));
  if (forward)
    hipLaunchKernelGGL((k_bs_fwd_prep<T>), gl, dim3(256), 0, st, static_cast<const C*>(in), B, pl->d_rows,
                       static_cast<const T*>(pl->d_tab[table]), hp.rows, int(hp.half), M, L, chirp);
  else
    hipLaunchKernelGGL((k_bs_inv_prep<T>), gl, dim3(256), 0, st, static_cast<const C*>(in), B, M, L, chirp);
  if (!launch_fft_cols<T, -1>(ilog2(pl->r2), B, A, pl->r1, count, L, pl->d_tw_r2, twr, st, 1) ||
      !launch_fft_rows_t<T, -1>(ilog2(pl->r1), A, B, pl->r2, count, L, pl->d_tw_r1, st))
    return false;
  hipLaunchKernelGGL((k_bs_mul<T>), gl, dim3(256), 0, st, B, L,
                     static_cast<const C*>(forward ? pl->d_bs_bf : pl->d_bs_bi));
  if (!launch_fft_cols<T, +1>(ilog2(pl->r2), B, A, pl->r1, count, L, pl->d_tw_r2, twr, st, 1) ||
      !launch_fft_rows_t<T, +1>(ilog2(pl->r1), A, B, pl->r2, count, L, pl->d_tw_r1, st))
    return false;
  if (forward)
    hipLaunchKernelGGL((k_bs_fwd_post<T>), gm, dim3(256), 0, st, B, static_cast<C*>(out), M, L, chirp);
  else
    hipLaunchKernelGGL((k_bs_inv_post<T>), gm, dim3(256), 0, st, B, static_cast<C*>(out), pl->d_rows,
                       static_cast<const T*>(pl->d_tab[table]), hp.rows, int64_t(hp.sum_len), M, L, chirp);
  return true;
}

// analysis, second half: spectrum -> rows (forward with T_FWD, inverse adjoint
// with T_AINV). Reads ws + lay.spec, writes y (and ws + lay.rows for long rows).
template <typename T>
bool analysis_rows(qtam_plan_s* pl, int table, void* y, int64_t segs, char* ws, const WsLayout& lay,
                   hipStream_t st, void* stats, const MaskArgs* mk = nullptr) {
  const HostPlan& hp = pl->hp;
  const int64_t half = hp.half;
  void* spec = ws + lay.spec;
  if (pl->big_rows) {
    using C = typename Complex<T>::type;
    const Twiddle2<C> twr{static_cast<const C*>(pl->d_twr_fine), static_cast<const C*>(pl->d_twr_coarse),
                          pl->twr_bits};
    void* A = ws + lay.rows;
    {
      Timed tm(pl, K_FWD_ROWS, st);
      if (!launch_fwd_rows_cols<T>(ilog2(pl->r2), spec, A, pl->d_rows, pl->d_tab[table], hp.rows,
                                   segs * hp.rows, half, hp.n_out, pl->r1, pl->d_tw_r2, twr, st))
        return false;
    }
    {
      Timed tm(pl, K_FWD_ROWS2, st);
      if (!launch_fft_rows_t<T, +1>(ilog2(pl->r1), A, y, pl->r2, segs * hp.rows, hp.n_out, pl->d_tw_r1, st))
        return false;
    }
    if (stats) {
      Timed tm(pl, K_ROW_STATS, st);
      hipLaunchKernelGGL((k_row_stats<T>), dim3(unsigned(segs * hp.rows)), dim3(256), 0, st, static_cast<const C*>(y),
                         static_cast<C*>(stats), int64_t(hp.n_out));
    }
    return true;
  }
  if (pl->bluestein) {
    using C = typename Complex<T>::type;
    if (pl->bs_long) {
      Timed tm(pl, K_FWD_ROWS, st);
      if (!chirp_rows_long<T>(pl, true, table, spec, y, segs, ws, lay, st)) return false;
    } else {
      Timed tm(pl, K_FWD_ROWS, st);
      if (!launch_rows_bs<T>(true, ilog2(pl->bs_len), spec, y, pl->d_rows, pl->d_tab[table], hp.rows, segs * hp.rows,
                             half, hp.sum_len, hp.n_out, pl->d_bs_chirp, pl->d_bs_bf, pl->d_bs_tw, st))
        return false;
    }
    if (stats) {
      Timed tm(pl, K_ROW_STATS, st);
      hipLaunchKernelGGL((k_row_stats<T>), dim3(unsigned(segs * hp.rows)), dim3(256), 0, st, static_cast<const C*>(y),
                         static_cast<C*>(stats), int64_t(hp.n_out));
    }
    return true;
  }
  Timed tm(pl, K_FWD_ROWS, st);
  return launch_rows<T>(true, table == T_FWD && pl->analytic_fwd, ilog2(hp.n_out), spec, y, pl->d_rows,
                        pl->d_roww, pl->d_tab[table], hp.rows, segs * hp.rows, half, hp.sum_len,
                        pl->d_tw_out, st, stats, mk);
}

template <typename T>
bool run_analysis(qtam_plan_s* pl, int table, const void* x, void* y, int64_t segs, char* ws,
                  const WsLayout& lay, hipStream_t st, void* stats, const MaskArgs* mk = nullptr) {
  return analysis_spectrum<T>(pl, x, segs, ws, lay, st) &&
         analysis_rows<T>(pl, table, y, segs, ws, lay, st, stats, mk);
}

// synthesis: rows -> real signal (inverse with T_DUAL, forward adjoint with T_AFWD)
template <typename T>
bool inverse_rows(qtam_plan_s* pl, int table, const void* y, int64_t segs, char* ws, const WsLayout& lay,
                  hipStream_t st, const MaskArgs* mk = nullptr) {
  using C = typename Complex<T>::type;
  const HostPlan& hp = pl->hp;
  const int64_t half = hp.half;
  void* pack = ws + lay.pack;
  bool ok;
  if (pl->big_rows) {
    const Twiddle2<C> twr{static_cast<const C*>(pl->d_twr_fine), static_cast<const C*>(pl->d_twr_coarse),
                          pl->twr_bits};
    void* A = ws + lay.rows;
    {
      Timed tm(pl, K_INV_ROWS, st);
      ok = launch_fft_cols<T, -1>(ilog2(pl->r2), y, A, pl->r1, segs * hp.rows, hp.n_out, pl->d_tw_r2, twr, st, 1);
    }
    if (ok) {
      Timed tm(pl, K_INV_ROWS2, st);
      ok = launch_inv_rows_rowst<T>(ilog2(pl->r1), A, pack, pl->d_rows, pl->d_tab[table], hp.rows,
                                    segs * hp.rows, hp.sum_len, hp.n_out, pl->r2, pl->d_tw_r1, st);
    }
  } else if (pl->bluestein && pl->bs_long) {
    Timed tm(pl, K_INV_ROWS, st);
    ok = chirp_rows_long<T>(pl, false, table, y, pack, segs, ws, lay, st);
  } else if (pl->bluestein) {
    Timed tm(pl, K_INV_ROWS, st);
    ok = launch_rows_bs<T>(false, ilog2(pl->bs_len), y, pack, pl->d_rows, pl->d_tab[table], hp.rows, segs * hp.rows,
                           half, hp.sum_len, hp.n_out, pl->d_bs_chirp, pl->d_bs_bi, pl->d_bs_tw, st);
  } else {
    Timed tm(pl, K_INV_ROWS, st);
    ok = launch_rows<T>(false, false, ilog2(hp.n_out), y, pack, pl->d_rows, nullptr, pl->d_tab[table],
                        hp.rows, segs * hp.rows, half, hp.sum_len, pl->d_tw_out, st, nullptr, mk);
  }
  return ok;
}

template <typename T>
bool synthesize(qtam_plan_s* pl, const void* pack, int64_t slen, const int* starts, const OlaRow* list, void* x,
                int64_t segs, char* ws, const WsLayout& lay, hipStream_t st);

template <typename T>
bool run_synthesis(qtam_plan_s* pl, int table, const void* y, void* x, int64_t segs, char* ws,
                   const WsLayout& lay, hipStream_t st, const MaskArgs* mk = nullptr) {
  const HostPlan& hp = pl->hp;
  void* pack = ws + lay.pack;
  bool ok = inverse_rows<T>(pl, table, y, segs, ws, lay, st, mk);
  if (!ok) return false;
  return synthesize<T>(pl, pack, hp.sum_len, pl->d_ola_start, pl->d_ola_rows, x, segs, ws, lay, st);
}

// Overlap-add of packed entries (per-wave row lists `starts`, `list`; `slen`
// entries per segment) with the real-signal pre-twist, then the inverse
// half-size transform to the real signal x.
template <typename T>
bool synthesize(qtam_plan_s* pl, const void* pack, int64_t slen, const int* starts, const OlaRow* list, void* x,
                int64_t segs, char* ws, const WsLayout& lay, hipStream_t st) {
  using C = typename Complex<T>::type;
  const int64_t half = pl->hp.half;
  void* spec = ws + lay.spec;
  {
    Timed tm(pl, K_OLA, st);
    hipLaunchKernelGGL((k_ola<T>), dim3(unsigned((pl->ola_waves + 3) / 4), unsigned(segs)), dim3(256), 0, st,
                       static_cast<const C*>(pack), static_cast<C*>(spec), starts, list, half, slen, pl->ola_waves,
                       tw2_of<T>(pl));
  }
  if (pl->radix_r == 1) return transform_m2<T, +1>(pl, spec, x, ws + lay.tmp, segs, st, K_SYN, K_SYN1, K_SYN2);
  void* tmp = ws + lay.tmp;
  void* tmp2 = ws + lay.tmp2;
  if (!launch_radix<T, +1>(pl, spec, tmp2, segs, st)) return false;
  void* f = pl->four_step ? tmp2 : tmp;
  if (!transform_m2<T, +1>(pl, tmp2, f, tmp, segs * pl->radix_r, st, K_SYN, K_SYN1, K_SYN2)) return false;
  Timed tm(pl, K_SYN_PERM, st);
  hipLaunchKernelGGL((k_permute<T, false>), dim3(unsigned((half + 255) / 256), unsigned(segs)), dim3(256), 0, st,
                     static_cast<const C*>(f), static_cast<C*>(x), pl->radix_r, pl->m2);
  return true;
}

// Dense tiles of a chunk: the kept DFT_{N_out} slots of every row (scaled),
// placed at their bins of an N-point row, then N-point inverse transforms.
// N a power of two: placed in `dtmp` and transformed into `dense` (one pass),
// or placed in `dense`, first pass into `dtmp`, second pass back into `dense`.
// N = r * Md (r = 3, 5): the radix-r combination first (decimated rows
// A_n1), then the Md-point transforms of the r rows, then the rows back to
// the natural order:
//   one pass:  place -> dtmp, radix -> dense, transform -> dtmp, permute -> dense;
//   two passes: place -> dense, radix -> dtmp, pass 1 -> dense, pass 2 -> dtmp,
//               permute -> dense.
template <typename T>
bool run_dense(qtam_plan_s* pl, const void* y, void* dense, int64_t segs, char* ws, const WsLayout& lay, void* dtmp,
               hipStream_t st) {
  using C = typename Complex<T>::type;
  const HostPlan& hp = pl->hp;
  if (!inverse_rows<T>(pl, T_DENSE, y, segs, ws, lay, st)) return false;
  const int64_t count = segs * hp.rows;
  const int r = pl->radix_r;
  const int64_t md = pl->dense_md;
  {
    Timed tm(pl, K_DENSE_PLACE, st);
    hipLaunchKernelGGL((k_place<T>), dim3(unsigned((hp.n + 255) / 256), unsigned(count)), dim3(256), 0, st,
                       static_cast<const C*>(static_cast<void*>(ws + lay.pack)),
                       static_cast<C*>(pl->dense_four_step ? dense : dtmp), pl->d_rows, hp.rows, hp.n, hp.sum_len);
  }
  // the buffer holding the placed rows, and the other one
  void* a = pl->dense_four_step ? dense : dtmp;
  void* b = pl->dense_four_step ? dtmp : dense;
  if (r > 1) {
    Timed tm(pl, K_DENSE_RADIX, st);
    const dim3 grid(unsigned((md + 255) / 256), unsigned(count));
    if (r == 3)
      hipLaunchKernelGGL((k_radix<T, 3, +1, 1>), grid, dim3(256), 0, st, static_cast<const C*>(a),
                         static_cast<C*>(b), md, tw2_of<T>(pl));
    else if (r == 5)
      hipLaunchKernelGGL((k_radix<T, 5, +1, 1>), grid, dim3(256), 0, st, static_cast<const C*>(a),
                         static_cast<C*>(b), md, tw2_of<T>(pl));
    else
      return false;
    std::swap(a, b);
  }
  // Md-point transforms of the rows in `a`, result in `b`
  const int64_t rows = count * r;
  bool ok;
  if (!pl->dense_four_step) {
    Timed tm(pl, K_DENSE_FFT, st);
    ok = launch_fft_rows<T, +1>(ilog2(md), a, b, rows, md, pl->d_tw_dense, st);
  } else {
    {
      Timed tm(pl, K_DENSE_FFT1, st);
      ok = launch_fft_cols<T, +1>(ilog2(pl->dn2), a, b, pl->dn1, rows, md, pl->d_tw_dn2, tw2_of<T>(pl), st, r);
    }
    if (ok) {
      Timed tm(pl, K_DENSE_FFT2, st);
      ok = launch_fft_rows_t<T, +1>(ilog2(pl->dn1), b, a, pl->dn2, rows, md, pl->d_tw_dn1, st);
    }
    std::swap(a, b);
  }
  if (!ok || r == 1) return ok;
  Timed tm(pl, K_DENSE_PERM, st);
  hipLaunchKernelGGL((k_permute<T, false>), dim3(unsigned((hp.n + 255) / 256), unsigned(count)), dim3(256), 0, st,
                     static_cast<const C*>(b), static_cast<C*>(a), r, md);
  return true;
}

// Segments per dense chunk: rows index grid.y, each chunk's tiles below 2 GiB.
int64_t dense_chunk_cap(const qtam_plan_s* pl) {
  const HostPlan& hp = pl->hp;
  const size_t per = size_t(hp.rows) * size_t(hp.n) * (hp.precision == QTAM_FP64 ? 16 : 8);
  int64_t cap = std::min<int64_t>(chunk_cap(pl), 65535 / (int64_t(hp.rows) * pl->radix_r));
  cap = std::min<int64_t>(cap, per >= (size_t(1) << 31) ? 0 : int64_t(((size_t(1) << 31) - 1) / per));
  return cap;
}

size_t dense_ws_bytes(const qtam_plan_s* pl, int64_t segs) {
  const size_t cb = pl->hp.precision == QTAM_FP64 ? 16 : 8;
  return align256(layout_for(pl, segs).total) + size_t(segs) * size_t(pl->hp.rows) * size_t(pl->hp.n) * cb;
}

// Single-tile recovery of row `row`: its N_out-point forward transform in one
// workgroup, or (rows longer than that) k_fft_cols over that row of each
// segment into the long-row workspace, then k_tile_rows_rowst.
template <typename T>
bool launch_tile_rows(qtam_plan_s* pl, const void* y, void* sx, int row, int64_t segs, char* ws, const WsLayout& lay,
                      hipStream_t st) {
  using C = typename Complex<T>::type;
  const HostPlan& hp = pl->hp;
  Timed tm(pl, K_INV_ROWS, st);
  if (pl->big_rows) {
    const Twiddle2<C> twr{static_cast<const C*>(pl->d_twr_fine), static_cast<const C*>(pl->d_twr_coarse),
                          pl->twr_bits};
    const int64_t stride = int64_t(hp.rows) * hp.n_out;   // row `row` of consecutive segments
    const C* yr = static_cast<const C*>(y) + int64_t(row) * hp.n_out;
    C* A = reinterpret_cast<C*>(ws + lay.rows) + int64_t(row) * hp.n_out;
    if (!launch_fft_cols<T, -1>(ilog2(pl->r2), yr, A, pl->r1, segs, stride, pl->d_tw_r2, twr, st, 1)) return false;
    switch (ilog2(pl->r1)) {
#define X(LG)                                                                                          \
  case LG:                                                                                             \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Col32 : kMaxLog2Col64)) {                          \
      using Geo = ColGeom<T, (1 << LG)>;                                                               \
      if (pl->r2 % Geo::CC) return false;                                                              \
      hipLaunchKernelGGL((k_tile_rows_rowst<T, (1 << LG)>), dim3(unsigned(pl->r2 / Geo::CC), unsigned(segs)), \
                         dim3(Geo::NT), 0, st, A, static_cast<C*>(sx), pl->d_rows,                     \
                         static_cast<const T*>(pl->d_tab[T_TILE]), row, int(hp.half), stride,          \
                         int64_t(hp.n_out), pl->r2, static_cast<const C*>(pl->d_tw_r1));               \
      return true;                                                                                     \
    }                                                                                                  \
    return false;
      QTAM_COL_CASES(X)
#undef X
      default: return false;
    }
  }
  switch (ilog2(hp.n_out)) {
#define X(LG)                                                                                          \
  case LG:                                                                                             \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Rows32 : kMaxLog2Rows64)) {                        \
      using Geo = RowGeom<T, (1 << LG)>;                                                               \
      hipLaunchKernelGGL((k_tile_rows<T, (1 << LG)>), dim3(unsigned((segs + Geo::G - 1) / Geo::G)),      \
                         dim3(Geo::NT), 0, st, static_cast<const C*>(y), static_cast<C*>(sx), pl->d_rows, \
                         static_cast<const T*>(pl->d_tab[T_TILE]), hp.rows, row, int(segs), int(hp.half),  \
                         static_cast<const C*>(pl->d_tw_out));                                         \
      return true;                                                                                     \
    }                                                                                                  \
    return false;
    QTAM_POW2_CASES(X)
#undef X
    default: return false;
  }
}

enum Op { OP_FORWARD, OP_INVERSE, OP_FWD_ADJ, OP_INV_ADJ };

// Bytes at the start of a masked adjoint's workspace for the gain
// gradient's partial sums (one real per segment and row), 256-aligned.
size_t mask_part_bytes(const qtam_plan_s* pl, int64_t batch) {
  const size_t b = size_t(batch) * size_t(pl->hp.rows) * (pl->hp.precision == QTAM_FP64 ? 8 : 4);
  return (b + 255) & ~size_t(255);
}

// mk: the denoiser's mask fused into a masked inverse (OP_INVERSE: gain,
// lam) or its adjoint (OP_INV_ADJ: also y; the partial sums take the start
// of ws and the gain gradient goes to dgain). Only rows transformed in one
// workgroup (power-of-two N_out up to 32768 FP32 / 8192 FP64) take it.
qtam_status run_op(qtam_plan_t pl, Op op, const void* in, void* out, int64_t batch, void* ws, size_t ws_bytes,
                   qtam_stream_t stream, void* stats = nullptr, const MaskArgs* mk = nullptr,
                   void* dgain = nullptr) {
  if (!pl || batch < 0) return QTAM_ERR_INVALID_ARG;
  if (batch == 0) return QTAM_OK;
  if (!in || !out || !ws) return QTAM_ERR_INVALID_ARG;
  if (!pl->gpu_supported) return pl->unsupported_reason;
  if (!pl->device) return QTAM_ERR_INVALID_ARG;
  if (mk && (pl->big_rows || pl->bluestein)) return QTAM_ERR_UNSUPPORTED;
  const HostPlan& hp = pl->hp;
  const bool f64 = hp.precision == QTAM_FP64;
  const size_t rb = f64 ? 8 : 4;
  const size_t part_bytes = (mk && op == OP_INV_ADJ) ? mask_part_bytes(pl, batch) : 0;
  if (part_bytes && ws_bytes <= part_bytes) return QTAM_ERR_WORKSPACE;
  char* part = static_cast<char*>(ws);
  char* tws = static_cast<char*>(ws) + part_bytes;
  const int64_t chunk = std::min<int64_t>(chunk_for(pl, batch, ws_bytes - part_bytes), 65535);
  if (chunk < 1) return QTAM_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t x_seg = size_t(hp.n) * rb;
  const size_t y_seg = size_t(hp.rows) * size_t(hp.n_out) * 2 * rb;
  const bool analysis = (op == OP_FORWARD || op == OP_INV_ADJ);
  const int table = op == OP_FORWARD ? T_FWD : op == OP_INVERSE ? T_DUAL : op == OP_FWD_ADJ ? T_AFWD : T_AINV;
  (void)hipGetLastError();
  for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
    const int64_t segs = std::min(chunk, batch - b0);
    const WsLayout lay = layout_for(pl, segs);
    const char* src = static_cast<const char*>(in) + size_t(b0) * (analysis ? x_seg : y_seg);
    char* dst = static_cast<char*>(out) + size_t(b0) * (analysis ? y_seg : x_seg);
    bool ok;
    void* chunk_stats = stats ? static_cast<char*>(stats) + size_t(b0) * size_t(hp.rows) * 2 * rb : nullptr;
    MaskArgs ck{};
    const MaskArgs* cm = nullptr;
    if (mk) {
      ck = *mk;
      if (op == OP_INV_ADJ) {
        ck.y = static_cast<const char*>(mk->y) + size_t(b0) * y_seg;
        ck.part = part + size_t(b0) * size_t(hp.rows) * rb;
      }
      cm = &ck;
    }
    if (analysis)
      ok = f64 ? run_analysis<double>(pl, table, src, dst, segs, tws, lay, st, chunk_stats, cm)
               : run_analysis<float>(pl, table, src, dst, segs, tws, lay, st, chunk_stats, cm);
    else
      ok = f64 ? run_synthesis<double>(pl, table, src, dst, segs, tws, lay, st, cm)
               : run_synthesis<float>(pl, table, src, dst, segs, tws, lay, st, cm);
    if (!ok) return QTAM_ERR_UNSUPPORTED;
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return hip_failed(e, "kernel launch");
  }
  if (part_bytes) {
    // the gain gradient: the rows' partial sums added over the segments
    Timed tm(pl, K_MASK_BWD, st);
    if (f64)
      hipLaunchKernelGGL((k_gain_sum<double>), dim3(unsigned(hp.rows)), dim3(64), 0, st,
                         reinterpret_cast<const double*>(part), static_cast<double*>(dgain), hp.rows, batch);
    else
      hipLaunchKernelGGL((k_gain_sum<float>), dim3(unsigned(hp.rows)), dim3(64), 0, st,
                         reinterpret_cast<const float*>(part), static_cast<float*>(dgain), hp.rows, batch);
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return hip_failed(e, "kernel launch");
  }
  return QTAM_OK;
}

// Which sizes the kernels cover; sets the four-step split of N/2.
void choose_geometry(qtam_plan_s* pl) {
  const HostPlan& hp = pl->hp;
  const bool f64 = hp.precision == QTAM_FP64;
  const int max_single = f64 ? kMaxLog2Single64 : kMaxLog2Single32;
  pl->gpu_supported = false;
  pl->unsupported_reason = QTAM_ERR_UNSUPPORTED;
  // N_out not a power of two: chirp-z rows of the next power of two >= 2 N_out - 1,
  // in one workgroup, or (longer) as r1 x r2 four-step transforms
  pl->bluestein = !is_pow2(hp.n_out);
  pl->bs_long = false;
  if (pl->bluestein) {
    int64_t lb = 1;
    while (lb < 2 * int64_t(hp.n_out) - 1) lb *= 2;
    pl->bs_len = lb;
    const int lg = ilog2(lb);
    if (lg < 2) return;
    if (lg > max_single) {
      pl->bs_long = true;
      const int l2 = lg / 2, l1 = lg - l2;   // bs_len = r1 * r2, r1 >= r2
      pl->r1 = int64_t(1) << l1;
      pl->r2 = int64_t(1) << l2;
      if (l1 > (f64 ? kMaxLog2Col64 : kMaxLog2Col32) || l2 < 3 || hp.rows > 65535) return;
    }
  }
  // N/2 = r * M2 with r in {1, 3, 5} and M2 a power of two
  pl->radix_r = 0;
  for (int r : {1, 3, 5})
    if (hp.half % r == 0 && is_pow2(hp.half / r)) {
      pl->radix_r = r;
      break;
    }
  if (pl->radix_r == 0) {
    pl->radix_r = 1;
    return;
  }
  pl->m2 = hp.half / pl->radix_r;
  const int ln = ilog2(hp.n_out);
  if (ln < 2) return;
  pl->big_rows = !pl->bluestein && ln > (f64 ? kMaxLog2Rows64 : kMaxLog2Rows32);
  if (pl->big_rows) {
    const int l2 = ln / 2, l1 = ln - l2;   // N_out = r1 * r2, r1 >= r2
    pl->r1 = int64_t(1) << l1;
    pl->r2 = int64_t(1) << l2;
    if (l1 > (f64 ? kMaxLog2Col64 : kMaxLog2Col32) || hp.rows > 65535) return;
  }
  const int lh = ilog2(pl->m2);
  if (lh < 3) return;
  if (lh <= std::min(max_single, 13)) {
    pl->four_step = false;
  } else {
    pl->four_step = true;
    const int l2 = lh / 2, l1 = lh - l2;   // M2 = N1 * N2, N1 >= N2
    pl->n1 = int64_t(1) << l1;
    pl->n2 = int64_t(1) << l2;
    if (l1 > (f64 ? kMaxLog2Col64 : kMaxLog2Col32) || l2 < 3) return;
  }
  pl->gpu_supported = true;
  pl->unsupported_reason = QTAM_OK;
  // dense tiles: N-point transforms, N = r * Md with the radix-r split of the
  // spectrum (r = 1, 3, 5); the Md-point transforms in one pass or Md = dn1 * dn2
  pl->dense_ok = false;
  pl->dense_md = hp.n / pl->radix_r;
  {
    const int lt = ilog2(pl->dense_md);
    if (lt <= max_single) {
      pl->dense_four_step = false;
      pl->dense_ok = true;
    } else {
      const int l2 = lt / 2, l1 = lt - l2;
      pl->dense_four_step = true;
      pl->dn1 = int64_t(1) << l1;
      pl->dn2 = int64_t(1) << l2;
      pl->dense_ok = l1 <= (f64 ? kMaxLog2Col64 : kMaxLog2Col32);
    }
  }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
// ---------------------------------------------------------------------------
// Static workspace of qtam_forward_noalloc: a device array of fixed size that
// every device the library runs on holds until the process ends. Host code
// never passes `scratch` itself to a kernel (in host code the name is a
// host-side stand-in): its device address, per device, comes from
// hipGetSymbolAddress once at plan creation with that device current.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = QTAM_NOALLOC_WORKSPACE_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Looks up this device's scratch address once (the device is current).
qtam_status scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return QTAM_OK;   // no static workspace on such devices
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return QTAM_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_failed(e, "hipGetSymbolAddress of the static workspace");
  g_scratch_ptr[device] = ptr;
  return QTAM_OK;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace

namespace {

// Plan creation proper; host allocations may throw std::bad_alloc, which
// qtam_plan_create turns into QTAM_ERR_OOM (*made holds the plan to free).
qtam_status create_plan(const qtam_params* params, qtam_plan_t* out, qtam_plan_s** made) {
  qtam_plan_s* pl = new qtam_plan_s();
  *made = pl;
  qtam_status st = build_host_plan(*params, pl->hp);
  if (st != QTAM_OK) {
    delete pl;
    *made = nullptr;
    return st;
  }
  choose_geometry(pl);
  pl->seg_bytes = layout_for(pl, 1).total;
  if (!(params->flags & QTAM_PLAN_HOST_ONLY) && pl->gpu_supported) {
    const hipError_t e = hipGetDevice(&pl->device_id);
    if (e != hipSuccess) {
      delete pl;
      *made = nullptr;
      return hip_failed(e, "hipGetDevice");
    }
    if (hipDeviceGetAttribute(&pl->num_cus, hipDeviceAttributeMultiprocessorCount, pl->device_id) != hipSuccess ||
        pl->num_cus < 1) {
      (void)hipGetLastError();
      pl->num_cus = 1;
    }
    pl->analytic_fwd = pl->hp.all_bisquare && pl->hp.eps == 0.0;
    st = scratch_setup(pl->device_id);
    if (st != QTAM_OK) {
      delete pl;
      *made = nullptr;
      return st;
    }
    st = pl->hp.precision == QTAM_FP64 ? upload<double>(pl) : upload<float>(pl);
    if (st != QTAM_OK) {
      if (pl->dmem) (void)hipFree(pl->dmem);
      delete pl;
      *made = nullptr;
      return st;
    }
    pl->device = true;
  }
  *out = pl;
  return QTAM_OK;
}

}  // namespace

extern "C" {

const char* qtam_last_error(void) { return g_last_error.c_str(); }

const char* qtam_version(void) { return "qtam-gfx950 1.0"; }

const char* qtam_status_string(qtam_status s) {
  switch (s) {
    case QTAM_OK: return "ok";
    case QTAM_ERR_INVALID_ARG: return "invalid argument";
    case QTAM_ERR_UNSUPPORTED: return "unsupported on this device path";
    case QTAM_ERR_WORKSPACE: return "workspace too small";
    case QTAM_ERR_OOM: return "out of memory (device, or host tables)";
    case QTAM_ERR_DEVICE: return "HIP device error";
  }
  return "unknown status";
}

qtam_status qtam_plan_create(const qtam_params* params, qtam_plan_t* out) {
  if (!out) return QTAM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!params) return QTAM_ERR_INVALID_ARG;
  qtam_plan_s* made = nullptr;
  try {
    return create_plan(params, out, &made);
  } catch (const std::bad_alloc&) {
    // host tables too large: nothing leaks, nothing crosses the C boundary
    if (made) {
      if (made->dmem) (void)hipFree(made->dmem);
      delete made;
    }
    *out = nullptr;
    g_last_error = "qtam_plan_create: host memory exhausted building the plan tables";
    return QTAM_ERR_OOM;
  }
}

qtam_status qtam_plan_info(qtam_plan_t pl, qtam_plan_info_t* info) {
  if (!pl || !info) return QTAM_ERR_INVALID_ARG;
  const HostPlan& hp = pl->hp;
  info->n_rows = hp.rows;
  info->n_planes = hp.planes;
  info->rows_per_plane = hp.rows_per_plane;
  info->row_q = hp.row_q.data();
  info->n_out = hp.n_out;
  info->max_len = hp.max_len;
  info->precision = hp.precision;
  info->n_samples = hp.n;
  info->n_bins = hp.n_bins;
  info->sum_len = hp.sum_len;
  info->l_max = hp.l_max;
  info->frame_A = hp.frame_A;
  info->frame_B = hp.frame_B;
  info->masked_fraction = hp.masked_fraction;
  info->workspace_bytes_per_segment = pl->seg_bytes;
  info->freqs = hp.freq.data();
  info->centre = hp.centre.data();
  info->half_width = hp.half_width.data();
  info->lo = hp.lo.data();
  info->hi = hp.hi.data();
  info->offset = hp.offset.data();
  info->window = hp.win.data();
  info->frame = hp.P.data();
  info->mask = hp.M.data();
  return QTAM_OK;
}

void qtam_plan_destroy(qtam_plan_t pl) {
  if (!pl) return;
  for (auto& p : pl->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : pl->pool) (void)hipEventDestroy(e);
  if (pl->dmem) (void)hipFree(pl->dmem);
  delete pl;
}

size_t qtam_workspace_size(qtam_plan_t pl, int64_t batch) {
  if (!pl || batch < 1) return 0;
  return layout_for(pl, batch).total;
}

qtam_status qtam_forward(qtam_plan_t pl, const void* x, void* y, int64_t batch, void* ws, size_t ws_bytes,
                         qtam_stream_t stream) {
  return run_op(pl, OP_FORWARD, x, y, batch, ws, ws_bytes, stream);
}

qtam_status qtam_forward_noalloc(qtam_plan_t pl, const void* x, void* y, int64_t batch, qtam_stream_t stream) {
  if (!pl || batch < 0) return QTAM_ERR_INVALID_ARG;
  if (!pl->gpu_supported) return pl->unsupported_reason;
  if (pl->seg_bytes > kScratchBytes) {
    g_last_error = "qtam_forward_noalloc: one segment of this plan needs " + std::to_string(pl->seg_bytes) +
                   " workspace bytes, above the static workspace of " + std::to_string(kScratchBytes);
    return QTAM_ERR_WORKSPACE;
  }
  if (batch == 0) return QTAM_OK;
  if (!pl->device) return QTAM_ERR_INVALID_ARG;
  void* ws = scratch_of(pl->device_id);
  if (!ws) return QTAM_ERR_INVALID_ARG;
  // every region of the workspace is written before it is read: nothing to clear
  g_untimed = true;
  const qtam_status st = run_op(pl, OP_FORWARD, x, y, batch, ws, kScratchBytes, stream);
  g_untimed = false;
  return st;
}

qtam_status qtam_forward_metric(qtam_plan_t pl, const void* x, void* y, void* metric, int64_t batch, void* ws,
                                size_t ws_bytes, qtam_stream_t stream) {
  if (batch > 0 && !metric) return QTAM_ERR_INVALID_ARG;
  return run_op(pl, OP_FORWARD, x, y, batch, ws, ws_bytes, stream, metric);
}

qtam_status qtam_forward_sweep(const qtam_plan_t* plans, int32_t n_plans, const void* x, void* const* y,
                               int64_t batch, void* ws, size_t ws_bytes, qtam_stream_t stream) {
  if (!plans || n_plans < 1 || batch < 0) return QTAM_ERR_INVALID_ARG;
  for (int32_t i = 0; i < n_plans; ++i)
    if (!plans[i]) return QTAM_ERR_INVALID_ARG;
  const qtam_plan_s* p0 = plans[0];
  for (int32_t i = 0; i < n_plans; ++i) {
    const qtam_plan_s* p = plans[i];
    if (p->hp.n != p0->hp.n || p->hp.precision != p0->hp.precision) return QTAM_ERR_INVALID_ARG;
  }
  if (batch == 0) return QTAM_OK;
  if (!x || !y || !ws) return QTAM_ERR_INVALID_ARG;
  int64_t chunk = 65535;
  for (int32_t i = 0; i < n_plans; ++i) {
    const qtam_plan_s* p = plans[i];
    if (!y[i]) return QTAM_ERR_INVALID_ARG;
    if (!p->gpu_supported) return p->unsupported_reason;
    if (!p->device || p->device_id != p0->device_id) return QTAM_ERR_INVALID_ARG;
    chunk = std::min(chunk, chunk_for(p, batch, ws_bytes));
  }
  if (chunk < 1) return QTAM_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool f64 = p0->hp.precision == QTAM_FP64;
  const size_t rb = f64 ? 8 : 4;
  (void)hipGetLastError();
  for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
    const int64_t segs = std::min(chunk, batch - b0);
    const char* src = static_cast<const char*>(x) + size_t(b0) * size_t(p0->hp.n) * rb;
    // the spectrum sits at the start of every plan's workspace layout, with the
    // same size, so the first plan computes it and every plan reads it
    qtam_plan_s* first = plans[0];
    const WsLayout lay0 = layout_for(first, segs);
    bool ok = f64 ? analysis_spectrum<double>(first, src, segs, static_cast<char*>(ws), lay0, st)
                  : analysis_spectrum<float>(first, src, segs, static_cast<char*>(ws), lay0, st);
    for (int32_t i = 0; ok && i < n_plans; ++i) {
      qtam_plan_s* p = plans[i];
      const WsLayout lay = layout_for(p, segs);
      const size_t y_seg = size_t(p->hp.rows) * size_t(p->hp.n_out) * 2 * rb;
      char* dst = static_cast<char*>(y[i]) + size_t(b0) * y_seg;
      ok = f64 ? analysis_rows<double>(p, T_FWD, dst, segs, static_cast<char*>(ws), lay, st, nullptr)
               : analysis_rows<float>(p, T_FWD, dst, segs, static_cast<char*>(ws), lay, st, nullptr);
    }
    if (!ok) return QTAM_ERR_UNSUPPORTED;
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return hip_failed(e, "kernel launch");
  }
  return QTAM_OK;
}

qtam_status qtam_select_planes(qtam_plan_t pl, const void* y, const void* metric, int32_t kind, void* score,
                               int32_t* best, void* y_best, int64_t batch, qtam_stream_t stream) {
  if (!pl || batch < 0 || (kind != QTAM_METRIC_ENERGY && kind != QTAM_METRIC_PEAK)) return QTAM_ERR_INVALID_ARG;
  if (batch == 0) return QTAM_OK;
  if (!y || !metric || !best || !y_best) return QTAM_ERR_INVALID_ARG;
  if (!pl->gpu_supported) return pl->unsupported_reason;
  if (!pl->device) return QTAM_ERR_INVALID_ARG;
  const HostPlan& hp = pl->hp;
  const bool f64 = hp.precision == QTAM_FP64;
  const size_t cb = f64 ? 16 : 8;
  const int64_t units = int64_t(hp.rows_per_plane) * hp.n_out * int64_t(cb) / 16;
  const int64_t gx = std::min<int64_t>((units + 255) / 256, 1024);
  hipStream_t st = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
    const int64_t segs = std::min<int64_t>(65535, batch - b0);
    const char* ys = static_cast<const char*>(y) + size_t(b0) * size_t(hp.rows) * size_t(hp.n_out) * cb;
    const char* ms = static_cast<const char*>(metric) + size_t(b0) * size_t(hp.rows) * cb;
    char* sc = score ? static_cast<char*>(score) + size_t(b0) * size_t(hp.planes) * cb / 2 : nullptr;
    {
      Timed tm(pl, K_PLANE_BEST, st);
      if (f64)
        hipLaunchKernelGGL((k_plane_best<double>), dim3(unsigned(segs)), dim3(256), 0, st,
                           reinterpret_cast<const double2*>(ms), hp.rows_per_plane, hp.planes,
                           int(kind == QTAM_METRIC_PEAK), reinterpret_cast<double*>(sc), best + b0);
      else
        hipLaunchKernelGGL((k_plane_best<float>), dim3(unsigned(segs)), dim3(256), 0, st,
                           reinterpret_cast<const float2*>(ms), hp.rows_per_plane, hp.planes,
                           int(kind == QTAM_METRIC_PEAK), reinterpret_cast<float*>(sc), best + b0);
    }
    Timed tm(pl, K_GATHER, st);
    hipLaunchKernelGGL(k_gather_plane, dim3(unsigned(gx), unsigned(segs)), dim3(256), 0, st,
                       reinterpret_cast<const uint4*>(ys), best + b0,
                       reinterpret_cast<uint4*>(static_cast<char*>(y_best) + size_t(b0) * size_t(units) * 16), units,
                       hp.planes);
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return hip_failed(e, "kernel launch");
  }
  return QTAM_OK;
}

qtam_status qtam_tile_inverse(qtam_plan_t pl, const void* y, int32_t row, void* x, int64_t batch, void* ws,
                              size_t ws_bytes, qtam_stream_t stream) {
  if (!pl || batch < 0 || row < 0 || row >= pl->hp.rows || !(pl->hp.eps > 0.0)) return QTAM_ERR_INVALID_ARG;
  if (batch == 0) return QTAM_OK;
  if (!y || !x || !ws) return QTAM_ERR_INVALID_ARG;
  if (!pl->gpu_supported) return pl->unsupported_reason;
  if (pl->bluestein) return QTAM_ERR_UNSUPPORTED;
  if (!pl->device) return QTAM_ERR_INVALID_ARG;
  const int64_t chunk = std::min<int64_t>(chunk_for(pl, batch, ws_bytes), 65535);
  if (chunk < 1) return QTAM_ERR_WORKSPACE;
  const HostPlan& hp = pl->hp;
  const bool f64 = hp.precision == QTAM_FP64;
  const size_t rb = f64 ? 8 : 4;
  hipStream_t st = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
    const int64_t segs = std::min(chunk, batch - b0);
    const WsLayout lay = layout_for(pl, segs);
    char* w = static_cast<char*>(ws);
    const char* src = static_cast<const char*>(y) + size_t(b0) * size_t(hp.rows) * size_t(hp.n_out) * 2 * rb;
    char* dst = static_cast<char*>(x) + size_t(b0) * size_t(hp.n) * rb;
    void* sx = w + lay.pack;   // [segs][N/2 + 1], within the packed region (R (N/2 + 1) entries per segment)
    const bool ok = f64 ? (launch_tile_rows<double>(pl, src, sx, row, segs, w, lay, st) &&
                           synthesize<double>(pl, sx, hp.half + 1, pl->d_one_start, pl->d_one_rows, dst, segs, w, lay, st))
                        : (launch_tile_rows<float>(pl, src, sx, row, segs, w, lay, st) &&
                           synthesize<float>(pl, sx, hp.half + 1, pl->d_one_start, pl->d_one_rows, dst, segs, w, lay, st));
    if (!ok) return QTAM_ERR_UNSUPPORTED;
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return hip_failed(e, "kernel launch");
  }
  return QTAM_OK;
}

size_t qtam_mask_workspace_size(qtam_plan_t pl, int64_t batch) {
  if (!pl || batch < 1) return 0;
  return size_t(batch) * size_t(pl->hp.rows) * (pl->hp.precision == QTAM_FP64 ? 8 : 4);
}

qtam_status qtam_mask_forward(qtam_plan_t pl, const void* y, const void* gain, const void* lambda, void* out,
                              int64_t batch, qtam_stream_t stream) {
  if (!pl || batch < 0) return QTAM_ERR_INVALID_ARG;
  if (batch == 0) return QTAM_OK;
  if (!y || !gain || !lambda || !out || !pl->device) return QTAM_ERR_INVALID_ARG;
  const HostPlan& hp = pl->hp;
  const bool f64 = hp.precision == QTAM_FP64;
  const size_t cb = f64 ? 16 : 8;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t chunk = std::max<int64_t>(1, 65535 / hp.rows);   // rows of a chunk index grid.y
  (void)hipGetLastError();
  for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
    const int64_t segs = std::min(chunk, batch - b0);
    const size_t off = size_t(b0) * size_t(hp.rows) * size_t(hp.n_out) * cb;
    const dim3 grid(unsigned((hp.n_out + 255) / 256), unsigned(segs * hp.rows));
    Timed tm(pl, K_MASK_FWD, st);
    if (f64)
      hipLaunchKernelGGL((k_mask_fwd<double>), grid, dim3(256), 0, st,
                         reinterpret_cast<const double2*>(static_cast<const char*>(y) + off),
                         static_cast<const double*>(gain), static_cast<const double*>(lambda),
                         reinterpret_cast<double2*>(static_cast<char*>(out) + off), hp.rows, hp.n_out);
    else
      hipLaunchKernelGGL((k_mask_fwd<float>), grid, dim3(256), 0, st,
                         reinterpret_cast<const float2*>(static_cast<const char*>(y) + off),
                         static_cast<const float*>(gain), static_cast<const float*>(lambda),
                         reinterpret_cast<float2*>(static_cast<char*>(out) + off), hp.rows, hp.n_out);
  }
  if (const hipError_t e = hipGetLastError(); e != hipSuccess) return hip_failed(e, "kernel launch");
  return QTAM_OK;
}

qtam_status qtam_mask_backward(qtam_plan_t pl, const void* y, const void* gain, const void* lambda, const void* gout,
                               void* gy, void* dgain, int64_t batch, void* ws, size_t ws_bytes,
                               qtam_stream_t stream) {
  if (!pl || batch < 0) return QTAM_ERR_INVALID_ARG;
  if (!gain || !lambda || !dgain || !pl->device) return QTAM_ERR_INVALID_ARG;
  if (batch > 0 && (!y || !gout || !gy || !ws)) return QTAM_ERR_INVALID_ARG;
  const HostPlan& hp = pl->hp;
  const bool f64 = hp.precision == QTAM_FP64;
  hipStream_t st = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  if (batch > 0) {
    if (ws_bytes < qtam_mask_workspace_size(pl, batch)) return QTAM_ERR_WORKSPACE;
    if (batch * int64_t(hp.rows) > int64_t(0x7fffffff)) return QTAM_ERR_INVALID_ARG;   // rows index grid.x
    Timed tm(pl, K_MASK_BWD, st);
    const dim3 grid(unsigned(batch * hp.rows));
    if (f64)
      hipLaunchKernelGGL((k_mask_bwd<double>), grid, dim3(256), 0, st, static_cast<const double2*>(y),
                         static_cast<const double2*>(gout), static_cast<const double*>(gain),
                         static_cast<const double*>(lambda), static_cast<double2*>(gy), static_cast<double*>(ws),
                         hp.rows, hp.n_out);
    else
      hipLaunchKernelGGL((k_mask_bwd<float>), grid, dim3(256), 0, st, static_cast<const float2*>(y),
                         static_cast<const float2*>(gout), static_cast<const float*>(gain),
                         static_cast<const float*>(lambda), static_cast<float2*>(gy), static_cast<float*>(ws),
                         hp.rows, hp.n_out);
  }
  // the gain gradient: the rows' partial sums added over the segments, one
  // wave per row in a fixed order (0 for an empty batch)
  const dim3 g2(unsigned(hp.rows));
  if (f64)
    hipLaunchKernelGGL((k_gain_sum<double>), g2, dim3(64), 0, st, static_cast<const double*>(ws),
                       static_cast<double*>(dgain), hp.rows, batch);
  else
    hipLaunchKernelGGL((k_gain_sum<float>), g2, dim3(64), 0, st, static_cast<const float*>(ws),
                       static_cast<float*>(dgain), hp.rows, batch);
  if (const hipError_t e = hipGetLastError(); e != hipSuccess) return hip_failed(e, "kernel launch");
  return QTAM_OK;
}

size_t qtam_dense_workspace_size(qtam_plan_t pl, int64_t batch) {
  if (!pl || batch < 1 || !pl->dense_ok) return 0;
  const int64_t cap = dense_chunk_cap(pl);
  if (cap < 1) return 0;
  return dense_ws_bytes(pl, std::min(batch, cap));
}

qtam_status qtam_dense(qtam_plan_t pl, const void* y, void* dense, int64_t batch, void* ws, size_t ws_bytes,
                       qtam_stream_t stream) {
  if (!pl || batch < 0) return QTAM_ERR_INVALID_ARG;
  if (batch == 0) return QTAM_OK;
  if (!y || !dense || !ws) return QTAM_ERR_INVALID_ARG;
  if (!pl->gpu_supported) return pl->unsupported_reason;
  if (!pl->dense_ok || dense_chunk_cap(pl) < 1) return QTAM_ERR_UNSUPPORTED;
  if (!pl->device) return QTAM_ERR_INVALID_ARG;
  const HostPlan& hp = pl->hp;
  const bool f64 = hp.precision == QTAM_FP64;
  const size_t cb = f64 ? 16 : 8;
  int64_t chunk = std::min(batch, dense_chunk_cap(pl));
  while (chunk > 1 && dense_ws_bytes(pl, chunk) > ws_bytes) --chunk;
  if (dense_ws_bytes(pl, chunk) > ws_bytes) return QTAM_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  for (int64_t b0 = 0; b0 < batch; b0 += chunk) {
    const int64_t segs = std::min(chunk, batch - b0);
    const WsLayout lay = layout_for(pl, segs);
    char* w = static_cast<char*>(ws);
    void* dtmp = w + align256(lay.total);
    const char* src = static_cast<const char*>(y) + size_t(b0) * size_t(hp.rows) * size_t(hp.n_out) * cb;
    char* dst = static_cast<char*>(dense) + size_t(b0) * size_t(hp.rows) * size_t(hp.n) * cb;
    const bool ok = f64 ? run_dense<double>(pl, src, dst, segs, w, lay, dtmp, st)
                        : run_dense<float>(pl, src, dst, segs, w, lay, dtmp, st);
    if (!ok) return QTAM_ERR_UNSUPPORTED;
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return hip_failed(e, "kernel launch");
  }
  return QTAM_OK;
}

qtam_status qtam_inverse(qtam_plan_t pl, const void* y, void* x, int64_t batch, void* ws, size_t ws_bytes,
                         qtam_stream_t stream) {
  return run_op(pl, OP_INVERSE, y, x, batch, ws, ws_bytes, stream);
}

qtam_status qtam_forward_adjoint(qtam_plan_t pl, const void* gy, void* gx, int64_t batch, void* ws,
                                 size_t ws_bytes, qtam_stream_t stream) {
  return run_op(pl, OP_FWD_ADJ, gy, gx, batch, ws, ws_bytes, stream);
}

qtam_status qtam_inverse_adjoint(qtam_plan_t pl, const void* gx, void* gy, int64_t batch, void* ws,
                                 size_t ws_bytes, qtam_stream_t stream) {
  return run_op(pl, OP_INV_ADJ, gx, gy, batch, ws, ws_bytes, stream);
}

qtam_status qtam_inverse_masked(qtam_plan_t pl, const void* y, const void* gain, const void* lambda, void* x,
                                int64_t batch, void* ws, size_t ws_bytes, qtam_stream_t stream) {
  if (!pl || batch < 0) return QTAM_ERR_INVALID_ARG;
  if (!pl->gpu_supported) return pl->unsupported_reason;
  if (pl->big_rows || pl->bluestein) return QTAM_ERR_UNSUPPORTED;   // also for batch = 0: a query
  if (batch == 0) return QTAM_OK;
  if (!gain || !lambda) return QTAM_ERR_INVALID_ARG;
  const MaskArgs mk{nullptr, gain, lambda, nullptr};
  return run_op(pl, OP_INVERSE, y, x, batch, ws, ws_bytes, stream, nullptr, &mk);
}

size_t qtam_masked_adjoint_workspace_size(qtam_plan_t pl, int64_t batch) {
  if (!pl || batch < 1) return 0;
  return mask_part_bytes(pl, batch) + layout_for(pl, batch).total;
}

qtam_status qtam_inverse_masked_adjoint(qtam_plan_t pl, const void* gx, const void* y, const void* gain,
                                        const void* lambda, void* gy, void* dgain, int64_t batch, void* ws,
                                        size_t ws_bytes, qtam_stream_t stream) {
  if (!pl || batch < 0 || !gain || !lambda || !dgain) return QTAM_ERR_INVALID_ARG;
  if (batch > 0 && !y) return QTAM_ERR_INVALID_ARG;
  if (!pl->gpu_supported) return pl->unsupported_reason;
  if (pl->big_rows || pl->bluestein) return QTAM_ERR_UNSUPPORTED;
  if (!pl->device) return QTAM_ERR_INVALID_ARG;
  if (batch == 0) {   // dgain = 0
    hipStream_t st = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    if (pl->hp.precision == QTAM_FP64)
      hipLaunchKernelGGL((k_gain_sum<double>), dim3(unsigned(pl->hp.rows)), dim3(64), 0, st, nullptr,
                         static_cast<double*>(dgain), pl->hp.rows, int64_t(0));
    else
      hipLaunchKernelGGL((k_gain_sum<float>), dim3(unsigned(pl->hp.rows)), dim3(64), 0, st, nullptr,
                         static_cast<float*>(dgain), pl->hp.rows, int64_t(0));
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return hip_failed(e, "kernel launch");
    return QTAM_OK;
  }
  const MaskArgs mk{y, gain, lambda, nullptr};
  return run_op(pl, OP_INV_ADJ, gx, gy, batch, ws, ws_bytes, stream, nullptr, &mk, dgain);
}

qtam_status qtam_timing_enable(qtam_plan_t pl, int32_t on) {
  if (!pl) return QTAM_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(pl->mu);
  pl->timing = on != 0;
  return QTAM_OK;
}

qtam_status qtam_timing_collect(qtam_plan_t pl, const char** names, double* total_ms, int64_t* launches,
                                int32_t max_kinds, int32_t* n_kinds) {
  if (!pl) return QTAM_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(pl->mu);
  qtam_status st = QTAM_OK;
  for (auto& p : pl->pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) {
      (void)hipGetLastError();
      st = QTAM_ERR_DEVICE;
    } else {
      pl->total_ms[p.kind] += ms;
      pl->launches[p.kind] += 1;
    }
    pl->pool.push_back(p.a);
    pl->pool.push_back(p.b);
  }
  pl->pending.clear();
  int32_t n = 0;
  for (int k = 0; k < K_NUM; ++k) {
    if (pl->launches[k] == 0) continue;
    if (n < max_kinds) {
      if (names) names[n] = kKindName[k];
      if (total_ms) total_ms[n] = pl->total_ms[k];
      if (launches) launches[n] = pl->launches[k];
    }
    ++n;
    pl->total_ms[k] = 0.0;
    pl->launches[k] = 0;
  }
  if (n_kinds) *n_kinds = n;
  return st;
}

}  // extern "C"
