// Host-side QTAM plan: the FP64 tables every launch reads (App. A grid, widths
// and windows; App. C frame operator and canonical dual).
#pragma once

#include <cstdint>
#include <vector>

#include "qtam.h"

namespace qtam {

struct HostPlan {
  // parameters
  double fs = 0.0, q = 0.0, f_min = 0.0, f_max = 0.0, p_floor_rel = 0.0, window_param = 0.0;
  int64_t n = 0;            // N samples per segment
  int64_t half = 0;         // N/2
  int64_t n_bins = 0;       // N/2 + 1
  int32_t rows = 0;         // R, all planes
  int32_t planes = 1;       // planes of a composite bank
  int32_t rows_per_plane = 0;
  bool all_bisquare = true; // every plane uses the bisquare window
  double eps = 0.0;         // regularised stop-band value (0: plain windows)
  int32_t n_out = 0;        // N_out
  int32_t max_len = 0;      // max 2 h_k + 1
  int32_t precision = QTAM_FP32;
  int32_t window = QTAM_WIN_BISQUARE;
  int64_t l_max = -1;       // cap on L_k, -1 if none
  int64_t sum_len = 0;      // sum of kept support lengths

  // per row
  std::vector<double> freq, row_q;
  std::vector<int32_t> centre, half_width, lo, hi;
  std::vector<int64_t> offset;

  // packed per (row, kept bin) tables, row k at [offset[k], offset[k] + hi[k]-lo[k]+1)
  std::vector<double> win;        // W_k[b]
  std::vector<double> fwd_tab;    // forward:  W * sqrt(N_out/N) / N_out
  std::vector<double> dual_tab;   // inverse:  sqrt(N/N_out) * W * M / P / N
  std::vector<double> afwd_tab;   // adjoint of forward: fwd_tab * (1/2 inside, 1 at DC/Nyquist)
  std::vector<double> ainv_tab;   // adjoint of inverse: sqrt(N/N_out) W M / P * c_b / N, c = 2 inside
  std::vector<double> tile_tab;   // single-tile recovery: sqrt(N/N_out) / W / N (eps > 0 only)

  // per bin
  std::vector<double> P;          // frame operator diagonal
  std::vector<uint8_t> M;         // reconstruction mask

  double frame_A = 0.0, frame_B = 0.0, masked_fraction = 0.0;
};

// Builds every host table. Returns QTAM_OK or QTAM_ERR_INVALID_ARG.
qtam_status build_host_plan(const qtam_params& p, HostPlan& hp);

}  // namespace qtam
