/* A C caller of libqtam.so without Python or a GPU: host-only plans, their
 * tables and sizes, and the status codes of calls that fail validation.
 * Built and run by tests/test_abi_host.py (gcc, linked against the library).
 * Prints one line per check and exits non-zero at the first failure. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "qtam.h"

static int failures = 0;
#define CHECK(cond)                                                  \
  do {                                                               \
    if (cond) {                                                      \
      printf("ok   %s\n", #cond);                                    \
    } else {                                                         \
      printf("FAIL %s (line %d)\n", #cond, __LINE__);                \
      ++failures;                                                    \
    }                                                                \
  } while (0)

static qtam_params workload(void) {
  /* one segment: 4 s at 4096 Hz, Q 8, 64 rows from 20 to 1000 Hz */
  qtam_params p;
  memset(&p, 0, sizeof p);
  p.sample_rate = 4096.0;
  p.n_samples = 16384;
  p.q = 8.0;
  p.f_min = 20.0;
  p.f_max = 1000.0;
  p.n_rows = 64;
  p.window = QTAM_WIN_BISQUARE;
  p.cap_mode = QTAM_CAP_COVER;
  p.norm_mode = QTAM_NORM_UNIT_ENERGY;
  p.p_floor_rel = 1e-6;
  p.precision = QTAM_FP32;
  p.flags = QTAM_PLAN_HOST_ONLY;
  return p;
}

int main(void) {
  qtam_params p = workload();
  qtam_plan_t plan = NULL;
  CHECK(qtam_plan_create(&p, &plan) == QTAM_OK && plan != NULL);
  if (!plan) return 1;

  qtam_plan_info_t info;
  CHECK(qtam_plan_info(plan, &info) == QTAM_OK);
  CHECK(info.n_rows == 64 && info.n_planes == 1 && info.n_samples == 16384);
  CHECK(info.n_bins == 8193);
  CHECK(info.n_out >= info.max_len && (info.n_out & (info.n_out - 1)) == 0);
  CHECK(info.frame_A > 0.0 && info.frame_B >= info.frame_A);

  /* rows: centres inside [lo, hi], packed offsets running over sum_len */
  int rows_ok = 1;
  int64_t next = 0;
  for (int k = 0; k < info.n_rows; ++k) {
    rows_ok &= info.lo[k] <= info.centre[k] && info.centre[k] <= info.hi[k];
    rows_ok &= info.offset[k] == next;
    next += info.hi[k] - info.lo[k] + 1;
    rows_ok &= info.freqs[k] >= p.f_min - 1e-9 && info.freqs[k] <= p.f_max + 1e-9;
  }
  CHECK(rows_ok && next == info.sum_len);
  /* the frame P is the sum over rows of W_k^2 on their kept bins, and frame_B its maximum on M */
  static double S[8193];
  double pmax = 0.0, dev = 0.0, bmax = 0.0;
  for (int k = 0; k < info.n_rows; ++k)
    for (int b = info.lo[k]; b <= info.hi[k]; ++b) {
      const double w = info.window[info.offset[k] + (b - info.lo[k])];
      S[b] += w * w;
    }
  for (int64_t b = 0; b < info.n_bins; ++b) {
    pmax = info.frame[b] > pmax ? info.frame[b] : pmax;
    dev = fabs(S[b] - info.frame[b]) > dev ? fabs(S[b] - info.frame[b]) : dev;
    if (info.mask[b] && info.frame[b] > bmax) bmax = info.frame[b];
  }
  CHECK(pmax > 0.0 && dev <= 1e-12 * pmax);
  CHECK(bmax == info.frame_B);

  /* workspace: grows with the batch; the masked adjoint's adds the partial sums */
  size_t w1 = qtam_workspace_size(plan, 1), w8 = qtam_workspace_size(plan, 8);
  CHECK(w1 > 0 && w8 > w1);
  CHECK(qtam_masked_adjoint_workspace_size(plan, 8) >= w8 + (size_t)8 * 64 * 4);
  CHECK(qtam_mask_workspace_size(plan, 8) == (size_t)8 * 64 * 4);

  /* calls that need device tables fail validation on a host-only plan, before any device work */
  char dummy[16];
  CHECK(qtam_forward(plan, dummy, dummy, 1, dummy, w1, NULL) == QTAM_ERR_INVALID_ARG);
  CHECK(qtam_inverse(plan, dummy, dummy, 1, dummy, w1, NULL) == QTAM_ERR_INVALID_ARG);
  CHECK(qtam_forward(plan, dummy, dummy, 0, dummy, w1, NULL) == QTAM_OK);   /* empty batch */
  CHECK(qtam_forward(NULL, dummy, dummy, 1, dummy, w1, NULL) == QTAM_ERR_INVALID_ARG);
  CHECK(qtam_inverse_masked(plan, NULL, NULL, NULL, NULL, 0, NULL, 0, NULL) == QTAM_OK);   /* supported */
  CHECK(strlen(qtam_status_string(QTAM_ERR_UNSUPPORTED)) > 0);
  CHECK(strlen(qtam_version()) > 0);

  /* invalid parameters: odd N, f_max above Nyquist */
  qtam_plan_t bad = NULL;
  qtam_params q = workload();
  q.n_samples = 16385;
  CHECK(qtam_plan_create(&q, &bad) == QTAM_ERR_INVALID_ARG && bad == NULL);
  q = workload();
  q.f_max = 4000.0;
  CHECK(qtam_plan_create(&q, &bad) == QTAM_ERR_INVALID_ARG && bad == NULL);

  qtam_plan_destroy(plan);
  qtam_plan_destroy(NULL);
  printf("%s\n", failures ? "FAILED" : "PASSED");
  return failures ? 1 : 0;
}
