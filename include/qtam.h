/*
 * qtam.h - C ABI of the MI355X (gfx950) QTAM library, libqtam.so.
 *
 * QTAM is the Q-transform with amplitude demodulation of Asprea et al.,
 * "QTAM: Q-Transform Amplitude Modulation" (arXiv 2603.29785). For each row k
 * of a log-spaced frequency grid the forward transform filters the real FFT of
 * a segment with a frequency-domain window W_k, rolls the band to baseband and
 * takes a short inverse FFT of length N_out, giving a decimated complex
 * envelope Y_k (Sec. III; App. A). The inverse FFTs each envelope, re-modulates
 * it to its carrier, overlap-adds W_k-weighted tiles, divides by the frame
 * operator P = sum_k |W_k|^2 and returns to the time domain (canonical dual
 * frame, Sec. III inverse equation; App. C).
 *
 * Conventions used by every entry point:
 *   - N samples per segment (even), sample rate fs, T = N/fs seconds.
 *   - DFT X[b] = sum_n x[n] e^{-2 pi i b n/N}, b = 0..N/2 (App. C).
 *   - Envelope Y_k[m] = sqrt(N_out/N) (1/N_out) sum_u Z_k[u] e^{+2 pi i u m/N_out},
 *     Z_k[j mod N_out] = X[s_k + j] W_k[s_k + j] for |j| <= h_k and
 *     0 <= s_k + j <= N/2 (Sec. III renormalisation; App. C demodulation;
 *     N_in is read as N). m = 0 is t = 0; no fftshift.
 *   - Inverse x = irfft( M/P * sum_k W_k * sqrt(N/N_out) DFT_{N_out}(Y_k)[b - s_k] ),
 *     M[b] = [P[b] >= p_floor_rel * max P] (App. C; bins no window covers, or
 *     covers too weakly, are projected out; p_floor_rel = 0 keeps every P > 0).
 *
 * Layouts (all contiguous, row-major):
 *   x : [batch, N] real (float for QTAM_FP32 plans, double for QTAM_FP64)
 *   y : [batch, R, N_out] interleaved complex (float2 / double2)
 *
 * Ownership: the caller owns x, y and the workspace (device memory). A plan
 * owns its host tables and, unless created host-only, device copies of them
 * on the device that was current at creation; it is immutable after creation.
 *
 * Concurrency and errors: transform calls only enqueue work on the given HIP
 * stream and never synchronise. Concurrent calls on one plan are legal when
 * they use distinct workspaces. Arguments are validated before any launch;
 * failures return a status and enqueue nothing. Launch failures are reported
 * as QTAM_ERR_DEVICE.
 */
#ifndef QTAM_H
#define QTAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qtam_plan_s* qtam_plan_t;   /* opaque, immutable after create */
typedef void* qtam_stream_t;               /* a hipStream_t; NULL = default stream */

typedef enum {
  QTAM_OK = 0,
  QTAM_ERR_INVALID_ARG = 1,   /* bad parameter, NULL pointer, or n_out < max L_k */
  QTAM_ERR_UNSUPPORTED = 2,   /* valid but not implemented on the GPU (e.g. size) */
  QTAM_ERR_WORKSPACE = 3,     /* workspace smaller than one segment needs */
  QTAM_ERR_OOM = 4,           /* plan tables: device or host allocation failed */
  QTAM_ERR_DEVICE = 5         /* HIP runtime / launch error, or no device */
} qtam_status;

typedef enum { QTAM_FP32 = 0, QTAM_FP64 = 1 } qtam_precision;

/* Cap on window length L_k (App. A, max_window_size). g = ceil(T * df_max),
 * df_max the largest gap between consecutive row frequencies.
 *   COVER : L_max = 2g + 1 (each clamped window reaches its neighbours'
 *           centres; no frame holes) - default
 *   PAPER : L_max = 2 floor(g/2) + 1 (the printed formula)
 *   NONE  : no cap (pure constant-Q)
 *   MANUAL: L_max = params.max_window bins                                  */
typedef enum { QTAM_CAP_COVER = 0, QTAM_CAP_PAPER = 1, QTAM_CAP_NONE = 2, QTAM_CAP_MANUAL = 3 } qtam_cap_mode;

/* Window normalisation (Sec. II): unit energy per tile (default), the printed
 * constant 1/sum W'^2, or none.                                              */
typedef enum { QTAM_NORM_UNIT_ENERGY = 0, QTAM_NORM_PAPER_INV_ENERGY = 1, QTAM_NORM_NONE = 2 } qtam_norm_mode;

/* Window shapes on x = j/h_k in [-1, 1] (Sec. II; App. A). window_param is
 * Kaiser beta, Tukey alpha or Planck-taper alpha.                           */
typedef enum { QTAM_WIN_BISQUARE = 0, QTAM_WIN_HANN = 1, QTAM_WIN_KAISER = 2,
               QTAM_WIN_TUKEY = 3, QTAM_WIN_PLANCK = 4 } qtam_window;

enum { QTAM_PLAN_HOST_ONLY = 1 };   /* qtam_params.flags: build tables, no device upload */

typedef struct {
  double sample_rate;       /* fs in Hz, > 0                                      */
  int64_t n_samples;        /* N, even, >= 16                                     */
  double q;                 /* quality factor Q = f / df, > 0                     */
  double f_min, f_max;      /* 0 < f_min <= f_max <= fs/2 (grid ends, inclusive)  */
  int32_t n_rows;           /* R >= 1; with freqs != NULL the list length         */
  const double* freqs;      /* optional explicit non-decreasing centre list (App. A); copied */
  int32_t window;           /* qtam_window                                        */
  double window_param;
  int32_t cap_mode;         /* qtam_cap_mode                                      */
  int32_t max_window;       /* bins, QTAM_CAP_MANUAL only                         */
  int32_t norm_mode;        /* qtam_norm_mode                                     */
  int32_t n_out;            /* 0: next power of two >= max L_k; else >= max L_k   */
  double p_floor_rel;       /* mask threshold relative to max P; default 1e-6     */
  int32_t precision;        /* qtam_precision                                     */
  int32_t flags;            /* QTAM_PLAN_HOST_ONLY or 0                           */
  /* Composite bank (App. A, multi-Q / multi-window extension). n_planes = 0:
   * one plane (q, window, window_param). n_planes >= 1: plane p uses
   * plane_q[p], plane_window[p], plane_window_param[p] (host arrays, copied)
   * and q / window / window_param are ignored. Every plane has the same
   * n_rows-row frequency grid; the plan has n_planes * n_rows rows, plane
   * after plane (row p * n_rows + k), and one frame P summed over all rows,
   * so the inverse reconstructs from the whole bank.                        */
  int32_t n_planes;
  const double* plane_q;
  const int32_t* plane_window;
  const double* plane_window_param;
  /* Regularised stop band (Sec. III; App. A): > 0 is a floor on every
   * window (before normalisation): each bin of 0..N/2 where its shape is
   * below this value (the stop band, the support's end points, a taper's
   * tails) takes this value, so each row keeps the whole band (max L_k =
   * N/2 + 1) and a single tile determines the signal (qtam_tile_inverse)
   * with rounding amplified by at most about 1/window_eps. 0: plain windows. */
  double window_eps;
} qtam_params;

typedef struct {
  int32_t n_rows;           /* R = n_planes * rows_per_plane                      */
  int32_t n_planes;         /* 1 for a plain plan                                 */
  int32_t rows_per_plane;
  int32_t n_out;            /* N_out                                              */
  int32_t max_len;          /* max_k L_k = 2 h_k + 1                              */
  int32_t precision;
  int64_t n_samples;        /* N                                                  */
  int64_t n_bins;           /* N/2 + 1                                            */
  int64_t sum_len;          /* sum_k of kept support lengths (packed table size)  */
  int64_t l_max;            /* cap, -1 if none                                    */
  double frame_A, frame_B;  /* min / max of P over the mask M                     */
  double masked_fraction;   /* fraction of bins 0..N/2 outside M                  */
  size_t workspace_bytes_per_segment;   /* max over forward / inverse / adjoints   */
  const double* freqs;      /* [R] nominal centre frequencies (Hz)                */
  const double* row_q;      /* [R] quality factor of each row's plane             */
  const int32_t* centre;    /* [R] centre bins s_k                                */
  const int32_t* half_width;/* [R] h_k                                            */
  const int32_t* lo;        /* [R] first kept bin                                 */
  const int32_t* hi;        /* [R] last kept bin                                  */
  const int64_t* offset;    /* [R] start of row k in the packed tables            */
  const double* window;     /* [sum_len] W_k on its kept bins, row after row      */
  const double* frame;      /* [N/2+1] P                                          */
  const uint8_t* mask;      /* [N/2+1] M                                          */
} qtam_plan_info_t;

/* Build the plan (host FP64 tables, App. A and C) and, unless
 * QTAM_PLAN_HOST_ONLY, upload the device tables of the requested precision to
 * the current HIP device. On failure *out is NULL.                           */
qtam_status qtam_plan_create(const qtam_params* params, qtam_plan_t* out);

/* Host pointers in *info stay valid until qtam_plan_destroy.                 */
qtam_status qtam_plan_info(qtam_plan_t plan, qtam_plan_info_t* info);

/* Frees host and device tables. Safe on NULL. The caller must make sure no
 * enqueued work still uses the plan.                                        */
void qtam_plan_destroy(qtam_plan_t plan);

/* Workspace one call needs for `batch` segments (bytes). A smaller workspace
 * that still holds one segment is accepted: the batch is then processed in
 * chunks that fit.                                                           */
size_t qtam_workspace_size(qtam_plan_t plan, int64_t batch);

/* Forward transform (Sec. III; App. A): x [batch, N] real -> y [batch, R, N_out]
 * complex. Device pointers; ws is device scratch of ws_bytes.               */
qtam_status qtam_forward(qtam_plan_t plan, const void* x, void* y, int64_t batch,
                         void* ws, size_t ws_bytes, qtam_stream_t stream);

/* Forward transform that allocates nothing, for callers that cannot call
 * hipMalloc: code under stream capture, tight serving loops, harnesses that
 * forbid allocation. Same arguments and results as qtam_forward without a
 * workspace: the library uses a static device array of
 * QTAM_NOALLOC_WORKSPACE_BYTES that every device it runs on holds until the
 * process ends (its address is looked up once per device at plan creation).
 * The batch is processed in chunks that fit that array; a plan one segment
 * of which needs more (qtam_workspace_size(plan, 1) above the size) returns
 * QTAM_ERR_WORKSPACE, with the sizes in qtam_last_error. Every call on one
 * device shares the array and every region of it is written before it is
 * read (nothing is cleared): calls that overlap on one device (different
 * streams, or several host threads) race; serialize them, for example on one
 * stream. Launches of this call are not timed by qtam_timing_enable.        */
#define QTAM_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
qtam_status qtam_forward_noalloc(qtam_plan_t plan, const void* x, void* y, int64_t batch,
                                 qtam_stream_t stream);

/* Inverse transform by the canonical dual frame (Sec. III; App. C):
 * y [batch, R, N_out] complex -> x [batch, N] real. Any y is accepted; the
 * result is the minimum-norm (canonical dual) synthesis restricted to M.    */
qtam_status qtam_inverse(qtam_plan_t plan, const void* y, void* x, int64_t batch,
                         void* ws, size_t ws_bytes, qtam_stream_t stream);

/* Adjoint of qtam_forward as a real-linear map (the gradient of a real loss,
 * App. C: the adjoint of analysis is synthesis): gy [batch, R, N_out] complex
 * (d loss/d Re y + i d loss/d Im y) -> gx [batch, N] real.                  */
qtam_status qtam_forward_adjoint(qtam_plan_t plan, const void* gy, void* gx, int64_t batch,
                                 void* ws, size_t ws_bytes, qtam_stream_t stream);

/* Adjoint of qtam_inverse as a real-linear map: gx [batch, N] real ->
 * gy [batch, R, N_out] complex.                                              */
qtam_status qtam_inverse_adjoint(qtam_plan_t plan, const void* gx, void* gy, int64_t batch,
                                 void* ws, size_t ws_bytes, qtam_stream_t stream);

/* The signal from the single row `row` of each segment by spectral division
 * (Sec. III, regularised windows): X[c] = sqrt(N/N_out) DFT_{N_out}(Y_row)
 * [(c - s_row) mod N_out] / W_row[c] on every bin, then the inverse real FFT.
 * y [batch, R, N_out] -> x [batch, N]. Needs window_eps > 0
 * (QTAM_ERR_INVALID_ARG otherwise) and a power-of-two N_out (chirp-z
 * lengths: QTAM_ERR_UNSUPPORTED); workspace as qtam_inverse.               */
qtam_status qtam_tile_inverse(qtam_plan_t plan, const void* y, int32_t row, void* x, int64_t batch,
                              void* ws, size_t ws_bytes, qtam_stream_t stream);

/* Dense full-rate tiles (App. C): dense [batch, R, N] complex (device),
 *   T_k[tau] = (1/N) sum_b X[b] W_k[b] e^{+2 pi i b tau / N},  tau = 0..N-1,
 * from the envelopes y [batch, R, N_out] (each row re-modulated to its
 * carrier and band-limited up-sampled to N samples; this is the dense row the
 * forward transform decimates). Needs N = r * 2^k with r in {1, 3, 5}, as
 * the plan's spectrum does (the paper's 6 s x 4096 Hz segment is 3 * 8192),
 * else QTAM_ERR_UNSUPPORTED, and the workspace qtam_dense_workspace_size gives
 * (0 when the plan has no dense path); one segment's tiles must stay below
 * 2 GiB. Smaller workspaces that hold one segment are used in chunks.       */
size_t qtam_dense_workspace_size(qtam_plan_t plan, int64_t batch);
qtam_status qtam_dense(qtam_plan_t plan, const void* y, void* dense, int64_t batch,
                       void* ws, size_t ws_bytes, qtam_stream_t stream);

/* Gain x soft-threshold mask on envelope coefficients, the denoising model
 * of a differentiable pipeline (masking complex coefficients before the
 * inverse, Sec. V; the transform inside a differentiable denoiser, App. A):
 *   out[b,k,m] = gain[k] * max(0, 1 - lambda[k] / |y[b,k,m]|) * y[b,k,m],
 * |y| floored at the smallest normal number. y, out [batch, R, N_out]
 * complex and gain, lambda [R] real, in the plan's precision, on the plan's
 * device; out may alias y. Elementwise, one launch per 65535/R segments.
 * batch = 0 does nothing (y and out may then be NULL).                      */
qtam_status qtam_mask_forward(qtam_plan_t plan, const void* y, const void* gain, const void* lambda, void* out,
                              int64_t batch, qtam_stream_t stream);

/* Its gradients: with gout = dL/dout as dL/dRe + i dL/dIm and
 * p = Re(conj(y) gout),
 *   gy = gain[k] * (m gout + [m > 0, lambda[k] > 0] (lambda/|y|)(p/|y|^2) * y),
 *   dgain[k] = sum over b and m of m p (each row by a fixed tree, then the
 *              segments by fixed lane strides and a fixed butterfly:
 *              identical bits run to run).
 * gy [batch, R, N_out] complex, dgain [R] real; ws holds the rows' partial
 * sums: at least qtam_mask_workspace_size(plan, batch) bytes
 * (QTAM_ERR_WORKSPACE otherwise). batch = 0 sets dgain to 0; y, gout, gy
 * and ws may then be NULL. NULL gain, lambda or dgain: QTAM_ERR_INVALID_ARG. */
size_t qtam_mask_workspace_size(qtam_plan_t plan, int64_t batch);
qtam_status qtam_mask_backward(qtam_plan_t plan, const void* y, const void* gain, const void* lambda,
                               const void* gout, void* gy, void* dgain, int64_t batch, void* ws,
                               size_t ws_bytes, qtam_stream_t stream);

/* The mask fused into the inverse: x = qtam_inverse(mask(y)) with mask as in
 * qtam_mask_forward, applied to each envelope value as the inverse rows
 * kernel loads it (the masked envelopes are never written). Same layouts,
 * workspace and results as qtam_mask_forward followed by qtam_inverse.
 * Rows transformed in one workgroup only (power-of-two N_out up to 32768
 * FP32 / 8192 FP64): other plans return QTAM_ERR_UNSUPPORTED before any
 * launch, also for batch = 0, which otherwise does nothing (a query: NULL
 * pointers are then accepted).                                              */
qtam_status qtam_inverse_masked(qtam_plan_t plan, const void* y, const void* gain, const void* lambda,
                                void* x, int64_t batch, void* ws, size_t ws_bytes, qtam_stream_t stream);

/* Its adjoint, the backward pass of the denoiser's mask and inverse: with gx
 * = dL/dx [batch, N], gy = dL/dy [batch, R, N_out] and dgain [R] as from
 * qtam_inverse_adjoint (giving dL/d mask(y)) followed by qtam_mask_backward,
 * the mask's gradient applied in the rows kernel's epilogue (dL/d mask(y)
 * is never written). y is the unmasked input of qtam_inverse_masked. ws: at
 * least qtam_masked_adjoint_workspace_size(plan, batch) bytes (its first
 * part holds the gain gradient's per-row partial sums; with less, the
 * transform runs in chunks down to one segment, below that
 * QTAM_ERR_WORKSPACE). dgain sums fixed trees per row and fixed lane strides
 * over the segments: identical bits run to run. batch = 0 sets dgain to 0.
 * Plans as for qtam_inverse_masked.                                          */
size_t qtam_masked_adjoint_workspace_size(qtam_plan_t plan, int64_t batch);
qtam_status qtam_inverse_masked_adjoint(qtam_plan_t plan, const void* gx, const void* y, const void* gain,
                                        const void* lambda, void* gy, void* dgain, int64_t batch, void* ws,
                                        size_t ws_bytes, qtam_stream_t stream);

/* Forward transform of one batch under several plans at once (the multi-Q
 * extension of App. A, where every configuration of the bank works from the
 * same spectrum): the real spectrum of each segment is computed once and
 * every plan's rows are taken from it. plans[0 .. n_plans-1] must share N
 * and the precision (else QTAM_ERR_INVALID_ARG) and may differ in anything
 * else (Q, rows, band, window, N_out). x [batch, N] real; y[i] is plan i's
 * output [batch, R_i, N_out_i] complex, exactly as qtam_forward(plans[i], ...)
 * writes it (the same kernels on the same spectrum: identical bits). ws must
 * hold qtam_workspace_size of every plan for one segment at least; with less
 * than the largest of them for the whole batch, the batch runs in chunks. All
 * pointers are device pointers except plans and y, which are host arrays of
 * n_plans entries. Work is enqueued on `stream`; errors as qtam_forward.     */
qtam_status qtam_forward_sweep(const qtam_plan_t* plans, int32_t n_plans, const void* x, void* const* y,
                               int64_t batch, void* ws, size_t ws_bytes, qtam_stream_t stream);

/* Plane metrics (the per-plane quality metric of the multi-Q extension,
 * App. A): which statistic of a plane scores it.                           */
typedef enum { QTAM_METRIC_ENERGY = 0,   /* sum over the plane's rows and m of |Y|^2 */
               QTAM_METRIC_PEAK = 1      /* max over the plane's rows and m of |Y|^2 */
} qtam_metric;

/* qtam_forward that also returns row statistics: metric [batch, R] complex
 * (float2 / double2, device) with metric[b, k] = (sum_m |Y_k[m]|^2,
 * max_m |Y_k[m]|^2) of segment b. The statistics come from the coefficients
 * while they are still on chip; y is written exactly as qtam_forward writes it. */
qtam_status qtam_forward_metric(qtam_plan_t plan, const void* x, void* y, void* metric, int64_t batch,
                                void* ws, size_t ws_bytes, qtam_stream_t stream);

/* Optimal-plane selection, independently for each segment (multi-Q
 * extension, App. A): score[b, p] is the energy (sum over the plane's rows of
 * metric.x) or peak (max of metric.y) of plane p; best[b] is the first plane
 * with the largest score; y_best[b] = y[b, best[b]*rows_per_plane ... +
 * rows_per_plane - 1], a [batch, rows_per_plane, N_out] complex copy.
 * y and metric as written by qtam_forward_metric; score (may be NULL) is
 * [batch, n_planes] real in the plan precision, best [batch] int32; all device;
 * y and y_best 16-byte aligned. A NaN score never wins.                     */
qtam_status qtam_select_planes(qtam_plan_t plan, const void* y, const void* metric, int32_t kind,
                               void* score, int32_t* best, void* y_best, int64_t batch,
                               qtam_stream_t stream);

/* Per-kernel timing with HIP events recorded on the call's own stream around
 * each launch. While enabled, every launch is bracketed by two events and the
 * durations are accumulated per kernel kind when qtam_timing_collect is
 * called (which synchronises on those events).                              */
qtam_status qtam_timing_enable(qtam_plan_t plan, int32_t on);
/* Fills up to max_kinds entries: names[i] (static strings), total_ms[i] and
 * launches[i]; returns the number of kinds in *n_kinds and resets the totals. */
qtam_status qtam_timing_collect(qtam_plan_t plan, const char** names, double* total_ms,
                                int64_t* launches, int32_t max_kinds, int32_t* n_kinds);

const char* qtam_status_string(qtam_status status);

/* Text of the last failure behind a QTAM_ERR_DEVICE or QTAM_ERR_OOM (and the
 * sizes behind qtam_forward_noalloc's QTAM_ERR_WORKSPACE) returned on the
 * calling thread: call name, HIP error name and message, or the host
 * allocation that failed; empty if none. Valid until the next call on this
 * thread.                                                                   */
const char* qtam_last_error(void);

/* Library version string, e.g. "qtam-gfx950 1.0".                           */
const char* qtam_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QTAM_H */
