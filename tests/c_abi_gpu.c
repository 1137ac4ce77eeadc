/* A C caller of libqtam.so on the GPU, through the HIP runtime only (no
 * Python, no torch): reads `batch` segments of N float64 samples from a file,
 * runs qtam_forward and qtam_inverse on the current device in the requested
 * precision, and writes the envelopes (interleaved complex, float64) and the
 * reconstructions (float64). tests/test_gpu_c_caller.py builds it, runs it
 * and compares the outputs with the oracle.
 *   c_abi_gpu fs N Q f_min f_max R fp32|fp64 batch in.bin y.bin x.bin */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "qtam.h"

#define HIP_OK(call)                                                            \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));          \
      return 3;                                                                 \
    }                                                                           \
  } while (0)
#define QTAM_OK_(call)                                                          \
  do {                                                                          \
    qtam_status s_ = (call);                                                    \
    if (s_ != QTAM_OK) {                                                        \
      fprintf(stderr, "%s: %s (%s)\n", #call, qtam_status_string(s_), qtam_last_error()); \
      return 4;                                                                 \
    }                                                                           \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 12) {
    fprintf(stderr, "usage: c_abi_gpu fs N Q f_min f_max R fp32|fp64 batch in.bin y.bin x.bin\n");
    return 2;
  }
  qtam_params p;
  memset(&p, 0, sizeof p);
  p.sample_rate = atof(argv[1]);
  p.n_samples = atoll(argv[2]);
  p.q = atof(argv[3]);
  p.f_min = atof(argv[4]);
  p.f_max = atof(argv[5]);
  p.n_rows = atoi(argv[6]);
  p.precision = strcmp(argv[7], "fp64") == 0 ? QTAM_FP64 : QTAM_FP32;
  p.p_floor_rel = 1e-6;
  const int64_t batch = atoll(argv[8]);
  const int f64 = p.precision == QTAM_FP64;
  const size_t rb = f64 ? 8 : 4;

  qtam_plan_t plan = NULL;
  QTAM_OK_(qtam_plan_create(&p, &plan));
  qtam_plan_info_t info;
  QTAM_OK_(qtam_plan_info(plan, &info));
  const int64_t n = p.n_samples, ny = (int64_t)info.n_rows * info.n_out;

  /* input: float64 on disk, the plan's precision on the device */
  double* xh = malloc((size_t)(batch * n) * sizeof(double));
  FILE* f = fopen(argv[9], "rb");
  if (!f || fread(xh, sizeof(double), (size_t)(batch * n), f) != (size_t)(batch * n)) return 5;
  fclose(f);
  void* xs = malloc((size_t)(batch * n) * rb);
  for (int64_t i = 0; i < batch * n; ++i) {
    if (f64) ((double*)xs)[i] = xh[i];
    else ((float*)xs)[i] = (float)xh[i];
  }

  void *xd, *yd, *xr, *ws;
  const size_t wsb = qtam_workspace_size(plan, batch);
  HIP_OK(hipMalloc(&xd, (size_t)(batch * n) * rb));
  HIP_OK(hipMalloc(&xr, (size_t)(batch * n) * rb));
  HIP_OK(hipMalloc(&yd, (size_t)(batch * ny) * 2 * rb));
  HIP_OK(hipMalloc(&ws, wsb));
  hipStream_t st;
  HIP_OK(hipStreamCreate(&st));
  HIP_OK(hipMemcpy(xd, xs, (size_t)(batch * n) * rb, hipMemcpyHostToDevice));
  QTAM_OK_(qtam_forward(plan, xd, yd, batch, ws, wsb, st));
  QTAM_OK_(qtam_inverse(plan, yd, xr, batch, ws, wsb, st));
  HIP_OK(hipStreamSynchronize(st));

  void* yh = malloc((size_t)(batch * ny) * 2 * rb);
  HIP_OK(hipMemcpy(yh, yd, (size_t)(batch * ny) * 2 * rb, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(xs, xr, (size_t)(batch * n) * rb, hipMemcpyDeviceToHost));
  double* y64 = malloc((size_t)(batch * ny) * 2 * sizeof(double));
  for (int64_t i = 0; i < 2 * batch * ny; ++i) y64[i] = f64 ? ((double*)yh)[i] : (double)((float*)yh)[i];
  for (int64_t i = 0; i < batch * n; ++i) xh[i] = f64 ? ((double*)xs)[i] : (double)((float*)xs)[i];
  f = fopen(argv[10], "wb");
  if (!f || fwrite(y64, sizeof(double), (size_t)(2 * batch * ny), f) != (size_t)(2 * batch * ny)) return 6;
  fclose(f);
  f = fopen(argv[11], "wb");
  if (!f || fwrite(xh, sizeof(double), (size_t)(batch * n), f) != (size_t)(batch * n)) return 6;
  fclose(f);

  HIP_OK(hipStreamDestroy(st));
  HIP_OK(hipFree(xd));
  HIP_OK(hipFree(xr));
  HIP_OK(hipFree(yd));
  HIP_OK(hipFree(ws));
  qtam_plan_destroy(plan);
  free(xh);
  free(xs);
  free(yh);
  free(y64);
  printf("done: %lld segments, R %d, N_out %d\n", (long long)batch, info.n_rows, info.n_out);
  return 0;
}
