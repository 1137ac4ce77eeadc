// Device-side row metadata, twiddle tables and launch geometry shared by the
// QTAM kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_engine.hpp"

namespace qtam {

// ---------------------------------------------------------------------------
// Device-side tables
// ---------------------------------------------------------------------------
struct RowMeta {
  int s, lo, hi, off;   // centre bin, kept bin range, offset in the packed tables
};

// exp(-2 pi i m / N) for m in [0, N) as fine[m & (F-1)] * coarse[m >> log2 F]
template <typename C>
struct Twiddle2 {
  const C* fine;
  const C* coarse;
  int bits;
  __device__ __forceinline__ C operator()(int64_t m) const {
    const int64_t lo = m & ((int64_t(1) << bits) - 1);
    return c_mul(fine[lo], coarse[m >> bits]);
  }
};

// ---------------------------------------------------------------------------
// Launch geometry
// ---------------------------------------------------------------------------
template <typename T> constexpr int elems_per_thread() { return sizeof(T) == 4 ? 16 : 8; }

template <typename T, int L>
struct RowGeom {
  static constexpr int E0 = L < elems_per_thread<T>() ? L : elems_per_thread<T>();
  static constexpr int E = L / E0 > 1024 ? L / 1024 : E0;   // at most 1024 threads per transform
  static constexpr int TPR = L / E;
  static constexpr int G = TPR >= 256 ? 1 : 256 / TPR;   // transforms per workgroup
  static constexpr int NT = G * TPR;
};

// Columns per workgroup of the four-step passes: C * L values fill at most
// 64 KiB of LDS, at least 4 columns for 32/64-byte contiguous runs.
// EP > 0 sets the values per thread (the second four-step pass of the
// spectrum and synthesis transforms runs faster with 8 in FP32: twice the
// waves per workgroup for its LDS-staged rows).
template <typename T, int L, int EP = 0>
struct ColGeom {
  static constexpr int E0 = EP > 0 ? EP : elems_per_thread<T>();
  static constexpr int E = L < E0 ? L : E0;
  static constexpr int TPR = L / E;
  static constexpr int CAP = (65536 / (2 * int(sizeof(T)))) / L;
  static constexpr int CC = CAP >= 16 ? 16 : (CAP >= 4 ? CAP : 4);
  static constexpr int NT = CC * TPR;
};

}  // namespace qtam
