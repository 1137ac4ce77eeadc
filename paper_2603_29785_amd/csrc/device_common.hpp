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

// Envelope slot u of a row holds the kept bin c with (c - s) mod L = u (the
// roll of bin s to slot 0, Sec. III / App. A). The support holds at most L
// bins, so that bin is unique when it exists: c = lo + d with
// d = (u + s - lo) mod L, kept iff d <= hi - lo. Slot entries of a
// power-of-two L:
template <int L>
__device__ __forceinline__ int slot_entry(int u, const RowMeta& rm) {
  static_assert((L & (L - 1)) == 0, "power-of-two rows");
  return (u + rm.s - rm.lo) & (L - 1);
}

// A row is centred when its support lies inside s - L/2 .. s + L/2 - 1: the
// signed slot offset j (u, or u - L above L/2) then gives c = s + j directly.
// Every row whose window is narrower than the band is centred (its support
// is within s - h .. s + h and 2h + 1 <= L); a row of a regularised window
// keeps the whole band 0..N/2 and may not be.
__device__ __forceinline__ bool row_centred(const RowMeta& rm, int L) {
  return rm.lo >= rm.s - L / 2 && rm.hi < rm.s + L / 2;
}

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
template <typename T, int L, int EP = 0, int CW = 0>
struct ColGeom {
  static constexpr int E0 = EP > 0 ? EP : elems_per_thread<T>();
  static constexpr int E = L < E0 ? L : E0;
  static constexpr int TPR = L / E;
  static constexpr int CAP = (65536 / (2 * int(sizeof(T)))) / L;
  // CW > 0 asks for CW columns where their LDS (with its padding) fits in
  // 144 KiB and CW * TPR threads make one workgroup
  static constexpr bool WIDE = CW > 0 && CW * (L + L / 32) * 2 * int(sizeof(T)) <= 147456 && CW * TPR <= 1024;
  static constexpr int CC = WIDE ? CW : (CAP >= 16 ? 16 : (CAP >= 4 ? CAP : 4));
  static constexpr int NT = CC * TPR;
};

}  // namespace qtam
