// Overlap-add of the packed row spectra with the real-signal pre-twist
// (Sec. III canonical dual; App. C), row statistics and plane selection of the
// multi-Q extension (App. A).
#pragma once

#include "device_common.hpp"

namespace qtam {

// Overlap-add. Each wave owns 64 consecutive bins p <= N/4 and their mirrors
// q = N/2 - p. For each side it walks the rows whose kept support meets its
// bins (a host list per wave, ascending row order, so every bin sums its
// terms in ascending row order, with no atomics): lanes inside a row's support
// add that row's packed entry, consecutive lanes reading consecutive entries;
// lanes outside get an offset beyond the buffer and read 0. Then the
// real-signal pre-twist turns the one-sided spectrum at p and N/2-p into the
// half-size spectrum the synthesis FFT consumes.
struct OlaRow {
  int lo, span, base, pad;   // kept bins [lo, lo + span], packed entry of bin c at base + c
};

template <typename C>
__device__ __forceinline__ C ola_side(rsrc_t rs, const OlaRow* __restrict__ list, int a, int b, int c) {
  C acc{0, 0};
#pragma unroll 4
  for (int i = a; i < b; ++i) {
    const OlaRow r = list[i];
    const bool in = static_cast<unsigned>(c - r.lo) <= static_cast<unsigned>(r.span);
    const unsigned vo = in ? static_cast<unsigned>(r.base + c) * static_cast<unsigned>(sizeof(C)) : 0xFFFFFFFFu;
    acc = c_add(acc, bload<C>(rs, vo));
  }
  return acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_ola(
    const typename Complex<T>::type* __restrict__ Sbuf, typename Complex<T>::type* __restrict__ Zout,
    const int* __restrict__ wave_start, const OlaRow* __restrict__ wave_rows, int64_t half, int64_t sum_len,
    int nwaves, Twiddle2<typename Complex<T>::type> tw2) {
  using C = typename Complex<T>::type;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x) * 4 + static_cast<int>(threadIdx.x >> 6));
  if (wave >= nwaves) return;
  const int64_t seg = blockIdx.y;
  const int p = wave * 64 + static_cast<int>(threadIdx.x & 63);
  const int q = static_cast<int>(half) - p;
  const rsrc_t rs = make_rsrc(Sbuf + seg * sum_len, static_cast<uint32_t>(sum_len * sizeof(C)));
  const int a0 = __builtin_amdgcn_readfirstlane(wave_start[2 * wave]);
  const int a1 = __builtin_amdgcn_readfirstlane(wave_start[2 * wave + 1]);
  const int a2 = __builtin_amdgcn_readfirstlane(wave_start[2 * wave + 2]);
  C A = ola_side<C>(rs, wave_rows, a0, a1, p);
  C B = ola_side<C>(rs, wave_rows, a1, a2, q);
  if (p > half / 2) return;
  if (p == 0) {   // DC and Nyquist: real parts only (irfft convention)
    A.y = 0;
    B.y = 0;
  }
  const C w = c_conj(tw2(p));   // exp(+2 pi i p / N)
  const C Bc = c_conj(B), Ac = c_conj(A);
  C* Zs = Zout + seg * half;
  Zs[p] = c_add(c_add(A, Bc), c_mul_si<+1>(c_mul(w, c_sub(A, Bc))));
  if (p > 0 && q != p) Zs[q] = c_add(c_add(B, Ac), c_mul_si<-1>(c_mul(c_conj(w), c_sub(B, Ac))));
}

// Row statistics read back from Y (rows too long for one workgroup): one
// workgroup per row, fixed-order partial sums and a fixed tree.
template <typename T>
__global__ __launch_bounds__(256) void k_row_stats(const typename Complex<T>::type* __restrict__ Y,
                                                   typename Complex<T>::type* __restrict__ stats, int64_t n_out) {
  using C = typename Complex<T>::type;
  __shared__ T se[256], sm[256];
  const C* row = Y + int64_t(blockIdx.x) * n_out;
  T e = 0, m = 0;
  for (int64_t i = threadIdx.x; i < n_out; i += 256) {
    const C v = row[i];
    const T a = v.x * v.x + v.y * v.y;
    e += a;
    m = fmax(m, a);
  }
  se[threadIdx.x] = e;
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) {
      se[threadIdx.x] += se[threadIdx.x + w];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) stats[blockIdx.x] = C{se[0], sm[0]};
}

// Plane scores and the best plane of each segment (one workgroup per
// segment): energy sums a plane's row energies, peak takes their maximum; the
// first plane with the largest score wins and a NaN score never does.
template <typename T>
__global__ __launch_bounds__(256) void k_plane_best(const typename Complex<T>::type* __restrict__ stats,
                                                    int rows_per_plane, int planes, int peak,
                                                    T* __restrict__ score, int* __restrict__ best) {
  using C = typename Complex<T>::type;
  __shared__ T red[256];
  const int64_t seg = blockIdx.x;
  const C* st = stats + seg * int64_t(rows_per_plane) * planes;
  T top = 0;
  int arg = -1;
  for (int p = 0; p < planes; ++p) {
    T a = 0;
    for (int k = threadIdx.x; k < rows_per_plane; k += 256) {
      const C v = st[int64_t(p) * rows_per_plane + k];
      a = peak ? fmax(a, v.y) : a + v.x;
    }
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (int(threadIdx.x) < w)
        red[threadIdx.x] = peak ? fmax(red[threadIdx.x], red[threadIdx.x + w]) : red[threadIdx.x] + red[threadIdx.x + w];
      __syncthreads();
    }
    const T sc = red[0];
    __syncthreads();
    if (threadIdx.x == 0) {
      if (score != nullptr) score[seg * planes + p] = sc;
      if (sc == sc && (arg < 0 || sc > top)) {
        top = sc;
        arg = p;
      }
    }
  }
  if (threadIdx.x == 0) best[seg] = arg < 0 ? 0 : arg;
}

// y_best[seg] = plane best[seg] of y[seg], copied in 16-byte units.
__global__ __launch_bounds__(256) void k_gather_plane(const uint4* __restrict__ y, const int* __restrict__ best,
                                                      uint4* __restrict__ out, int64_t plane_units, int planes) {
  const int64_t seg = blockIdx.y;
  const int b = best[seg];
  const uint4* src = y + (seg * planes + b) * plane_units;
  uint4* dst = out + seg * plane_units;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < plane_units; i += int64_t(gridDim.x) * 256)
    dst[i] = src[i];
}

}  // namespace qtam
