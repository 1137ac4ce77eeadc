// Spectrum and synthesis kernels: the N/2-point complex transforms of the
// packed real signal (one pass, or the two passes of the four-step
// factorisation N/2 = N1 * N2), the real-signal twist, and the decimation by
// 3 or 5 around power-of-two transforms (App. A RFFT; App. C DFT convention).
#pragma once

#include "device_common.hpp"

namespace qtam {

// Batched contiguous complex FFTs of length L: transform t reads
// in[t*stride + n] and writes out[t*stride + k]. A chunk holds count
// transforms; every buffer of it is below 2 GiB.
template <typename T, int L, int S>
__global__ __launch_bounds__((RowGeom<T, L>::NT)) void k_fft_rows(
    const typename Complex<T>::type* __restrict__ in, typename Complex<T>::type* __restrict__ out,
    int64_t count, int64_t stride, const typename Complex<T>::type* __restrict__ tw) {
  using C = typename Complex<T>::type;
  using Geo = RowGeom<T, L>;
  using F = BlockFft<T, L, Geo::E, S>;
  __shared__ C lds[Geo::G * lds_size(L)];
  const int t = threadIdx.x, g = t / Geo::TPR, tl = t % Geo::TPR;
  const int64_t tr0 = int64_t(blockIdx.x) * Geo::G;
  const int64_t nt = count - tr0 < Geo::G ? count - tr0 : Geo::G;   // transforms of this block
  const uint32_t bytes = static_cast<uint32_t>((nt - 1) * stride + L) * sizeof(C);
  // lanes of transforms past the end fall outside [0, bytes): loads give 0
  const rsrc_t rin = make_rsrc(in + tr0 * stride, bytes);
  const rsrc_t rout = make_rsrc(out + tr0 * stride, bytes);
  const uint32_t vb = static_cast<uint32_t>(g * stride + tl) * sizeof(C);
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = bload<C>(rin, vb, F::in_off(i) * sizeof(C));
  F::run(v, lds + g * lds_size(L), tl, F::twiddles(tw));
  if (g < nt) {
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) bstore<C>(rout, v[i], vb, F::out_off(i) * sizeof(C));
  }
}

// Four-step, first pass: length-N2 FFTs down the columns n1 of the N1 x N2
// view (element stride N1), times exp(S 2 pi i n1 k2 / M), written back in
// place-order. CC adjacent columns per workgroup, column index fastest
// across threads so every access is a contiguous run of CC values.
template <typename T, int L, int S, int CW = 0>
__global__ __launch_bounds__((ColGeom<T, L, 0, CW>::NT)) void k_fft_cols(
    const typename Complex<T>::type* __restrict__ in, typename Complex<T>::type* __restrict__ out,
    int64_t n1_count, int64_t seg_stride, const typename Complex<T>::type* __restrict__ tw,
    Twiddle2<typename Complex<T>::type> tw2, int tw_mul) {
  using C = typename Complex<T>::type;
  using Geo = ColGeom<T, L, 0, CW>;
  using F = BlockFft<T, L, Geo::E, S>;
  __shared__ C lds[Geo::CC * lds_size(L)];
  const int t = threadIdx.x, c = t % Geo::CC, tl = t / Geo::CC;
  const int64_t n1 = int64_t(blockIdx.x) * Geo::CC + c;
  const int64_t base = int64_t(blockIdx.y) * seg_stride + n1;
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = in[base + n1_count * F::in_index(tl, i)];
  F::run(v, lds + c * lds_size(L), tl, F::twiddles(tw));
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int64_t k2 = F::out_index(tl, i);
    // exp(-2 pi i n1 k2 / M), M = N1 N2, from the table of exp(-2 pi i m / (tw_mul M))
    C w = tw2(tw_mul * n1 * k2);
    if constexpr (S > 0) w.y = -w.y;
    out[base + n1_count * k2] = c_mul(v[i], w);
  }
}

// Four-step, second pass: length-N1 FFTs along the contiguous rows k2 of the
// intermediate; CC rows per workgroup are staged through LDS with a linear
// (coalesced) load, results go to Z[k2 + N2 k1] in runs of CC values.
template <typename T, int L, int S, int EP = 0, int CW = 0>
__global__ __launch_bounds__((ColGeom<T, L, EP, CW>::NT)) void k_fft_rows_t(
    const typename Complex<T>::type* __restrict__ in, typename Complex<T>::type* __restrict__ out,
    int64_t n2_count, int64_t seg_stride, const typename Complex<T>::type* __restrict__ tw) {
  using C = typename Complex<T>::type;
  using Geo = ColGeom<T, L, EP, CW>;
  using F = BlockFft<T, L, Geo::E, S>;
  __shared__ C lds[Geo::CC * lds_size(L)];
  const int t = threadIdx.x;
  const int64_t k2_0 = int64_t(blockIdx.x) * Geo::CC;
  const C* src = in + int64_t(blockIdx.y) * seg_stride + k2_0 * L;
  for (int i = t; i < Geo::CC * L; i += Geo::NT) lds[(i / L) * lds_size(L) + lds_pad(i % L)] = src[i];
  __syncthreads();
  const int c = t % Geo::CC, tl = t / Geo::CC;
  C* reg = lds + c * lds_size(L);
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = reg[lds_pad(F::in_index(tl, i))];
  __syncthreads();
  F::run(v, reg, tl, F::twiddles(tw));
  C* dst = out + int64_t(blockIdx.y) * seg_stride + k2_0 + c;
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) dst[n2_count * F::out_index(tl, i)] = v[i];
}

// Four-step second pass fused with the real-signal twist (k_twist below): the
// output of row k2 at k1 (bin m = k2 + N2 k1 of Z) meets its mirror
// N/2 - m in row N2 - k2 at N1 - 1 - k1 (row 0: itself at N1 - k1 mod N1), so
// a workgroup takes mirrored row pairs: H = CC/2 rows j H + c and their
// mirrors N2 - j H - c (workgroup 0: rows 0 .. H-1, N2/2 and N2-H+1 .. N2-1,
// rows 0 and N2/2 being their own mirrors). After the row transforms the
// values go through LDS to the thread that twists each bin.
template <typename T, int L, int EP = 0, int CW = 0>
__global__ __launch_bounds__((ColGeom<T, L, EP, CW>::NT)) void k_spec_rows_twist(
    const typename Complex<T>::type* __restrict__ in, typename Complex<T>::type* __restrict__ out, int64_t n2,
    int64_t seg_stride, const typename Complex<T>::type* __restrict__ tw, Twiddle2<typename Complex<T>::type> tw2) {
  using C = typename Complex<T>::type;
  using Geo = ColGeom<T, L, EP, CW>;
  using F = BlockFft<T, L, Geo::E, -1>;
  constexpr int CC = Geo::CC, H = CC / 2;
  static_assert(CC % 2 == 0, "paired rows");
  __shared__ C lds[CC * lds_size(L)];
  const int t = threadIdx.x;
  const int64_t j = blockIdx.x;
  auto row_of = [&](int c) -> int64_t {
    if (j == 0) return c < H ? c : (c == H ? n2 / 2 : n2 - (c - H));
    return c < H ? j * H + c : n2 - (j * H + (c - H));
  };
  const C* src = in + int64_t(blockIdx.y) * seg_stride;
  for (int i = t; i < CC * L; i += Geo::NT) {
    const int c = i / L;
    lds[c * lds_size(L) + lds_pad(i % L)] = src[row_of(c) * L + (i % L)];
  }
  __syncthreads();
  const int c = t % CC, tl = t / CC;
  C* reg = lds + c * lds_size(L);
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = reg[lds_pad(F::in_index(tl, i))];
  __syncthreads();
  F::run(v, reg, tl, F::twiddles(tw));
  // every transform's output into its own LDS column, then the twist
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) reg[lds_pad(F::out_index(tl, i))] = v[i];
  __syncthreads();
  const int64_t r = row_of(c);
  const int pc = (j == 0 && (c == 0 || c == H)) ? c : (c < H ? c + H : c - H);
  const C* preg = lds + pc * lds_size(L);
  C* dst = out + int64_t(blockIdx.y) * seg_stride;
  const T hh = T(0.5);
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int k1 = F::out_index(tl, i);
    const int64_t m = r + n2 * k1;
    const C zp = v[i];
    if (m == 0) {   // X[0] and X[N/2] share slot 0
      dst[0] = C{zp.x + zp.y, zp.x - zp.y};
      continue;
    }
    const int k1m = r == 0 ? (L - k1) & (L - 1) : L - 1 - k1;
    const C zq = preg[lds_pad(k1m)];
    const C w = tw2(m);                          // e^{-2 pi i m / N}
    const C a = c_add(zp, c_conj(zq)), b = c_sub(zp, c_conj(zq));
    const C xp = c_add(a, c_mul_si<-1>(c_mul(w, b)));
    dst[m] = C{xp.x * hh, xp.y * hh};
  }
}

// Real-signal spectrum from the N/2-point FFT Z of the even/odd pairs of a
// segment, in place: for c in [0, N/2]
//   X[c] = (Z[c] + Z*[N/2-c])/2 - (i/2) e^{-2 pi i c/N} (Z[c] - Z*[N/2-c])
// (indices of Z mod N/2). Thread p owns the pair (p, N/2-p); the two real
// values X[0] and X[N/2] share slot 0 as (X[0], X[N/2]).
template <typename T>
__global__ __launch_bounds__(256) void k_twist(typename Complex<T>::type* __restrict__ Z, int64_t half,
                                              Twiddle2<typename Complex<T>::type> tw2) {
  using C = typename Complex<T>::type;
  const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (p > half / 2) return;
  C* z = Z + int64_t(blockIdx.y) * half;
  const T h = T(0.5);
  if (p == 0) {
    const C z0 = z[0];
    z[0] = C{z0.x + z0.y, z0.x - z0.y};
    return;
  }
  const int64_t q = half - p;
  const C zp = z[p], zq = z[q];
  const C w = tw2(p);                           // e^{-2 pi i p/N}; at q it is -conj(w)
  const C a = c_add(zp, c_conj(zq)), b = c_sub(zp, c_conj(zq));
  const C xp = c_add(a, c_mul_si<-1>(c_mul(w, b)));
  const C a2 = c_add(zq, c_conj(zp)), b2 = c_sub(zq, c_conj(zp));
  const C xq = c_sub(a2, c_mul_si<-1>(c_mul(c_conj(w), b2)));
  z[p] = C{xp.x * h, xp.y * h};
  if (q != p) z[q] = C{xq.x * h, xq.y * h};
}

// Segment lengths with N/2 = r * M2, r in {3, 5}, M2 a power of two: the
// half-size transform splits into r interleaved length-M2 transforms
// (decimation by r) and one radix-r combination.
//   forward:  Zp[n1][n2] = z[n1 + r n2];  F_n1 = DFT_M2(Zp[n1]);
//             Z[k2 + M2 k1] = sum_n1 e^{-2 pi i n1 k1 / r} e^{-2 pi i n1 k2 / (N/2)} F_n1[k2]
//   inverse:  A_n1[k2] = e^{+2 pi i n1 k2 / (N/2)} sum_k1 Z[k2 + M2 k1] e^{+2 pi i n1 k1 / r};
//             z[n1 + r n2] = IDFT_M2(A_n1)[n2]
// k_permute moves a segment between the natural order z[n] and the decimated
// rows Zp[n1][n2] (TO_ROWS) or back; k_radix does the combination. The same
// split serves full-length transforms of N = r * M points (the dense tiles):
// then the twiddles are e^{-+2 pi i n1 k2 / N}, one step of the N-point table
// per unit of n1 k2 (TSTEP = 1) instead of two.
template <typename T, bool TO_ROWS>
__global__ __launch_bounds__(256) void k_permute(const typename Complex<T>::type* __restrict__ in,
                                                 typename Complex<T>::type* __restrict__ out, int r, int64_t m2) {
  const int64_t half = r * m2;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;   // index in the decimated rows
  if (i >= half) return;
  const int64_t n1 = i / m2, n2 = i - n1 * m2;
  const int64_t n = n1 + r * n2;
  const int64_t base = int64_t(blockIdx.y) * half;
  if constexpr (TO_ROWS) out[base + i] = in[base + n];
  else out[base + n] = in[base + i];
}

// cos / sin of 2 pi k / R for R = 3, 5
template <typename T, int R>
__device__ __forceinline__ typename Complex<T>::type root_r(int k) {
  using C = typename Complex<T>::type;
  if constexpr (R == 3) {
    constexpr T c1 = static_cast<T>(-0.5), s1 = static_cast<T>(0.86602540378443864676);
    return k == 0 ? C{1, 0} : (k == 1 ? C{c1, s1} : C{c1, -s1});
  } else {
    constexpr T c1 = static_cast<T>(0.30901699437494742410), s1 = static_cast<T>(0.95105651629515357212);
    constexpr T c2 = static_cast<T>(-0.80901699437494742410), s2 = static_cast<T>(0.58778525229247312917);
    return k == 0 ? C{1, 0} : k == 1 ? C{c1, s1} : k == 2 ? C{c2, s2} : k == 3 ? C{c2, -s2} : C{c1, -s1};
  }
}

template <typename T, int R, int S, int TSTEP = 2>
__global__ __launch_bounds__(256) void k_radix(const typename Complex<T>::type* __restrict__ in,
                                               typename Complex<T>::type* __restrict__ out, int64_t m2,
                                               Twiddle2<typename Complex<T>::type> tw2) {
  using C = typename Complex<T>::type;
  const int64_t k2 = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k2 >= m2) return;
  const int64_t base = int64_t(blockIdx.y) * R * m2;
  C a[R], b[R];
  if constexpr (S < 0) {
    // F_n1[k2] times e^{-2 pi i n1 k2 / (N/2)} = tw2(2 n1 k2), then the radix-R DFT over n1
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) {
      const C f = in[base + n1 * m2 + k2];
      a[n1] = n1 == 0 ? f : c_mul(f, tw2(TSTEP * n1 * k2));
    }
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      C acc = a[0];
#pragma unroll
      for (int n1 = 1; n1 < R; ++n1) acc = c_add(acc, c_mul(a[n1], c_conj(root_r<T, R>((n1 * k1) % R))));
      b[k1] = acc;
    }
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) out[base + k2 + m2 * k1] = b[k1];
  } else {
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) a[k1] = in[base + k2 + m2 * k1];
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) {
      C acc = a[0];
#pragma unroll
      for (int k1 = 1; k1 < R; ++k1) acc = c_add(acc, c_mul(a[k1], root_r<T, R>((n1 * k1) % R)));
      b[n1] = n1 == 0 ? acc : c_mul(acc, c_conj(tw2(TSTEP * n1 * k2)));
    }
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) out[base + n1 * m2 + k2] = b[n1];
  }
}

}  // namespace qtam
