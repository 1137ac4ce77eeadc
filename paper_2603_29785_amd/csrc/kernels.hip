// QTAM forward / inverse transform kernels for gfx950 (MI355X).
//
// Forward (Sec. III; App. A):
//   1. spectrum: the N real samples of a segment, read as N/2 complex pairs
//      z[m] = x[2m] + i x[2m+1], go through an N/2-point complex FFT
//      (one LDS pass when N/2 fits a workgroup, else two passes of the
//      four-step factorisation N/2 = N1 * N2 through the workspace);
//   2. rows: one fused kernel per (segment, row) rebuilds the real-signal
//      spectrum X[c] from the packed halves on the fly, multiplies by the
//      window table, drops each bin at its baseband slot (c - s_k) mod N_out
//      (roll to baseband, crop, zero pad) and runs the N_out-point inverse
//      FFT in registers and LDS, storing the envelope row coalesced.
// Inverse (Sec. III canonical dual; App. C):
//   1. rows: N_out-point FFT of each envelope row; the kept slots, weighted
//      by the dual table sqrt(N/N_out) W M / P / N, go to a packed buffer;
//   2. overlap-add: each thread sums the covering rows of a bin pair
//      (b, N/2-b) in fixed row order (no atomics) and applies the real-signal
//      pre-twist, giving the N/2-point half-size spectrum;
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

#include "fft_engine.hpp"
#include "plan.hpp"
#include "qtam.h"

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
  static constexpr int E = L < elems_per_thread<T>() ? L : elems_per_thread<T>();
  static constexpr int TPR = L / E;
  static constexpr int G = TPR >= 256 ? 1 : 256 / TPR;   // transforms per workgroup
  static constexpr int NT = G * TPR;
};

// Columns per workgroup of the four-step passes: C * L values fill at most
// 64 KiB of LDS, at least 4 columns for 32/64-byte contiguous runs.
template <typename T, int L>
struct ColGeom {
  static constexpr int E = L < elems_per_thread<T>() ? L : elems_per_thread<T>();
  static constexpr int TPR = L / E;
  static constexpr int CAP = (65536 / (2 * int(sizeof(T)))) / L;
  static constexpr int CC = CAP >= 16 ? 16 : (CAP >= 4 ? CAP : 4);
  static constexpr int NT = CC * TPR;
};

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

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
template <typename T, int L, int S>
__global__ __launch_bounds__((ColGeom<T, L>::NT)) void k_fft_cols(
    const typename Complex<T>::type* __restrict__ in, typename Complex<T>::type* __restrict__ out,
    int64_t n1_count, int64_t seg_stride, const typename Complex<T>::type* __restrict__ tw,
    Twiddle2<typename Complex<T>::type> tw2, int tw_mul) {
  using C = typename Complex<T>::type;
  using Geo = ColGeom<T, L>;
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
template <typename T, int L, int S>
__global__ __launch_bounds__((ColGeom<T, L>::NT)) void k_fft_rows_t(
    const typename Complex<T>::type* __restrict__ in, typename Complex<T>::type* __restrict__ out,
    int64_t n2_count, int64_t seg_stride, const typename Complex<T>::type* __restrict__ tw) {
  using C = typename Complex<T>::type;
  using Geo = ColGeom<T, L>;
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
template <typename T, int L>
__global__ __launch_bounds__((ColGeom<T, L>::NT)) void k_spec_rows_twist(
    const typename Complex<T>::type* __restrict__ in, typename Complex<T>::type* __restrict__ out, int64_t n2,
    int64_t seg_stride, const typename Complex<T>::type* __restrict__ tw, Twiddle2<typename Complex<T>::type> tw2) {
  using C = typename Complex<T>::type;
  using Geo = ColGeom<T, L>;
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
// rows Zp[n1][n2] (TO_ROWS) or back; k_radix does the combination.
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

template <typename T, int R, int S>
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
      a[n1] = n1 == 0 ? f : c_mul(f, tw2(2 * n1 * k2));
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
      b[n1] = n1 == 0 ? acc : c_mul(acc, c_conj(tw2(2 * n1 * k2)));
    }
#pragma unroll
    for (int n1 = 0; n1 < R; ++n1) out[base + n1 * m2 + k2] = b[n1];
  }
}

// Dense tiles: row k of segment s as an N-point spectrum holding its packed
// kept entries at their bins lo..hi and zeros elsewhere (the inverse FFT of
// that row is the dense tile). One thread per output bin, rows in grid.y.
template <typename T>
__global__ __launch_bounds__(256) void k_place(const typename Complex<T>::type* __restrict__ Sbuf,
                                               typename Complex<T>::type* __restrict__ D, const RowMeta* __restrict__ rows,
                                               int R, int64_t n, int64_t sum_len) {
  using C = typename Complex<T>::type;
  const int64_t b = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (b >= n) return;
  const int64_t gr = blockIdx.y;
  const int64_t seg = gr / R;
  const RowMeta rm = rows[gr - seg * R];
  const bool in = b >= rm.lo && b <= rm.hi;
  D[gr * n + b] = in ? Sbuf[seg * sum_len + rm.off + (b - rm.lo)] : C{0, 0};
}

// Single-tile recovery: row `row` of each segment, its N_out-point forward
// transform, every slot whose bin c = s + j lies in 0..N/2 times the tile
// table (sqrt(N/N_out) / W / N) into Sx[seg][c]. One segment per row group.
template <typename T, int L>
__global__ __launch_bounds__((RowGeom<T, L>::NT)) void k_tile_rows(
    const typename Complex<T>::type* __restrict__ Y, typename Complex<T>::type* __restrict__ Sx,
    const RowMeta* __restrict__ rows, const T* __restrict__ tab, int R, int row, int segs, int half,
    const typename Complex<T>::type* __restrict__ tw) {
  using C = typename Complex<T>::type;
  using Geo = RowGeom<T, L>;
  using F = BlockFft<T, L, Geo::E, -1, TW_MIXED>;
  __shared__ C lds[Geo::G * lds_size(L)];
  const int t = threadIdx.x, g = t / Geo::TPR, tl = t % Geo::TPR;
  const int seg = static_cast<int>(blockIdx.x) * Geo::G + g;
  const bool ok = seg < segs;
  const rsrc_t ry = make_rsrc(Y + (int64_t(ok ? seg : 0) * R + row) * L, ok ? static_cast<uint32_t>(L * sizeof(C)) : 0u);
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = bload<C>(ry, static_cast<uint32_t>(tl + F::in_off(i)) * sizeof(C));
  F::run(v, lds + g * lds_size(L), tl, F::twiddles(tw));
  if (!ok) return;
  const RowMeta rm = rows[row];
  C* dst = Sx + int64_t(seg) * (half + 1);
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int off = F::out_off(i);
    const int c = rm.s + tl + (off < L / 2 ? off : off - L);
    if (c >= rm.lo && c <= rm.hi) {
      const T w = tab[rm.off + c - rm.lo];
      dst[c] = C{v[i].x * w, v[i].y * w};
    }
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup i runs on
// XCD i mod 8) and roughly in index order. Renumbering them so that XCD x
// takes the x-th eighth of the units makes the workgroups resident on one XCD
// at a time work on neighbouring rows, whose spectrum that XCD's L2 holds.
__device__ __forceinline__ int xcd_major_block(int nblocks) {
  const int b = blockIdx.x;
  if (nblocks & 7) return b;
  return (b & 7) * (nblocks >> 3) + (b >> 3);
}

// Fused forward rows: the windowed spectrum bins of a row are dropped at
// their baseband slots (c - s_k) mod N_out (roll to baseband, crop, zero pad),
// the N_out-point inverse FFT runs in registers and LDS, and the envelope row
// is stored. One unit of G consecutive rows per workgroup.
// Cache policy of the envelope stores: Y is written once and not read again
// by the forward, so streaming it past the L2 keeps the spectrum and the plan
// tables, which every row re-reads, resident there (measured: the forward
// rows kernel of the batched workload drops from 0.70 to 0.50 ms). Loads of
// Y by the inverse keep the default policy (streaming them measured no gain
// and slowed the overlap-add that follows).
constexpr int kYStore = kCacheNT;
constexpr int kYLoad = kCacheDefault;
// The packed kept slots are read once, by the overlap-add after the whole
// inverse-rows launch: streamed as well (measured 1-3% on both kernels).
constexpr int kSStore = kCacheNT;

// Hides a value's derivation from the optimiser (an empty asm that keeps it
// in a VGPR), so per-element offsets stay one add from a precomputed base
// instead of being refolded into an add and a shift per resource.
__device__ __forceinline__ void opaque(unsigned& v) { asm volatile("" : "+v"(v)); }

// Row statistics (sum and max of |Y|^2 over the row) of the E values each of
// a row's TPR threads holds. Lanes of one row inside a wave combine by an xor
// butterfly (every lane ends with the same bits); rows spanning several waves
// then add the per-wave results in wave order through `part` (LDS the
// transform no longer reads, NT/64 elements). Every thread of the block must
// call it.
template <typename T, int E, int TPR, int NT>
__device__ __forceinline__ void row_stats(const typename Complex<T>::type (&v)[E], int tl, bool ok,
                                          typename Complex<T>::type* __restrict__ dst,
                                          typename Complex<T>::type* __restrict__ part) {
  using C = typename Complex<T>::type;
  constexpr int W = TPR < 64 ? TPR : 64;     // lanes of a row within one wave
  constexpr int WPR = TPR > 64 ? TPR / 64 : 1;
  T e = 0, m = 0;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const T a = v[i].x * v[i].x + v[i].y * v[i].y;
    e += a;
    m = fmax(m, a);
  }
#pragma unroll
  for (int o = 1; o < W; o <<= 1) {
    e += __shfl_xor(e, o, W);
    m = fmax(m, __shfl_xor(m, o, W));
  }
  if constexpr (WPR == 1) {
    if (ok && tl == 0) *dst = C{e, m};
  } else {
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = C{e, m};
    __syncthreads();
    if (ok && tl == 0) {
      const C* pr = part + (threadIdx.x >> 6);
      C r = pr[0];
#pragma unroll
      for (int w = 1; w < WPR; ++w) {
        r.x += pr[w].x;
        r.y = fmax(r.y, pr[w].y);
      }
      *dst = r;
    }
  }
}

// When a wave holds one row (TPR >= 64) and the row touches neither DC nor
// Nyquist, buffer resources scoped to the row's kept support do the cropping:
// slots outside it fall outside the resources and read 0, with no test.
// Otherwise each slot is tested; ANALYTIC then computes the bisquare weight
// scale_k (1 - (j/h_k)^2)^2 instead of reading the table.
template <typename T, int L, bool ANALYTIC, bool STATS>
__global__ __launch_bounds__((RowGeom<T, L>::NT)) void k_fwd_rows(
    const typename Complex<T>::type* __restrict__ spec, typename Complex<T>::type* __restrict__ Y,
    const RowMeta* __restrict__ rows, const typename Complex<T>::type* __restrict__ roww,
    const T* __restrict__ tab, int R, int total, int half, int sum_len, int64_t spec_elems,
    const typename Complex<T>::type* __restrict__ tw, int nblocks, typename Complex<T>::type* __restrict__ stats) {
  using C = typename Complex<T>::type;
  using Geo = RowGeom<T, L>;
  using F = BlockFft<T, L, Geo::E, +1, TW_MIXED>;
  constexpr bool kWaveRow = Geo::TPR >= 64;   // every lane of a wave is on the same row
  __shared__ C lds[Geo::G * lds_size(L)];
  const int t = threadIdx.x, g = t / Geo::TPR, tl = t % Geo::TPR;
  const int u = xcd_major_block(nblocks);
  int gr = u * Geo::G + g;
  if constexpr (kWaveRow) gr = __builtin_amdgcn_readfirstlane(gr);
  const bool ok = gr < total;
  const int seg = ok ? gr / R : 0;
  const int row = ok ? gr - seg * R : 0;
  const RowMeta rm = rows[row];
  C v[Geo::E];
  if (kWaveRow && rm.lo > 0 && rm.hi < half) {
    const int len = rm.hi - rm.lo + 1;
    const rsrc_t rz = make_rsrc(spec + int64_t(seg) * half + rm.lo, ok ? static_cast<uint32_t>(len * sizeof(C)) : 0u);
    const rsrc_t rt = make_rsrc(tab + rm.off, ok ? static_cast<uint32_t>(len * sizeof(T)) : 0u);
    const int db = rm.s - rm.lo + tl;   // kept-bin index d = c - lo of the slot with offset 0
    // byte offsets of d in both resources, advanced by constants (negative d
    // wraps beyond the resource and reads 0)
    unsigned bx = static_cast<unsigned>(db) * static_cast<unsigned>(sizeof(C));
    unsigned bw = static_cast<unsigned>(db) * static_cast<unsigned>(sizeof(T));
    opaque(bx);
    opaque(bw);
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) {
      const int off = F::in_off(i);
      const unsigned j = static_cast<unsigned>(off < L / 2 ? off : off - L);
      const C x = bload<C>(rz, bx + j * static_cast<unsigned>(sizeof(C)));
      const T w = bload<T>(rt, bw + j * static_cast<unsigned>(sizeof(T)));
      v[i] = C{x.x * w, x.y * w};
    }
  } else {
    const rsrc_t rz = make_rsrc(spec, static_cast<uint32_t>(spec_elems * sizeof(C)));
    const rsrc_t rt = make_rsrc(tab, static_cast<uint32_t>(sum_len * sizeof(T)));

    const unsigned zb = static_cast<unsigned>(seg) * static_cast<unsigned>(half);
    const int cb = rm.s + tl;
    // X[c] of the slots in the kept support; other slots get an offset beyond
    // the buffer and read 0 without touching memory
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) {
      const int off = F::in_off(i);
      const int c = cb + (off < L / 2 ? off : off - L);   // slot tl + off holds offset j = slot or slot - L
      const bool in = ok && c >= rm.lo && c <= rm.hi;
      const unsigned vo = in ? (zb + static_cast<unsigned>(c == half ? 0 : c)) * static_cast<unsigned>(sizeof(C))
                             : 0xFFFFFFFFu;
      v[i] = bload<C>(rz, vo);
    }
    C sw{0, 0};
    if constexpr (ANALYTIC) sw = roww[row];   // (scale_k, 1/h_k)
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) {
      const int off = F::in_off(i);
      const int j = tl + (off < L / 2 ? off : off - L);
      const int c = rm.s + j;
      C val = v[i];
      if (c == 0) val.y = 0;               // slot 0 of the spectrum holds (X[0], X[N/2])
      if (c == half) val = C{val.y, 0};
      T w;
      if constexpr (ANALYTIC) {
        const T x = static_cast<T>(j) * sw.y;
        const T b = (T(1) - x) * (T(1) + x);
        w = sw.x * b * b;
      } else {
        const bool in = ok && c >= rm.lo && c <= rm.hi;
        w = bload<T>(rt, static_cast<uint32_t>(in ? rm.off - rm.lo + c : 0) * sizeof(T));
      }
      v[i] = C{val.x * w, val.y * w};
    }
  }
  // Inputs outside the row's kept offsets [jlo, jhi] are zero; when every
  // lane of this wave has zeros in first-pass inputs 1..14 (or 2..13) the
  // first pass skips them (same results, fewer operations).
  int nz = 0;
  if constexpr (kWaveRow && F::R0 == 16) {
    const int jlo = rm.lo - rm.s, jhi = rm.hi - rm.s;
    const int t0 = __builtin_amdgcn_readfirstlane(tl) & ~63;
    constexpr int Q = L / 16;   // input i of lane tl sits at slot tl + i Q
    auto zero = [&](int a, int b) { return t0 + a * Q > jhi && t0 + 63 + b * Q < L + jlo; };
    nz = zero(1, 14) ? 2 : (zero(2, 13) ? 4 : 0);
  }
  F::run(v, lds + g * lds_size(L), tl, F::twiddles(tw), nz);
  const int64_t r0 = int64_t(u) * Geo::G;
  const int64_t nrow = total - r0 < Geo::G ? total - r0 : Geo::G;
  const rsrc_t ry = make_rsrc(Y + r0 * L, static_cast<uint32_t>(nrow * L * sizeof(C)));
  const uint32_t vb = static_cast<uint32_t>(g * L + tl) * sizeof(C);
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) bstore<C, kYStore>(ry, v[i], vb, F::out_off(i) * sizeof(C));
  if constexpr (STATS) row_stats<T, Geo::E, Geo::TPR, Geo::NT>(v, tl, ok, stats + gr, lds);
}

// Inverse rows: N_out-point FFT of each envelope row; the kept slots times the
// table go to the packed per-segment buffer Sbuf[seg * sum_len + off + c - lo].
// With one row per wave, resources scoped to the row's packed entries drop
// the other slots' stores without a test.
template <typename T, int L>
__global__ __launch_bounds__((RowGeom<T, L>::NT)) void k_inv_rows(
    const typename Complex<T>::type* __restrict__ Y, typename Complex<T>::type* __restrict__ Sbuf,
    const RowMeta* __restrict__ rows, const T* __restrict__ tab, int R, int total, int sum_len, int segs,
    const typename Complex<T>::type* __restrict__ tw) {
  using C = typename Complex<T>::type;
  using Geo = RowGeom<T, L>;
  using F = BlockFft<T, L, Geo::E, -1, TW_MIXED>;
  constexpr bool kWaveRow = Geo::TPR >= 64;
  __shared__ C lds[Geo::G * lds_size(L)];
  const int t = threadIdx.x, g = t / Geo::TPR, tl = t % Geo::TPR;
  const int64_t r0 = int64_t(blockIdx.x) * Geo::G;
  const int64_t nrow = total - r0 < Geo::G ? total - r0 : Geo::G;
  const rsrc_t ry = make_rsrc(Y + r0 * L, static_cast<uint32_t>(nrow * L * sizeof(C)));
  const uint32_t vb = static_cast<uint32_t>(g * L + tl) * sizeof(C);
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = bload<C, kYLoad>(ry, vb, F::in_off(i) * sizeof(C));
  if constexpr (kWaveRow) {
    // the row's weights are requested before the transform, so their latency
    // hides behind it; rows past the end get empty resources
    const int gr = __builtin_amdgcn_readfirstlane(static_cast<int>(r0) + g);
    const bool ok = gr < total;
    const int seg = ok ? gr / R : 0;
    const RowMeta rm = rows[ok ? gr - seg * R : 0];
    const int len = ok ? rm.hi - rm.lo + 1 : 0;
    const int db = rm.s - rm.lo + tl;   // d = c - lo for the slot u = tl + off
    const rsrc_t rs = make_rsrc(Sbuf + int64_t(seg) * sum_len + rm.off, static_cast<uint32_t>(len * sizeof(C)));
    const rsrc_t rt = make_rsrc(tab + rm.off, static_cast<uint32_t>(len * sizeof(T)));
    unsigned bs = static_cast<unsigned>(db) * static_cast<unsigned>(sizeof(C));
    unsigned bw = static_cast<unsigned>(db) * static_cast<unsigned>(sizeof(T));
    opaque(bs);
    opaque(bw);
    T w[Geo::E];
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) {
      const int off = F::out_off(i);
      const unsigned j = static_cast<unsigned>(off < L / 2 ? off : off - L);
      w[i] = bload<T>(rt, bw + j * static_cast<unsigned>(sizeof(T)));
    }
    F::run(v, lds + g * lds_size(L), tl, F::twiddles(tw));
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) {
      const int off = F::out_off(i);
      const unsigned j = static_cast<unsigned>(off < L / 2 ? off : off - L);
      bstore<C, kSStore>(rs, C{v[i].x * w[i], v[i].y * w[i]}, bs + j * static_cast<unsigned>(sizeof(C)));
    }
  } else {
    F::run(v, lds + g * lds_size(L), tl, F::twiddles(tw));
    const int gr = static_cast<int>(r0) + g;
    if (gr >= total) return;
    const int seg = gr / R;
    const RowMeta rm = rows[gr - seg * R];
    const int len = rm.hi - rm.lo + 1;
    const int db = rm.s - rm.lo + tl;   // d = c - lo for the slot u = tl + off
    const rsrc_t rs = make_rsrc(Sbuf, static_cast<uint32_t>(int64_t(segs) * sum_len * sizeof(C)));
    const rsrc_t rt = make_rsrc(tab, static_cast<uint32_t>(sum_len * sizeof(T)));
    const unsigned sb = static_cast<unsigned>(seg) * static_cast<unsigned>(sum_len) + static_cast<unsigned>(rm.off);
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) {
      const int off = F::out_off(i);
      const int d = db + (off < L / 2 ? off : off - L);
      if (static_cast<unsigned>(d) < static_cast<unsigned>(len)) {
        const T w = bload<T>(rt, (rm.off + d) * sizeof(T));
        bstore<C, kSStore>(rs, C{v[i].x * w, v[i].y * w}, (sb + d) * sizeof(C));
      }
    }
  }
}

// Envelope lengths M = N_out that are not powers of two (the paper's minimal
// N_out, say): each row's length-M DFT by Bluestein's chirp-z identity,
//   sum_u g[u] e^{S 2 pi i u m / M} = a[m] sum_u (g[u] a[u]) b[m - u],
//   a[v] = e^{S pi i v^2 / M}, b[v] = conj(a[v]),
// the convolution as a cyclic one of power-of-two length L >= 2M - 1: a
// forward FFT, a product with Bhat = FFT_L(b wrapped) / L, an inverse FFT.
// Tables (FP64-built): chirp a[0..M) and Bhat[0..L) of the transform's sign.
template <typename T, int L, typename C, int E>
__device__ __forceinline__ void chirp_convolve(C (&v)[E], C* lds, int tl, const C* __restrict__ bhat,
                                               const C* __restrict__ tw) {
  using Geo = RowGeom<T, L>;
  static_assert(Geo::E == E, "row geometry");
  using F = BlockFft<T, L, Geo::E, -1, TW_POW>;
  using Fi = BlockFft<T, L, Geo::E, +1, TW_POW>;
  F::run(v, lds, tl, F::twiddles(tw));
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = c_mul(v[i], bhat[tl + F::out_off(i)]);
  // back to the input order of the second transform
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) lds[lds_pad(tl + F::out_off(i))] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = lds[lds_pad(tl + Fi::in_off(i))];
  __syncthreads();
  Fi::run(v, lds, tl, Fi::twiddles(tw));
}

// Forward rows, M not a power of two: gather the kept bins of each row at
// their slots (c - s) mod M times the forward table and the chirp, then
// Bluestein (sign +) and the output chirp; outputs m < M are stored.
template <typename T, int L>
__global__ __launch_bounds__((RowGeom<T, L>::NT)) void k_fwd_rows_bs(
    const typename Complex<T>::type* __restrict__ spec, typename Complex<T>::type* __restrict__ Y,
    const RowMeta* __restrict__ rows, const T* __restrict__ tab, int R, int total, int half, int sum_len,
    int64_t spec_elems, int M, const typename Complex<T>::type* __restrict__ chirp,
    const typename Complex<T>::type* __restrict__ bhat, const typename Complex<T>::type* __restrict__ tw) {
  using C = typename Complex<T>::type;
  using Geo = RowGeom<T, L>;
  using F = BlockFft<T, L, Geo::E, -1, TW_POW>;
  using Fi = BlockFft<T, L, Geo::E, +1, TW_POW>;
  __shared__ C lds[Geo::G * lds_size(L)];
  const int t = threadIdx.x, g = t / Geo::TPR, tl = t % Geo::TPR;
  const int gr = static_cast<int>(blockIdx.x) * Geo::G + g;
  const bool ok = gr < total;
  const int seg = ok ? gr / R : 0;
  const RowMeta rm = rows[ok ? gr - seg * R : 0];
  const rsrc_t rz = make_rsrc(spec, static_cast<uint32_t>(spec_elems * sizeof(C)));
  const rsrc_t rt = make_rsrc(tab, static_cast<uint32_t>(sum_len * sizeof(T)));
  const unsigned zb = static_cast<unsigned>(seg) * static_cast<unsigned>(half);
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int u = tl + F::in_off(i);                 // Bluestein slot; < M holds data
    const int j = u <= M / 2 ? u : u - M;            // offset from the centre bin
    const int c = rm.s + j;
    const bool in = ok && u < M && c >= rm.lo && c <= rm.hi;
    const unsigned vo = in ? (zb + static_cast<unsigned>(c == half ? 0 : c)) * static_cast<unsigned>(sizeof(C))
                           : 0xFFFFFFFFu;
    C x = bload<C>(rz, vo);
    if (c == 0) x.y = 0;
    if (c == half) x = C{x.y, 0};
    const T w = bload<T>(rt, static_cast<uint32_t>(in ? rm.off - rm.lo + c : 0) * sizeof(T));
    const C a = chirp[u < M ? u : 0];   // x is 0 outside the support
    v[i] = c_mul(C{x.x * w, x.y * w}, a);
  }
  chirp_convolve<T, L>(v, lds + g * lds_size(L), tl, bhat, tw);
  if (!ok) return;
  C* yrow = Y + int64_t(gr) * M;
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int m = tl + Fi::out_off(i);
    if (m < M) yrow[m] = c_mul(v[i], chirp[m]);
  }
}

// Inverse rows, M not a power of two: Bluestein (sign -) over each envelope
// row, then the kept slots times the table into the packed buffer.
template <typename T, int L>
__global__ __launch_bounds__((RowGeom<T, L>::NT)) void k_inv_rows_bs(
    const typename Complex<T>::type* __restrict__ Y, typename Complex<T>::type* __restrict__ Sbuf,
    const RowMeta* __restrict__ rows, const T* __restrict__ tab, int R, int total, int sum_len, int M,
    const typename Complex<T>::type* __restrict__ chirp, const typename Complex<T>::type* __restrict__ bhat,
    const typename Complex<T>::type* __restrict__ tw) {
  using C = typename Complex<T>::type;
  using Geo = RowGeom<T, L>;
  using F = BlockFft<T, L, Geo::E, -1, TW_POW>;
  using Fi = BlockFft<T, L, Geo::E, +1, TW_POW>;
  __shared__ C lds[Geo::G * lds_size(L)];
  const int t = threadIdx.x, g = t / Geo::TPR, tl = t % Geo::TPR;
  const int gr = static_cast<int>(blockIdx.x) * Geo::G + g;
  const bool ok = gr < total;
  const C* yrow = Y + int64_t(ok ? gr : 0) * M;
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int u = tl + F::in_off(i);
    const bool in = ok && u < M;
    const int uc = in ? u : 0;
    const C z = c_mul(yrow[uc], c_conj(chirp[uc]));
    v[i] = in ? z : C{0, 0};
  }
  chirp_convolve<T, L>(v, lds + g * lds_size(L), tl, bhat, tw);
  if (!ok) return;
  const int seg = gr / R;
  const RowMeta rm = rows[gr - seg * R];
  C* srow = Sbuf + int64_t(seg) * sum_len + rm.off;
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int u = tl + Fi::out_off(i);
    if (u >= M) continue;
    const int j = u <= M / 2 ? u : u - M;
    const int c = rm.s + j;
    if (c < rm.lo || c > rm.hi) continue;
    const C z = c_mul(v[i], c_conj(chirp[u]));
    const T w = tab[rm.off + c - rm.lo];
    srow[c - rm.lo] = C{z.x * w, z.y * w};
  }
}

// Rows longer than one workgroup's LDS transform (four-step over the
// workspace, N_out = L1 * L2, slot u = n1 + L1 n2, output m = k2 + L2 k1).
// Forward, first pass: for every row, column n1 gathers its L2 slots from the
// spectrum (windowed, zero outside the kept support), runs the length-L2
// inverse FFT, multiplies by exp(+2 pi i n1 k2 / N_out) and stores A[n1 + L1 k2]
// of the row. The second pass is k_fft_rows_t over the rows (lengths L1).
template <typename T, int L2>
__global__ __launch_bounds__((ColGeom<T, L2>::NT)) void k_fwd_rows_cols(
    const typename Complex<T>::type* __restrict__ spec, typename Complex<T>::type* __restrict__ A,
    const RowMeta* __restrict__ rows, const T* __restrict__ tab, int R, int half, int64_t n_out, int64_t l1,
    const typename Complex<T>::type* __restrict__ tw, Twiddle2<typename Complex<T>::type> tw2) {
  using C = typename Complex<T>::type;
  using Geo = ColGeom<T, L2>;
  using F = BlockFft<T, L2, Geo::E, +1>;
  __shared__ C lds[Geo::CC * lds_size(L2)];
  const int t = threadIdx.x, cc = t % Geo::CC, tl = t / Geo::CC;
  const int64_t n1 = int64_t(blockIdx.x) * Geo::CC + cc;
  const int64_t gr = blockIdx.y;               // row of the chunk
  const int64_t seg = gr / R;
  const RowMeta rm = rows[int(gr - seg * R)];
  const C* Z = spec + seg * half;
  const int64_t hn = n_out / 2;
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int64_t u = n1 + l1 * F::in_index(tl, i);
    const int64_t c = rm.s + (u < hn ? u : u - n_out);
    C val{0, 0};
    if (c >= rm.lo && c <= rm.hi) {
      val = Z[c == half ? 0 : c];
      if (c == 0) val.y = 0;                  // slot 0 holds (X[0], X[N/2])
      if (c == half) val = C{val.y, 0};
      const T w = tab[rm.off + (c - rm.lo)];
      val = C{val.x * w, val.y * w};
    }
    v[i] = val;
  }
  F::run(v, lds + cc * lds_size(L2), tl, F::twiddles(tw));
  C* dst = A + gr * n_out + n1;
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int64_t k2 = F::out_index(tl, i);
    C w = tw2(n1 * k2);
    w.y = -w.y;                               // exp(+2 pi i n1 k2 / N_out)
    dst[l1 * k2] = c_mul(v[i], w);
  }
}

// Inverse, second pass over long rows: length-L1 FFTs along the rows k2 of
// the intermediate (CC rows per workgroup, staged through LDS), then the kept
// output slots m = k2 + L2 k1 times the table go to the packed buffer.
template <typename T, int L1>
__global__ __launch_bounds__((ColGeom<T, L1>::NT)) void k_inv_rows_rowst(
    const typename Complex<T>::type* __restrict__ A, typename Complex<T>::type* __restrict__ Sbuf,
    const RowMeta* __restrict__ rows, const T* __restrict__ tab, int R, int64_t sum_len, int64_t n_out,
    int64_t l2, const typename Complex<T>::type* __restrict__ tw) {
  using C = typename Complex<T>::type;
  using Geo = ColGeom<T, L1>;
  using F = BlockFft<T, L1, Geo::E, -1>;
  __shared__ C lds[Geo::CC * lds_size(L1)];
  const int t = threadIdx.x;
  const int64_t gr = blockIdx.y;
  const int64_t k2_0 = int64_t(blockIdx.x) * Geo::CC;
  const C* src = A + gr * n_out + k2_0 * L1;
  for (int i = t; i < Geo::CC * L1; i += Geo::NT) lds[(i / L1) * lds_size(L1) + lds_pad(i % L1)] = src[i];
  __syncthreads();
  const int cc = t % Geo::CC, tl = t / Geo::CC;
  C* reg = lds + cc * lds_size(L1);
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = reg[lds_pad(F::in_index(tl, i))];
  __syncthreads();
  F::run(v, reg, tl, F::twiddles(tw));
  const int64_t seg = gr / R;
  const RowMeta rm = rows[int(gr - seg * R)];
  C* dst = Sbuf + seg * sum_len + rm.off - rm.lo;
  const T* tb = tab + rm.off - rm.lo;
  const int64_t hn = n_out / 2;
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int64_t m = k2_0 + cc + l2 * F::out_index(tl, i);
    const int64_t c = rm.s + (m < hn ? m : m - n_out);
    if (c >= rm.lo && c <= rm.hi) {
      const T w = tb[c];
      dst[c] = C{v[i].x * w, v[i].y * w};
    }
  }
}

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

// ===========================================================================
// Host side: plan object, dispatch, C ABI
// ===========================================================================
using namespace qtam;

namespace {

enum Kind { K_SPEC = 0, K_SPEC1, K_SPEC2, K_TWIST, K_FWD_ROWS, K_FWD_ROWS2, K_INV_ROWS, K_INV_ROWS2, K_OLA,
            K_SYN, K_SYN1, K_SYN2, K_ROW_STATS, K_PLANE_BEST, K_GATHER, K_SPEC_PERM, K_SPEC_RADIX, K_SYN_RADIX,
            K_SYN_PERM, K_DENSE_PLACE, K_DENSE_FFT, K_DENSE_FFT1, K_DENSE_FFT2, K_NUM };
const char* const kKindName[K_NUM] = {"spectrum_fft", "spectrum_fft_pass1", "spectrum_fft_pass2",
                                       "spectrum_twist", "fwd_rows", "fwd_rows_pass2", "inv_rows",
                                       "inv_rows_pass2", "overlap_add", "synthesis_fft",
                                       "synthesis_fft_pass1", "synthesis_fft_pass2", "row_stats",
                                       "plane_best", "gather_plane", "spectrum_permute", "spectrum_radix",
                                       "synthesis_radix", "synthesis_permute", "dense_place", "dense_fft",
                                       "dense_fft_pass1", "dense_fft_pass2"};

enum Table { T_FWD = 0, T_DUAL = 1, T_AFWD = 2, T_AINV = 3, T_DENSE = 4, T_TILE = 5 };

constexpr int kMaxLog2Single32 = 14;   // LDS-resident FFT up to 16384 points (FP32)
constexpr int kMaxLog2Single64 = 13;   // and 8192 points (FP64)

int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Text of the last HIP failure seen on this thread (qtam_last_error).
thread_local std::string g_last_error;

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
  bool dense_ok = false;        // N a power of two: dense tiles available
  bool dense_four_step = false; // N-point dense transforms in two passes, N = dn1 * dn2
  int64_t dn1 = 0, dn2 = 0;
  void* d_tw_dense = nullptr;   // Stockham twiddles of N (single pass)
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
  int64_t r1 = 0, r2 = 0;       // N_out = r1 * r2
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
  auto radix = [&](int64_t ns) { return (L / ns >= e) ? e : L / ns; };
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

int64_t engine_e(int64_t L, bool f64) { return std::min<int64_t>(L, f64 ? 8 : 16); }

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
    stockham_twiddles(tw, pl->n1, engine_e(pl->n1, f64), TW_POW);
    o_n1 = blob.add(tw.data(), tw.size() * sizeof(T));
    stockham_twiddles(tw, pl->n2, engine_e(pl->n2, f64), TW_POW);
    o_n2 = blob.add(tw.data(), tw.size() * sizeof(T));
  }
  size_t o_r1 = 0, o_r2 = 0, o_rf = 0, o_rc = 0;
  if (pl->big_rows) {
    stockham_twiddles(tw, pl->r1, engine_e(pl->r1, f64), TW_POW);
    o_r1 = blob.add(tw.data(), tw.size() * sizeof(T));
    stockham_twiddles(tw, pl->r2, engine_e(pl->r2, f64), TW_POW);
    o_r2 = blob.add(tw.data(), tw.size() * sizeof(T));
    const int nbr = ilog2(hp.n_out);
    pl->twr_bits = (nbr + 1) / 2;
    const int64_t nf = int64_t(1) << pl->twr_bits, ncs = int64_t(hp.n_out) >> pl->twr_bits;
    twiddles_strided(tw, nf, 1, hp.n_out);
    o_rf = blob.add(tw.data(), tw.size() * sizeof(T));
    twiddles_strided(tw, ncs, nf, hp.n_out);
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
    stockham_twiddles(tw, Lb, engine_e(Lb, f64), TW_POW);
    o_bstw = blob.add(tw.data(), tw.size() * sizeof(T));
  }
  size_t o_dt = 0, o_dn1 = 0, o_dn2 = 0;
  if (pl->dense_ok) {
    if (!pl->dense_four_step) {
      stockham_twiddles(tw, hp.n, engine_e(hp.n, f64), TW_POW);
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
    pl->d_bs_tw = d + o_bstw;
  }
  pl->d_tw_half = pl->four_step ? nullptr : d + o_half;
  pl->d_tw_n1 = pl->four_step ? d + o_n1 : nullptr;
  pl->d_tw_n2 = pl->four_step ? d + o_n2 : nullptr;
  if (pl->big_rows) {
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
    if (!pl->timing) return;
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
    pl->pending.push_back({kind, a, b});
  }
};

// ---------------------------------------------------------------------------
// Dispatch over compile-time sizes
// ---------------------------------------------------------------------------
#define QTAM_POW2_CASES(X) \
  X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14)

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

template <typename T, int S>
bool launch_fft_rows_t(int log2l, const void* in, void* out, int64_t n2, int64_t segs, int64_t seg_stride,
                       const void* tw, hipStream_t st) {
  using C = typename Complex<T>::type;
  switch (log2l) {
#define X(LG)                                                                                       \
  case LG:                                                                                          \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Col32 : kMaxLog2Col64)) {                       \
      using Geo = ColGeom<T, (1 << LG)>;                                                            \
      if (n2 % Geo::CC) return false;                                                               \
      hipLaunchKernelGGL((k_fft_rows_t<T, (1 << LG), S>), dim3(unsigned(n2 / Geo::CC), unsigned(segs)), \
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
      using Geo = ColGeom<T, (1 << LG)>;                                                            \
      if (n2 % Geo::CC) return false;                                                               \
      hipLaunchKernelGGL((k_spec_rows_twist<T, (1 << LG)>), dim3(unsigned(n2 / Geo::CC), unsigned(segs)), \
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

template <typename T>
bool launch_rows(bool forward, bool analytic, int log2l, const void* in, void* out, const RowMeta* rows,
                 const void* roww, const void* tab, int R, int64_t total_rows, int64_t half, int64_t sum_len,
                 const void* tw, hipStream_t st, void* stats = nullptr) {
  using C = typename Complex<T>::type;
  switch (log2l) {
#define X(LG)                                                                                          \
  case LG:                                                                                             \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Single32 : kMaxLog2Single64)) {                    \
      using Geo = RowGeom<T, (1 << LG)>;                                                               \
      const int blocks = static_cast<int>((total_rows + Geo::G - 1) / Geo::G);                         \
      if (forward) {                                                                                   \
        auto kern = stats ? (analytic ? k_fwd_rows<T, (1 << LG), true, true>                          \
                                      : k_fwd_rows<T, (1 << LG), false, true>)                         \
                          : (analytic ? k_fwd_rows<T, (1 << LG), true, false>                          \
                                      : k_fwd_rows<T, (1 << LG), false, false>);                       \
        hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(Geo::NT), 0, st, static_cast<const C*>(in), \
                           static_cast<C*>(out), rows, static_cast<const C*>(roww),                    \
                           static_cast<const T*>(tab), R, int(total_rows), int(half), int(sum_len),    \
                           (total_rows / R) * half, static_cast<const C*>(tw), blocks,                 \
                           static_cast<C*>(stats));                                                    \
      } else {                                                                                         \
        hipLaunchKernelGGL((k_inv_rows<T, (1 << LG)>), dim3(unsigned(blocks)), dim3(Geo::NT), 0, st,   \
                           static_cast<const C*>(in), static_cast<C*>(out), rows,                      \
                           static_cast<const T*>(tab), R, int(total_rows), int(sum_len),               \
                           int(total_rows / R), static_cast<const C*>(tw));                           \
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
  if (pl->big_rows) cap = std::min<int64_t>(cap, 65535 / hp.rows);   // rows of a chunk index grid.y
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
  return launch_fft_rows_t<T, S>(ilog2(pl->n1), tmp, out, pl->n2, count, m2, pl->d_tw_n1, st);
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

// analysis, second half: spectrum -> rows (forward with T_FWD, inverse adjoint
// with T_AINV). Reads ws + lay.spec, writes y (and ws + lay.rows for long rows).
template <typename T>
bool analysis_rows(qtam_plan_s* pl, int table, void* y, int64_t segs, char* ws, const WsLayout& lay,
                   hipStream_t st, void* stats) {
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
    {
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
                        pl->d_tw_out, st, stats);
}

template <typename T>
bool run_analysis(qtam_plan_s* pl, int table, const void* x, void* y, int64_t segs, char* ws,
                  const WsLayout& lay, hipStream_t st, void* stats) {
  return analysis_spectrum<T>(pl, x, segs, ws, lay, st) && analysis_rows<T>(pl, table, y, segs, ws, lay, st, stats);
}

// synthesis: rows -> real signal (inverse with T_DUAL, forward adjoint with T_AFWD)
template <typename T>
bool inverse_rows(qtam_plan_s* pl, int table, const void* y, int64_t segs, char* ws, const WsLayout& lay,
                  hipStream_t st) {
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
  } else if (pl->bluestein) {
    Timed tm(pl, K_INV_ROWS, st);
    ok = launch_rows_bs<T>(false, ilog2(pl->bs_len), y, pack, pl->d_rows, pl->d_tab[table], hp.rows, segs * hp.rows,
                           half, hp.sum_len, hp.n_out, pl->d_bs_chirp, pl->d_bs_bi, pl->d_bs_tw, st);
  } else {
    Timed tm(pl, K_INV_ROWS, st);
    ok = launch_rows<T>(false, false, ilog2(hp.n_out), y, pack, pl->d_rows, nullptr, pl->d_tab[table],
                        hp.rows, segs * hp.rows, half, hp.sum_len, pl->d_tw_out, st);
  }
  return ok;
}

template <typename T>
bool synthesize(qtam_plan_s* pl, const void* pack, int64_t slen, const int* starts, const OlaRow* list, void* x,
                int64_t segs, char* ws, const WsLayout& lay, hipStream_t st);

template <typename T>
bool run_synthesis(qtam_plan_s* pl, int table, const void* y, void* x, int64_t segs, char* ws,
                   const WsLayout& lay, hipStream_t st) {
  const HostPlan& hp = pl->hp;
  void* pack = ws + lay.pack;
  bool ok = inverse_rows<T>(pl, table, y, segs, ws, lay, st);
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
// placed at their bins of an N-point row, then N-point inverse transforms:
// placed in `dtmp` and transformed into `dense` (one pass), or placed in
// `dense`, first pass into `dtmp`, second pass back into `dense`.
template <typename T>
bool run_dense(qtam_plan_s* pl, const void* y, void* dense, int64_t segs, char* ws, const WsLayout& lay, void* dtmp,
               hipStream_t st) {
  using C = typename Complex<T>::type;
  const HostPlan& hp = pl->hp;
  if (!inverse_rows<T>(pl, T_DENSE, y, segs, ws, lay, st)) return false;
  const int64_t count = segs * hp.rows;
  {
    Timed tm(pl, K_DENSE_PLACE, st);
    hipLaunchKernelGGL((k_place<T>), dim3(unsigned((hp.n + 255) / 256), unsigned(count)), dim3(256), 0, st,
                       static_cast<const C*>(static_cast<void*>(ws + lay.pack)),
                       static_cast<C*>(pl->dense_four_step ? dense : dtmp), pl->d_rows, hp.rows, hp.n, hp.sum_len);
  }
  if (!pl->dense_four_step) {
    Timed tm(pl, K_DENSE_FFT, st);
    return launch_fft_rows<T, +1>(ilog2(hp.n), dtmp, dense, count, hp.n, pl->d_tw_dense, st);
  }
  bool ok;
  {
    Timed tm(pl, K_DENSE_FFT1, st);
    ok = launch_fft_cols<T, +1>(ilog2(pl->dn2), dense, dtmp, pl->dn1, count, hp.n, pl->d_tw_dn2, tw2_of<T>(pl), st, 1);
  }
  if (!ok) return false;
  Timed tm(pl, K_DENSE_FFT2, st);
  return launch_fft_rows_t<T, +1>(ilog2(pl->dn1), dtmp, dense, pl->dn2, count, hp.n, pl->d_tw_dn1, st);
}

// Segments per dense chunk: rows index grid.y, each chunk's tiles below 2 GiB.
int64_t dense_chunk_cap(const qtam_plan_s* pl) {
  const HostPlan& hp = pl->hp;
  const size_t per = size_t(hp.rows) * size_t(hp.n) * (hp.precision == QTAM_FP64 ? 16 : 8);
  int64_t cap = std::min<int64_t>(chunk_cap(pl), 65535 / hp.rows);
  cap = std::min<int64_t>(cap, per >= (size_t(1) << 31) ? 0 : int64_t(((size_t(1) << 31) - 1) / per));
  return cap;
}

size_t dense_ws_bytes(const qtam_plan_s* pl, int64_t segs) {
  const size_t cb = pl->hp.precision == QTAM_FP64 ? 16 : 8;
  return align256(layout_for(pl, segs).total) + size_t(segs) * size_t(pl->hp.rows) * size_t(pl->hp.n) * cb;
}

template <typename T>
bool launch_tile_rows(qtam_plan_s* pl, const void* y, void* sx, int row, int64_t segs, hipStream_t st) {
  using C = typename Complex<T>::type;
  const HostPlan& hp = pl->hp;
  Timed tm(pl, K_INV_ROWS, st);
  switch (ilog2(hp.n_out)) {
#define X(LG)                                                                                          \
  case LG:                                                                                             \
    if constexpr ((LG) <= (sizeof(T) == 4 ? kMaxLog2Single32 : kMaxLog2Single64)) {                    \
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

qtam_status run_op(qtam_plan_t pl, Op op, const void* in, void* out, int64_t batch, void* ws, size_t ws_bytes,
                   qtam_stream_t stream, void* stats = nullptr) {
  if (!pl || batch < 0) return QTAM_ERR_INVALID_ARG;
  if (batch == 0) return QTAM_OK;
  if (!in || !out || !ws) return QTAM_ERR_INVALID_ARG;
  if (!pl->gpu_supported) return pl->unsupported_reason;
  if (!pl->device) return QTAM_ERR_INVALID_ARG;
  const int64_t chunk = std::min<int64_t>(chunk_for(pl, batch, ws_bytes), 65535);
  if (chunk < 1) return QTAM_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const HostPlan& hp = pl->hp;
  const bool f64 = hp.precision == QTAM_FP64;
  const size_t rb = f64 ? 8 : 4;
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
    if (analysis)
      ok = f64 ? run_analysis<double>(pl, table, src, dst, segs, static_cast<char*>(ws), lay, st, chunk_stats)
               : run_analysis<float>(pl, table, src, dst, segs, static_cast<char*>(ws), lay, st, chunk_stats);
    else
      ok = f64 ? run_synthesis<double>(pl, table, src, dst, segs, static_cast<char*>(ws), lay, st)
               : run_synthesis<float>(pl, table, src, dst, segs, static_cast<char*>(ws), lay, st);
    if (!ok) return QTAM_ERR_UNSUPPORTED;
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
  // N_out not a power of two: chirp-z rows of the next power of two >= 2 N_out - 1
  pl->bluestein = !is_pow2(hp.n_out);
  if (pl->bluestein) {
    int64_t lb = 1;
    while (lb < 2 * int64_t(hp.n_out) - 1) lb *= 2;
    pl->bs_len = lb;
    if (ilog2(lb) > max_single || ilog2(lb) < 2) return;
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
  pl->big_rows = !pl->bluestein && ln > max_single;
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
  // dense tiles: N-point transforms, one pass or N = dn1 * dn2
  pl->dense_ok = false;
  if (is_pow2(hp.n)) {
    const int lt = ilog2(hp.n);
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
extern "C" {

const char* qtam_last_error(void) { return g_last_error.c_str(); }

const char* qtam_version(void) { return "qtam-gfx950 1.0"; }

const char* qtam_status_string(qtam_status s) {
  switch (s) {
    case QTAM_OK: return "ok";
    case QTAM_ERR_INVALID_ARG: return "invalid argument";
    case QTAM_ERR_UNSUPPORTED: return "unsupported on this device path";
    case QTAM_ERR_WORKSPACE: return "workspace too small";
    case QTAM_ERR_OOM: return "device out of memory";
    case QTAM_ERR_DEVICE: return "HIP device error";
  }
  return "unknown status";
}

qtam_status qtam_plan_create(const qtam_params* params, qtam_plan_t* out) {
  if (!out) return QTAM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!params) return QTAM_ERR_INVALID_ARG;
  qtam_plan_s* pl = new (std::nothrow) qtam_plan_s();
  if (!pl) return QTAM_ERR_OOM;
  qtam_status st = build_host_plan(*params, pl->hp);
  if (st != QTAM_OK) {
    delete pl;
    return st;
  }
  choose_geometry(pl);
  pl->seg_bytes = layout_for(pl, 1).total;
  if (!(params->flags & QTAM_PLAN_HOST_ONLY) && pl->gpu_supported) {
    const hipError_t e = hipGetDevice(&pl->device_id);
    if (e != hipSuccess) {
      delete pl;
      return hip_failed(e, "hipGetDevice");
    }
    if (hipDeviceGetAttribute(&pl->num_cus, hipDeviceAttributeMultiprocessorCount, pl->device_id) != hipSuccess ||
        pl->num_cus < 1) {
      (void)hipGetLastError();
      pl->num_cus = 1;
    }
    pl->analytic_fwd = pl->hp.all_bisquare && pl->hp.eps == 0.0;
    st = pl->hp.precision == QTAM_FP64 ? upload<double>(pl) : upload<float>(pl);
    if (st != QTAM_OK) {
      if (pl->dmem) (void)hipFree(pl->dmem);
      delete pl;
      return st;
    }
    pl->device = true;
  }
  *out = pl;
  return QTAM_OK;
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
  if (pl->big_rows || pl->bluestein) return QTAM_ERR_UNSUPPORTED;
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
    const bool ok = f64 ? (launch_tile_rows<double>(pl, src, sx, row, segs, st) &&
                           synthesize<double>(pl, sx, hp.half + 1, pl->d_one_start, pl->d_one_rows, dst, segs, w, lay, st))
                        : (launch_tile_rows<float>(pl, src, sx, row, segs, st) &&
                           synthesize<float>(pl, sx, hp.half + 1, pl->d_one_start, pl->d_one_rows, dst, segs, w, lay, st));
    if (!ok) return QTAM_ERR_UNSUPPORTED;
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) return hip_failed(e, "kernel launch");
  }
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
