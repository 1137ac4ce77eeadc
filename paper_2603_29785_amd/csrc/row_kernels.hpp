// Row kernels: the fused forward rows (gather x window, baseband placement,
// N_out-point inverse FFT; Sec. III, App. A and C demodulation) and the
// inverse rows (N_out-point FFT, kept slots x dual weights; Sec. III inverse,
// App. C re-modulation), their chirp-z forms for N_out that are not powers of
// two, their four-step forms for rows longer than one workgroup, and the
// dense-tile and single-tile kernels.
#pragma once

#include "device_common.hpp"
#include "mask_kernels.hpp"

namespace qtam {

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
// transform, every slot that holds a kept bin c (slot_entry) times the tile
// table (sqrt(N/N_out) / W / N) into Sx[seg][c]. One segment per row group.
template <typename T, int L>
__global__ __launch_bounds__((RowGeom<T, L>::NT)) void k_tile_rows(
    const typename Complex<T>::type* __restrict__ Y, typename Complex<T>::type* __restrict__ Sx,
    const RowMeta* __restrict__ rows, const T* __restrict__ tab, int R, int row, int segs, int half,
    const typename Complex<T>::type* __restrict__ tw) {
  using C = typename Complex<T>::type;
  using Geo = RowGeom<T, L>;
  using F = BlockFft<T, L, Geo::E, -1, TW_MIXED>;
  __shared__ C lds[Geo::G * fft_lds_elems<T, L>()];
  const int t = threadIdx.x, g = t / Geo::TPR, tl = t % Geo::TPR;
  const int seg = static_cast<int>(blockIdx.x) * Geo::G + g;
  const bool ok = seg < segs;
  const rsrc_t ry = make_rsrc(Y + (int64_t(ok ? seg : 0) * R + row) * L, ok ? static_cast<uint32_t>(L * sizeof(C)) : 0u);
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = bload<C>(ry, static_cast<uint32_t>(tl + F::in_off(i)) * sizeof(C));
  F::run(v, lds + g * fft_lds_elems<T, L>(), tl, F::twiddles(tw));
  if (!ok) return;
  const RowMeta rm = rows[row];
  C* dst = Sx + int64_t(seg) * (half + 1);
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int d = slot_entry<L>(tl + F::out_off(i), rm);
    if (d <= rm.hi - rm.lo) {
      const T w = tab[rm.off + d];
      dst[rm.lo + d] = C{v[i].x * w, v[i].y * w};
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

// Sum of one value per thread over each row of the block, in a fixed order:
// an xor butterfly over a row's lanes within a wave, then (rows spanning
// several waves) the per-wave sums in wave order through `part` (LDS the
// transform no longer reads, NT/64 elements). Every thread of the block must
// call it.
template <typename T, int TPR, int NT>
__device__ __forceinline__ void row_sum(T s, int tl, bool ok, T* __restrict__ dst, T* __restrict__ part) {
  constexpr int W = TPR < 64 ? TPR : 64;
  constexpr int WPR = TPR > 64 ? TPR / 64 : 1;
#pragma unroll
  for (int o = 1; o < W; o <<= 1) s += __shfl_xor(s, o, W);
  if constexpr (WPR == 1) {
    if (ok && tl == 0) *dst = s;
  } else {
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (ok && tl == 0) {
      const T* pr = part + (threadIdx.x >> 6);
      T r = pr[0];
#pragma unroll
      for (int w = 1; w < WPR; ++w) r += pr[w];
      *dst = r;
    }
  }
}

// When a wave holds one row (TPR >= 64) and the row touches neither DC nor
// Nyquist, buffer resources scoped to the row's kept support do the cropping:
// slots outside it fall outside the resources and read 0, with no test.
// Otherwise each slot is tested; ANALYTIC then computes the bisquare weight
// scale_k (1 - (j/h_k)^2)^2 instead of reading the table.
// MBWD (the inverse adjoint of a masked inverse): the transform's output is
// the gradient G with respect to the masked envelope Y' = g_k m Y; the kernel
// reads Y (mY, same layout as the output) and stores dL/dY instead, and the
// row's sum of m Re(conj(Y) G) goes to mpart[row] (the gain gradient's share).
template <typename T, int L, bool ANALYTIC, bool STATS, bool MBWD = false>
__global__ __launch_bounds__((RowGeom<T, L>::NT)) void k_fwd_rows(
    const typename Complex<T>::type* __restrict__ spec, typename Complex<T>::type* __restrict__ Y,
    const RowMeta* __restrict__ rows, const typename Complex<T>::type* __restrict__ roww,
    const T* __restrict__ tab, int R, int total, int half, int sum_len, int64_t spec_elems,
    const typename Complex<T>::type* __restrict__ tw, int nblocks, typename Complex<T>::type* __restrict__ stats,
    const typename Complex<T>::type* __restrict__ mY, const T* __restrict__ mgain, const T* __restrict__ mlam,
    T* __restrict__ mpart) {
  using C = typename Complex<T>::type;
  using Geo = RowGeom<T, L>;
  using F = BlockFft<T, L, Geo::E, +1, TW_MIXED>;
  constexpr bool kWaveRow = Geo::TPR >= 64;   // every lane of a wave is on the same row
  __shared__ C lds[Geo::G * fft_lds_elems<T, L>()];
  const int t = threadIdx.x, g = t / Geo::TPR, tl = t % Geo::TPR;
  const int u = xcd_major_block(nblocks);
  int gr = u * Geo::G + g;
  if constexpr (kWaveRow) gr = __builtin_amdgcn_readfirstlane(gr);
  const bool ok = gr < total;
  const int seg = ok ? gr / R : 0;
  const int row = ok ? gr - seg * R : 0;
  const RowMeta rm = rows[row];
  const bool centred = row_centred(rm, L);
  C v[Geo::E];
  if (kWaveRow && rm.lo > 0 && rm.hi < half && centred) {
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
    const int last = rm.hi - rm.lo;
    // X[c] of the slots holding a kept bin c = lo + d; other slots get an
    // offset beyond the buffer and read 0 without touching memory
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) {
      const int d = slot_entry<L>(tl + F::in_off(i), rm);
      const int c = rm.lo + d;
      const bool in = ok && d <= last;
      const unsigned vo = in ? (zb + static_cast<unsigned>(c == half ? 0 : c)) * static_cast<unsigned>(sizeof(C))
                             : 0xFFFFFFFFu;
      v[i] = bload<C>(rz, vo);
    }
    C sw{0, 0};
    if constexpr (ANALYTIC) sw = roww[row];   // (scale_k, 1/h_k)
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) {
      const int d = slot_entry<L>(tl + F::in_off(i), rm);
      const int c = rm.lo + d;
      const int j = c - rm.s;
      C val = v[i];
      if (c == 0) val.y = 0;               // slot 0 of the spectrum holds (X[0], X[N/2])
      if (c == half) val = C{val.y, 0};
      T w;
      if constexpr (ANALYTIC) {
        const T x = static_cast<T>(j) * sw.y;
        const T b = (T(1) - x) * (T(1) + x);
        w = sw.x * b * b;
      } else {
        const bool in = ok && d <= last;
        w = bload<T>(rt, static_cast<uint32_t>(in ? rm.off + d : 0) * sizeof(T));
      }
      v[i] = C{val.x * w, val.y * w};
    }
  }
  // Inputs of a centred row outside its kept offsets [jlo, jhi] are zero; when every
  // lane of this wave has zeros in first-pass inputs 1..14 (or 2..13) the
  // first pass skips them (same results, fewer operations).
  int nz = 0;
  if constexpr (kWaveRow && F::R0 == 16 && Geo::E == 16) {
    const int jlo = rm.lo - rm.s, jhi = rm.hi - rm.s;
    const int t0 = __builtin_amdgcn_readfirstlane(tl) & ~63;
    constexpr int Q = L / 16;   // input i of lane tl sits at slot tl + i Q
    auto zero = [&](int a, int b) { return t0 + a * Q > jhi && t0 + 63 + b * Q < L + jlo; };
    nz = !centred ? 0 : (zero(1, 14) ? 2 : (zero(2, 13) ? 4 : 0));
  }
  F::run(v, lds + g * fft_lds_elems<T, L>(), tl, F::twiddles(tw), nz);
  const int64_t r0 = int64_t(u) * Geo::G;
  const int64_t nrow = total - r0 < Geo::G ? total - r0 : Geo::G;
  const rsrc_t ry = make_rsrc(Y + r0 * L, static_cast<uint32_t>(nrow * L * sizeof(C)));
  const uint32_t vb = static_cast<uint32_t>(g * L + tl) * sizeof(C);
  if constexpr (MBWD) {
    const rsrc_t rm = make_rsrc(mY + r0 * L, static_cast<uint32_t>(nrow * L * sizeof(C)));
    const T gk = ok ? mgain[row] : T(0), lk = ok ? mlam[row] : T(0);
    T acc = 0;
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) {
      const C yv = bload<C>(rm, vb, F::out_off(i) * sizeof(C));
      v[i] = MaskMath<T>::grad(yv, v[i], gk, lk, acc);
    }
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) bstore<C, kYStore>(ry, v[i], vb, F::out_off(i) * sizeof(C));
    row_sum<T, Geo::TPR, Geo::NT>(acc, tl, ok, mpart + gr, reinterpret_cast<T*>(lds));
  } else {
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) bstore<C, kYStore>(ry, v[i], vb, F::out_off(i) * sizeof(C));
    if constexpr (STATS) row_stats<T, Geo::E, Geo::TPR, Geo::NT>(v, tl, ok, stats + gr, lds);
  }
}

// Inverse rows: N_out-point FFT of each envelope row; the kept slots times the
// table go to the packed per-segment buffer Sbuf[seg * sum_len + off + c - lo].
// With one row per wave, resources scoped to the row's packed entries drop
// the other slots' stores without a test.
// MASK (a masked inverse): each loaded value y becomes g_k max(0, 1 -
// lambda_k / |y|) y (the mask of the denoiser) before the transform.
template <typename T, int L, bool MASK = false>
__global__ __launch_bounds__((RowGeom<T, L>::NT)) void k_inv_rows(
    const typename Complex<T>::type* __restrict__ Y, typename Complex<T>::type* __restrict__ Sbuf,
    const RowMeta* __restrict__ rows, const T* __restrict__ tab, int R, int total, int sum_len, int segs,
    const typename Complex<T>::type* __restrict__ tw, const T* __restrict__ mgain, const T* __restrict__ mlam) {
  using C = typename Complex<T>::type;
  using Geo = RowGeom<T, L>;
  using F = BlockFft<T, L, Geo::E, -1, TW_MIXED>;
  constexpr bool kWaveRow = Geo::TPR >= 64;
  __shared__ C lds[Geo::G * fft_lds_elems<T, L>()];
  const int t = threadIdx.x, g = t / Geo::TPR, tl = t % Geo::TPR;
  const int64_t r0 = int64_t(blockIdx.x) * Geo::G;
  const int64_t nrow = total - r0 < Geo::G ? total - r0 : Geo::G;
  const rsrc_t ry = make_rsrc(Y + r0 * L, static_cast<uint32_t>(nrow * L * sizeof(C)));
  const uint32_t vb = static_cast<uint32_t>(g * L + tl) * sizeof(C);
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = bload<C, kYLoad>(ry, vb, F::in_off(i) * sizeof(C));
  if constexpr (MASK) {
    int gm = static_cast<int>(r0) + g;
    if constexpr (kWaveRow) gm = __builtin_amdgcn_readfirstlane(gm);
    const int km = gm < total ? gm % R : 0;
    const T gk = mgain[km], lk = mlam[km];
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) v[i] = MaskMath<T>::apply(v[i], gk, lk);
  }
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
    const bool centred = row_centred(rm, L);
    unsigned bs = static_cast<unsigned>(db) * static_cast<unsigned>(sizeof(C));
    unsigned bw = static_cast<unsigned>(db) * static_cast<unsigned>(sizeof(T));
    opaque(bs);
    opaque(bw);
    // (rows of 32 values per thread load them after the transform: registers)
    constexpr bool kEarly = Geo::E <= 16;
    T w[kEarly ? Geo::E : 1];
    if constexpr (kEarly) {
#pragma unroll
      for (int i = 0; i < Geo::E; ++i) {
        const int off = F::out_off(i);
        const unsigned j = static_cast<unsigned>(off < L / 2 ? off : off - L);
        w[i] = bload<T>(rt, bw + j * static_cast<unsigned>(sizeof(T)));
      }
    }
    F::run(v, lds + g * fft_lds_elems<T, L>(), tl, F::twiddles(tw));
    if (!centred) {
      // a row of a regularised window: slot entries taken modulo L (the
      // early weights above are not used)
#pragma unroll
      for (int i = 0; i < Geo::E; ++i) {
        const unsigned d = static_cast<unsigned>(slot_entry<L>(tl + F::out_off(i), rm));
        const T wi = bload<T>(rt, d * static_cast<unsigned>(sizeof(T)));
        bstore<C, kSStore>(rs, C{v[i].x * wi, v[i].y * wi}, d * static_cast<unsigned>(sizeof(C)));
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) {
      const int off = F::out_off(i);
      const unsigned j = static_cast<unsigned>(off < L / 2 ? off : off - L);
      T wi;
      if constexpr (kEarly) wi = w[i];
      else wi = bload<T>(rt, bw + j * static_cast<unsigned>(sizeof(T)));
      bstore<C, kSStore>(rs, C{v[i].x * wi, v[i].y * wi}, bs + j * static_cast<unsigned>(sizeof(C)));
    }
  } else {
    F::run(v, lds + g * fft_lds_elems<T, L>(), tl, F::twiddles(tw));
    const int gr = static_cast<int>(r0) + g;
    if (gr >= total) return;
    const int seg = gr / R;
    const RowMeta rm = rows[gr - seg * R];
    const int len = rm.hi - rm.lo + 1;
    const rsrc_t rs = make_rsrc(Sbuf, static_cast<uint32_t>(int64_t(segs) * sum_len * sizeof(C)));
    const rsrc_t rt = make_rsrc(tab, static_cast<uint32_t>(sum_len * sizeof(T)));
    const unsigned sb = static_cast<unsigned>(seg) * static_cast<unsigned>(sum_len) + static_cast<unsigned>(rm.off);
#pragma unroll
    for (int i = 0; i < Geo::E; ++i) {
      const int d = slot_entry<L>(tl + F::out_off(i), rm);
      if (d < len) {
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
  // slot u holds the kept bin c = lo + d, d = (u + s - lo) mod M, if d <= hi - lo
  int sh = (rm.s - rm.lo) % M;
  if (sh < 0) sh += M;
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int u = tl + F::in_off(i);                 // Bluestein slot; < M holds data
    const int d = u + sh < M ? u + sh : u + sh - M;
    const int c = rm.lo + d;
    const bool in = ok && u < M && d <= rm.hi - rm.lo;
    const unsigned vo = in ? (zb + static_cast<unsigned>(c == half ? 0 : c)) * static_cast<unsigned>(sizeof(C))
                           : 0xFFFFFFFFu;
    C x = bload<C>(rz, vo);
    if (c == 0) x.y = 0;
    if (c == half) x = C{x.y, 0};
    const T w = bload<T>(rt, static_cast<uint32_t>(in ? rm.off + d : 0) * sizeof(T));
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
  int sh = (rm.s - rm.lo) % M;   // slot u holds kept entry d = (u + s - lo) mod M
  if (sh < 0) sh += M;
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int u = tl + Fi::out_off(i);
    if (u >= M) continue;
    const int d = u + sh < M ? u + sh : u + sh - M;
    if (d > rm.hi - rm.lo) continue;
    const C z = c_mul(v[i], c_conj(chirp[u]));
    const T w = tab[rm.off + d];
    srow[d] = C{z.x * w, z.y * w};
  }
}

// Chirp-z rows whose convolution length L exceeds one workgroup's transform:
// the products before and after the length-L cyclic convolution run as
// element passes around four-step transforms through the workspace (rows of
// L values, row gr = seg * R + k). Same identity and tables as above.
// Forward, before: B[gr][u] = X[c] F_k[c] a[u] for the kept bin c of slot
// u < M (slot_entry modulo M), 0 for the other u < L.
template <typename T>
__global__ __launch_bounds__(256) void k_bs_fwd_prep(const typename Complex<T>::type* __restrict__ spec,
                                                     typename Complex<T>::type* __restrict__ B,
                                                     const RowMeta* __restrict__ rows, const T* __restrict__ tab,
                                                     int R, int half, int M, int64_t L,
                                                     const typename Complex<T>::type* __restrict__ chirp) {
  using C = typename Complex<T>::type;
  const int64_t u = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (u >= L) return;
  const int64_t gr = blockIdx.y;
  const int64_t seg = gr / R;
  const RowMeta rm = rows[gr - seg * R];
  C val{0, 0};
  if (u < M) {
    int sh = (rm.s - rm.lo) % M;
    if (sh < 0) sh += M;
    const int d = static_cast<int>(u) + sh < M ? static_cast<int>(u) + sh : static_cast<int>(u) + sh - M;
    if (d <= rm.hi - rm.lo) {
      const int c = rm.lo + d;
      C x = spec[seg * half + (c == half ? 0 : c)];
      if (c == 0) x.y = 0;                     // slot 0 of the spectrum holds (X[0], X[N/2])
      if (c == half) x = C{x.y, 0};
      const T w = tab[rm.off + d];
      val = c_mul(C{x.x * w, x.y * w}, chirp[u]);
    }
  }
  B[gr * L + u] = val;
}

// Inverse, before: B[gr][u] = Y[gr][u] conj(a[u]) for u < M, 0 for u < L.
template <typename T>
__global__ __launch_bounds__(256) void k_bs_inv_prep(const typename Complex<T>::type* __restrict__ Y,
                                                     typename Complex<T>::type* __restrict__ B, int M, int64_t L,
                                                     const typename Complex<T>::type* __restrict__ chirp) {
  using C = typename Complex<T>::type;
  const int64_t u = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (u >= L) return;
  const int64_t gr = blockIdx.y;
  B[gr * L + u] = u < M ? c_mul(Y[gr * M + u], c_conj(chirp[u])) : C{0, 0};
}

// The spectrum of the convolution: B[gr][k] *= Bhat[k] (Bhat holds the 1/L).
template <typename T>
__global__ __launch_bounds__(256) void k_bs_mul(typename Complex<T>::type* __restrict__ B, int64_t L,
                                                const typename Complex<T>::type* __restrict__ bhat) {
  const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (k >= L) return;
  const int64_t i = int64_t(blockIdx.y) * L + k;
  B[i] = c_mul(B[i], bhat[k]);
}

// Forward, after: Y[gr][m] = B[gr][m] a[m], m < M.
template <typename T>
__global__ __launch_bounds__(256) void k_bs_fwd_post(const typename Complex<T>::type* __restrict__ B,
                                                     typename Complex<T>::type* __restrict__ Y, int M, int64_t L,
                                                     const typename Complex<T>::type* __restrict__ chirp) {
  const int64_t m = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (m >= M) return;
  const int64_t gr = blockIdx.y;
  Y[gr * M + m] = c_mul(B[gr * L + m], chirp[m]);
}

// Inverse, after: the kept slots u < M times conj(a[u]) and the table into
// the packed buffer Sbuf[seg * sum_len + off + d].
template <typename T>
__global__ __launch_bounds__(256) void k_bs_inv_post(const typename Complex<T>::type* __restrict__ B,
                                                     typename Complex<T>::type* __restrict__ Sbuf,
                                                     const RowMeta* __restrict__ rows, const T* __restrict__ tab,
                                                     int R, int64_t sum_len, int M, int64_t L,
                                                     const typename Complex<T>::type* __restrict__ chirp) {
  using C = typename Complex<T>::type;
  const int u = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
  if (u >= M) return;
  const int64_t gr = blockIdx.y;
  const int64_t seg = gr / R;
  const RowMeta rm = rows[gr - seg * R];
  int sh = (rm.s - rm.lo) % M;
  if (sh < 0) sh += M;
  const int d = u + sh < M ? u + sh : u + sh - M;
  if (d > rm.hi - rm.lo) return;
  const C z = c_mul(B[gr * L + u], c_conj(chirp[u]));
  const T w = tab[rm.off + d];
  Sbuf[seg * sum_len + rm.off + d] = C{z.x * w, z.y * w};
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
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int64_t u = n1 + l1 * F::in_index(tl, i);
    const int64_t c = rm.lo + ((u + rm.s - rm.lo) & (n_out - 1));   // kept bin of slot u, if <= hi
    C val{0, 0};
    if (c <= rm.hi) {
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
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int64_t m = k2_0 + cc + l2 * F::out_index(tl, i);
    const int64_t c = rm.lo + ((m + rm.s - rm.lo) & (n_out - 1));   // kept bin of slot m, if <= hi
    if (c <= rm.hi) {
      const T w = tb[c];
      dst[c] = C{v[i].x * w, v[i].y * w};
    }
  }
}

// Single-tile recovery on rows longer than one workgroup: the second pass of
// the row's N_out-point forward transform (after k_fft_cols over row `row` of
// each segment, intermediate rows of stride a_stride), then the kept slots
// times the tile table into Sx[seg][c], as k_tile_rows does.
template <typename T, int L1>
__global__ __launch_bounds__((ColGeom<T, L1>::NT)) void k_tile_rows_rowst(
    const typename Complex<T>::type* __restrict__ A, typename Complex<T>::type* __restrict__ Sx,
    const RowMeta* __restrict__ rows, const T* __restrict__ tab, int row, int half, int64_t a_stride,
    int64_t n_out, int64_t l2, const typename Complex<T>::type* __restrict__ tw) {
  using C = typename Complex<T>::type;
  using Geo = ColGeom<T, L1>;
  using F = BlockFft<T, L1, Geo::E, -1>;
  __shared__ C lds[Geo::CC * lds_size(L1)];
  const int t = threadIdx.x;
  const int64_t seg = blockIdx.y;
  const int64_t k2_0 = int64_t(blockIdx.x) * Geo::CC;
  const C* src = A + seg * a_stride + k2_0 * L1;
  for (int i = t; i < Geo::CC * L1; i += Geo::NT) lds[(i / L1) * lds_size(L1) + lds_pad(i % L1)] = src[i];
  __syncthreads();
  const int cc = t % Geo::CC, tl = t / Geo::CC;
  C* reg = lds + cc * lds_size(L1);
  C v[Geo::E];
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) v[i] = reg[lds_pad(F::in_index(tl, i))];
  __syncthreads();
  F::run(v, reg, tl, F::twiddles(tw));
  const RowMeta rm = rows[row];
  C* dst = Sx + seg * (half + 1);
  const T* tb = tab + rm.off - rm.lo;
#pragma unroll
  for (int i = 0; i < Geo::E; ++i) {
    const int64_t m = k2_0 + cc + l2 * F::out_index(tl, i);
    const int64_t c = rm.lo + ((m + rm.s - rm.lo) & (n_out - 1));   // kept bin of slot m, if <= hi
    if (c <= rm.hi) {
      const T w = tb[c];
      dst[c] = C{v[i].x * w, v[i].y * w};
    }
  }
}

}  // namespace qtam
