// Block-level Stockham FFT engine for gfx950.
//
// A transform of length L (a power of two) is processed by TPR = L/E threads,
// each holding E complex values in registers. Every pass applies radix-R
// butterflies (R = min(E, 16), the last pass possibly smaller; with E = 32 a
// thread holds two groups) to values held in registers; between passes the
// values are exchanged through an LDS region of the transform (in two rounds
// over half of it when the whole would not fit). First-pass inputs and last-pass outputs are addressed so that
// consecutive threads touch consecutive elements: kernels feed the engine
// straight from global memory and store its results straight back, coalesced.
//
// Layout of the registers of thread tl (tl in [0, TPR)):
//   before the first pass: v[q*R0 + r] = a[tl + q*TPR + r*(L/R0)]
//   after the last pass:   v[q*RL + r] = A[tl + q*TPR + r*(L/RL)]
// Twiddles: every pass after the first (stride NS, radix R) needs
// w^r, w = exp(-2 pi i k / (NS R)), r in [1, R), for its k = j mod NS. A
// per-pass table built on the host in FP64 holds only the base powers
// w^1, w^2, w^4, w^8 (those below R) in blocks [s*NS + k], so the threads of a
// wave, which hold consecutive k, read consecutive entries; the other powers
// are products of at most three of them. Four loads instead of fifteen per
// radix-16 pass keep the twiddle traffic small next to the data streamed
// through the caches. Direction S = -1 computes sum_n a_n e^{-2 pi i nk/L},
// S = +1 the unnormalised inverse kernel e^{+2 pi i nk/L} (conjugated
// twiddles).
#pragma once

#include <hip/hip_runtime.h>

#include "gmem.hpp"

namespace qtam {

template <typename T> struct Complex;
template <> struct Complex<float> { using type = float2; };
template <> struct Complex<double> { using type = double2; };

template <typename C> __device__ __forceinline__ C c_add(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C c_sub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C c_conj(C a) { return C{a.x, -a.y}; }
// Fused multiply-add with the product and the addend chosen here, not by the
// compiler: every kernel instantiation then rounds the same way, so variants
// of one kernel (with or without row statistics, say) write identical bits.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename C> __device__ __forceinline__ C c_mul(C a, C b) {
  return C{fmadd(a.x, b.x, -(a.y * b.y)), fmadd(a.x, b.y, a.y * b.x)};
}
template <typename C, typename T> __device__ __forceinline__ C c_scale(C a, T s) { return C{a.x * s, a.y * s}; }
// a * (S i): S = +1 multiplies by i, S = -1 by -i
template <int S, typename C> __device__ __forceinline__ C c_mul_si(C a) {
  if constexpr (S > 0) return C{-a.y, a.x};
  else return C{a.y, -a.x};
}

// cos and sin of 2 pi k / 16, k = 0..4 (the rest follow by symmetry)
struct Root16 {
  static constexpr double c1 = 0.92387953251128675613;
  static constexpr double s1 = 0.38268343236508977173;
  static constexpr double r2 = 0.70710678118654752440;
};

// a * exp(S 2 pi i k / 16) for a compile-time k
template <int S, int K, typename C>
__device__ __forceinline__ C c_mul_root16(C a) {
  using T = decltype(a.x);
  constexpr int k = ((K % 16) + 16) % 16;
  if constexpr (k == 0) return a;
  else if constexpr (k == 4) return c_mul_si<S>(a);
  else if constexpr (k == 8) return C{-a.x, -a.y};
  else if constexpr (k == 12) return c_mul_si<-S>(a);
  else if constexpr (k == 2 || k == 6 || k == 10 || k == 14) {
    // exp(S i pi/4 * k/2) = (cx + i sy) / sqrt 2, cx, sy in {+1, -1}
    constexpr T r = static_cast<T>(Root16::r2);
    constexpr bool cpos = (k == 2 || k == 14);
    constexpr bool spos = (k == 2 || k == 6) == (S > 0);
    const T re = cpos ? (spos ? a.x - a.y : a.x + a.y) : (spos ? -a.x - a.y : a.y - a.x);
    const T im = cpos ? (spos ? a.x + a.y : a.y - a.x) : (spos ? a.x - a.y : -a.x - a.y);
    return C{re * r, im * r};
  } else {
    // k odd: cos / sin of 2 pi k/16 from the first-octant values
    constexpr int m = k % 8;                     // reduce by pi
    constexpr T sg = k >= 8 ? T(-1) : T(1);
    constexpr T cs = static_cast<T>(m == 1 ? Root16::c1 : m == 3 ? Root16::s1 : m == 5 ? -Root16::s1 : -Root16::c1);
    constexpr T sn = static_cast<T>(m == 1 ? Root16::s1 : m == 3 ? Root16::c1 : m == 5 ? Root16::c1 : Root16::s1);
    constexpr T cx = sg * cs;
    constexpr T sy = sg * sn * static_cast<T>(S);
    return C{fmadd(a.x, cx, -(a.y * sy)), fmadd(a.x, sy, a.y * cx)};
  }
}

template <int S, typename C>
__device__ __forceinline__ void dft2(C& a0, C& a1) {
  const C t = a0;
  a0 = c_add(t, a1);
  a1 = c_sub(t, a1);
}

template <int S, typename C>
__device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
  const C t0 = c_add(a0, a2), t1 = c_sub(a0, a2);
  const C t2 = c_add(a1, a3), t3 = c_mul_si<S>(c_sub(a1, a3));
  a0 = c_add(t0, t2);
  a2 = c_sub(t0, t2);
  a1 = c_add(t1, t3);
  a3 = c_sub(t1, t3);
}

// Second half of a radix-16 DFT split as n = 4 n1 + n2: group n2's output
// k1 sits at a[4 k1 + n2]; twiddles exp(S 2 pi i n2 k1 / 16), then the outer
// length-4 DFTs over the groups, results in natural order.
template <int S, typename C>
__device__ __forceinline__ void dft16_outer(C* a) {
  a[5] = c_mul_root16<S, 1>(a[5]);
  a[9] = c_mul_root16<S, 2>(a[9]);
  a[13] = c_mul_root16<S, 3>(a[13]);
  a[6] = c_mul_root16<S, 2>(a[6]);
  a[10] = c_mul_root16<S, 4>(a[10]);
  a[14] = c_mul_root16<S, 6>(a[14]);
  a[7] = c_mul_root16<S, 3>(a[7]);
  a[11] = c_mul_root16<S, 6>(a[11]);
  a[15] = c_mul_root16<S, 9>(a[15]);
  C y[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C b0 = a[4 * k1], b1 = a[4 * k1 + 1], b2 = a[4 * k1 + 2], b3 = a[4 * k1 + 3];
    dft4<S>(b0, b1, b2, b3);
    y[k1] = b0;
    y[k1 + 4] = b1;
    y[k1 + 8] = b2;
    y[k1 + 12] = b3;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = y[i];
}

// Radix-16 DFT of inputs known to be zero except a[0], a[1], a[14], a[15]
// (NZ = 4) or a[0], a[15] (NZ = 2): the operations of dft_small<S, 16> on the
// non-zero terms only, in the same order, so the results are the same bits
// (up to the sign of zeros). Each inner length-4 DFT then has one non-zero
// input: at n1 = 0 it copies it to all four outputs; at n1 = 3 the outputs
// are x, S i (-x), -x, -(S i (-x)).
template <int S, int NZ, typename C>
__device__ __forceinline__ void dft16_sparse(C* a) {
  static_assert(NZ == 2 || NZ == 4, "two or four non-zero inputs");
  auto from_first = [&](int n2) {   // group n2 with its only input at n1 = 0
    a[n2 + 4] = a[n2];
    a[n2 + 8] = a[n2];
    a[n2 + 12] = a[n2];
  };
  auto from_last = [&](int n2) {    // group n2 with its only input at n1 = 3
    const C x = a[n2 + 12];
    const C r = c_mul_si<S>(C{-x.x, -x.y});
    a[n2] = x;
    a[n2 + 4] = r;
    a[n2 + 8] = C{-x.x, -x.y};
    a[n2 + 12] = C{-r.x, -r.y};
  };
  from_first(0);
  from_last(3);
  if constexpr (NZ == 4) {
    from_first(1);
    from_last(2);
    dft16_outer<S>(a);
  } else {
    // groups 1 and 2 are zero: twiddles only on group 3, and each outer
    // length-4 DFT sees (b0, 0, 0, b3)
    a[7] = c_mul_root16<S, 3>(a[7]);
    a[11] = c_mul_root16<S, 6>(a[11]);
    a[15] = c_mul_root16<S, 9>(a[15]);
    C y[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      const C b0 = a[4 * k1], b3 = a[4 * k1 + 3];
      const C t3 = c_mul_si<S>(C{-b3.x, -b3.y});
      y[k1] = c_add(b0, b3);
      y[k1 + 4] = c_add(b0, t3);
      y[k1 + 8] = c_sub(b0, b3);
      y[k1 + 12] = c_sub(b0, t3);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = y[i];
  }
}

// In-register DFT of R values in natural order (R in 1, 2, 4, 8, 16).
// R = 8 and 16 split as n = 4 n1 + n2 ... : inner radix-4 DFTs over strided
// groups, twiddles exp(S 2 pi i n2 k1 / R), outer DFTs over the groups.
template <int S, int R, typename C>
__device__ __forceinline__ void dft_small(C* a) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2<S>(a[0], a[1]);
  } else if constexpr (R == 4) {
    dft4<S>(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 8) {
    // n = 2 n1 + n2, k = k1 + 4 k2
    dft4<S>(a[0], a[2], a[4], a[6]);
    dft4<S>(a[1], a[3], a[5], a[7]);
    a[3] = c_mul_root16<S, 2>(a[3]);
    a[5] = c_mul_root16<S, 4>(a[5]);
    a[7] = c_mul_root16<S, 6>(a[7]);
    C y[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C e = a[2 * k1], o = a[2 * k1 + 1];
      dft2<S>(e, o);
      y[k1] = e;
      y[k1 + 4] = o;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = y[i];
  } else if constexpr (R == 16) {
    // n = 4 n1 + n2: group n2 holds a[n2], a[4+n2], a[8+n2], a[12+n2]
    dft4<S>(a[0], a[4], a[8], a[12]);
    dft4<S>(a[1], a[5], a[9], a[13]);
    dft4<S>(a[2], a[6], a[10], a[14]);
    dft4<S>(a[3], a[7], a[11], a[15]);
    dft16_outer<S>(a);
  }
}

// LDS index with one pad element every 32, which spreads power-of-two strides
// over the banks; the map is affine inside each run of 32, so exchanges keep
// constant instruction offsets.
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 5); }
constexpr int lds_size(int l) { return l + l / 32 + 1; }

// Twiddle table layouts: TW_POW stores the base powers w^1, w^2, w^4, w^8 of
// each pass and forms the others by products (little table traffic, for
// kernels that stream their data); TW_FULL stores every w^r, r in [1, R)
// (no products, for kernels whose vector ALU is the limit); TW_MIXED stores
// every power for passes of stride at most kFullStride (a table of a few KiB
// that stays in the L1 cache) and base powers for the longer strides.
enum TwiddleMode { TW_POW = 0, TW_FULL = 1, TW_MIXED = 2 };
constexpr int kFullStride = 16;
constexpr bool tw_full_pass(int mode, int ns) { return mode == TW_FULL || (mode == TW_MIXED && ns <= kFullStride); }

// LDS a transform of length L needs: the padded exchange region, or half of
// it when the whole one would not fit the 160 KiB of a workgroup (the
// exchanges then go in two rounds, one per half of the destination indices).
template <typename T, int L>
constexpr bool fft_split() {
  return size_t(lds_size(L)) * sizeof(typename Complex<T>::type) > 160u * 1024u;
}
template <typename T, int L>
constexpr int fft_lds_elems() {
  return fft_split<T, L>() ? lds_size(L / 2) : lds_size(L);
}

template <typename T, int L, int E, int S, int TW = TW_POW>
struct BlockFft {
  using C = typename Complex<T>::type;
  static_assert((L & (L - 1)) == 0 && (E & (E - 1)) == 0 && E <= L && E <= 32, "pow2 sizes");
  static constexpr int TPR = L / E;
  static constexpr int RMAX = E < 16 ? E : 16;   // butterflies of at most radix 16; E = 32 holds two groups
  static constexpr int radix(int ns) { return (L / ns >= RMAX) ? RMAX : L / ns; }
  static constexpr bool SPLIT = fft_split<T, L>();
  static constexpr int WN = E > 16 ? 16 : E;     // twiddle registers: one group at a time when E > 16
  static constexpr int last_ns() {
    int ns = 1;
    while (ns * radix(ns) < L) ns *= radix(ns);
    return ns;
  }
  static constexpr int R0 = radix(1);
  static constexpr int RL = radix(last_ns());
  // number of stored powers of the radix-R pass of stride ns: w^(2^s) < R,
  // or all w^r, r < R
  static constexpr int slots(int r, int ns) {
    return tw_full_pass(TW, ns) ? r - 1 : (r >= 16 ? 4 : r >= 8 ? 3 : r >= 4 ? 2 : r >= 2 ? 1 : 0);
  }
  // start of the twiddle block of the pass with stride ns
  static constexpr int tw_offset(int ns) {
    int off = 0, n = 1;
    while (n < ns) {
      if (n > 1) off += slots(radix(n), n) * n;
      n *= radix(n);
    }
    return off;
  }
  static constexpr int tw_size() { return tw_offset(L); }
  // registers of a radix-R2 pass whose input index lies below L/2
  static constexpr int lower_reads(int r2) {
    int n = 0;
    for (int q = 0; q < E / r2; ++q)
      for (int r = 0; r < r2; ++r) n += (q * TPR + r * (L / r2) < L / 2) ? 1 : 0;
    return n;
  }

  __device__ static __forceinline__ int in_index(int tl, int i) {
    return tl + (i / R0) * TPR + (i % R0) * (L / R0);
  }
  __device__ static __forceinline__ int out_index(int tl, int i) {
    return tl + (i / RL) * TPR + (i % RL) * (L / RL);
  }

  // Twiddles of the pass with stride NS for this thread: w[q*R + r], r >= 1,
  // from the base powers w^1, w^2, w^4, w^8 (groups q0 .. q1-1, stored from
  // w[0] on when only one group is held at a time).
  template <int NS>
  __device__ static __forceinline__ void load_twiddles(C (&w)[WN], int tl, rsrc_t tw, int q0 = 0,
                                                       int q1 = E / radix(NS)) {
    constexpr int R = radix(NS);
#pragma unroll
    for (int q = q0; q < q1; ++q) {
      const uint32_t k = static_cast<uint32_t>((tl + q * TPR) & (NS - 1));
      if constexpr (tw_full_pass(TW, NS)) {
#pragma unroll
        for (int r = 1; r < R; ++r)
          w[(q - q0) * R + r] = bload<C>(tw, k * sizeof(C), (tw_offset(NS) + (r - 1) * NS) * sizeof(C));
      } else {
        C a[16];
#pragma unroll
        for (int sl = 0; sl < slots(R, NS); ++sl)
          a[1 << sl] = bload<C>(tw, k * sizeof(C), (tw_offset(NS) + sl * NS) * sizeof(C));
        if constexpr (R > 2) a[3] = c_mul(a[2], a[1]);
        if constexpr (R > 4) {
          a[5] = c_mul(a[4], a[1]);
          a[6] = c_mul(a[4], a[2]);
          a[7] = c_mul(a[4], a[3]);
        }
        if constexpr (R > 8) {
#pragma unroll
          for (int r = 9; r < 16; ++r) a[r] = c_mul(a[8], a[r - 8]);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) w[(q - q0) * R + r] = a[r];
      }
    }
  }

  // One radix-R pass on registers: for NS > 1 its twiddles are read and
  // applied, then the butterflies; unless it was the last pass the values
  // are exchanged through LDS into the next pass's order.
  template <int NS>
  __device__ static __forceinline__ void pass(C (&v)[E], C (&w)[WN], C* lds, int tl, rsrc_t tw, int nz) {
    constexpr int R = radix(NS);
    constexpr bool kAll = WN == E;   // all groups' twiddles at once, else one group at a time
    if constexpr (NS > 1 && kAll) load_twiddles<NS>(w, tl, tw);
#pragma unroll
    for (int q = 0; q < E / R; ++q) {
      if constexpr (NS > 1) {
        if constexpr (!kAll) load_twiddles<NS>(w, tl, tw, q, q + 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C t = w[(kAll ? q * R : 0) + r];
          if constexpr (S > 0) t.y = -t.y;
          v[q * R + r] = c_mul(v[q * R + r], t);
        }
      }
      if constexpr (NS == 1 && R == 16) {
        if (nz == 2) dft16_sparse<S, 2>(&v[q * R]);
        else if (nz == 4) dft16_sparse<S, 4>(&v[q * R]);
        else dft_small<S, R>(&v[q * R]);
      } else {
        dft_small<S, R>(&v[q * R]);
      }
    }
    if constexpr (NS * R < L) {
      constexpr int NS2 = NS * R;
      constexpr int R2 = radix(NS2);
      if constexpr (!SPLIT) {
#pragma unroll
        for (int q = 0; q < E / R; ++q) {
          const int j = tl + q * TPR;
          const int k = j & (NS - 1);
          const int base = (j - k) * R + k;
#pragma unroll
          for (int r = 0; r < R; ++r) lds[lds_pad(base + r * NS)] = v[q * R + r];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < E / R2; ++q) {
          const int j = tl + q * TPR;
#pragma unroll
          for (int r = 0; r < R2; ++r) v[q * R2 + r] = lds[lds_pad(j + r * (L / R2))];
        }
        __syncthreads();
      } else {
        // The LDS region holds half of the indices. With two register groups
        // per pass (E = 2R) and NS dividing TPR, group 0 holds exactly the
        // values bound for indices below L/2 and group 1 the others, and a
        // value bound for register (q, r) of the next pass comes from below
        // L/2 iff q TPR + r L/R2 < L/2 (tl < TPR; both terms are multiples of
        // TPR). Round 0 moves the lower half (into tmp, since the registers it
        // fills may still hold group-1 values), round 1 the upper half.
        static_assert(E / R == 2 && TPR % NS == 0 && lower_reads(R2) == E / 2, "split exchange layout");
        constexpr int H = L / 2;
        C tmp[E / 2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          {
            const int j = tl + h * TPR;
            const int k = j & (NS - 1);
            const int base = (j - k) * R + k - h * H;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[lds_pad(base + r * NS)] = v[h * R + r];
          }
          __syncthreads();
          int n = 0;
#pragma unroll
          for (int q = 0; q < E / R2; ++q) {
#pragma unroll
            for (int r = 0; r < R2; ++r) {
              const int off = q * TPR + r * (L / R2);   // compile-time after unrolling
              if ((off < H) == (h == 0)) {
                const C x = lds[lds_pad(tl + off - h * H)];
                if (h == 0) tmp[n++] = x;
                else v[q * R2 + r] = x;
              }
            }
          }
          __syncthreads();
        }
        int n = 0;
#pragma unroll
        for (int q = 0; q < E / R2; ++q) {
#pragma unroll
          for (int r = 0; r < R2; ++r) {
            if (q * TPR + r * (L / R2) < H) v[q * R2 + r] = tmp[n++];
          }
        }
      }
      pass<NS2>(v, w, lds, tl, tw, 0);
    }
  }

  // Every thread of the workgroup must call run (it contains barriers).
  // tw: buffer resource over the per-pass twiddle table of this (L, E).
  // nz = 2 or 4 (wave-uniform) when the first pass is radix 16 and each of
  // the wave's first-pass groups is zero except v[0] and v[15] (2), or except
  // v[0], v[1], v[14], v[15] (4): that pass then skips the zero terms, with
  // the same results; any other value runs the full transform.
  __device__ static __forceinline__ void run(C (&v)[E], C* lds, int tl, rsrc_t tw, int nz = 0) {
    C w[WN];
    pass<1>(v, w, lds, tl, tw, nz);
  }
  // offsets of register element i from the thread's own index tl
  static constexpr int in_off(int i) { return (i / R0) * TPR + (i % R0) * (L / R0); }
  static constexpr int out_off(int i) { return (i / RL) * TPR + (i % RL) * (L / RL); }
  __device__ static __forceinline__ rsrc_t twiddles(const C* tw) {
    return make_rsrc(tw, static_cast<uint32_t>((tw_size() > 0 ? tw_size() : 1) * sizeof(C)));
  }
};

}  // namespace qtam
