// Gain x soft-threshold mask on envelope coefficients, and its gradients:
// the denoising model of the differentiable workload (masking the complex
// coefficients before the inverse, Sec. V; the transform inside a
// differentiable denoising pipeline, App. A).
//   forward:  out[b,k,m] = g_k * m * y,   m = max(0, 1 - lambda_k / |y|)
//   backward: with G = dL/dout (dL/dRe + i dL/dIm) and p = Re(conj(y) G),
//             dL/dy = g_k * (m G + [m > 0 and lambda_k > 0] lambda_k p / |y|^3 * y),
//             dL/dg_k = sum over b and m of m p.
// |y| is floored at the smallest normal number (no 0/0 where y = 0), and
// lambda p / |y|^3 is formed as (lambda/|y|) (p (1/|y|)) (1/|y|), which stays
// finite wherever m > 0 (there |y| > lambda and |p| <= |y| |G|).
#pragma once

#include "device_common.hpp"

namespace qtam {

template <typename T>
struct MaskMath {
  using C = typename Complex<T>::type;
  static __device__ __forceinline__ T tiny() { return sizeof(T) == 4 ? T(1.17549435e-38f) : T(2.2250738585072014e-308); }
  static __device__ __forceinline__ T absc(C v) { return fmax(sqrt(fmadd(v.x, v.x, v.y * v.y)), tiny()); }
  // mask value max(0, 1 - lambda / r)
  static __device__ __forceinline__ T mask(T lam, T r) { return fmax(T(0), T(1) - lam / r); }
  // g * mask * v
  static __device__ __forceinline__ C apply(C v, T g, T lam) {
    const T s = mask(lam, absc(v)) * g;
    return C{v.x * s, v.y * s};
  }
  // dL/dv of apply at v for the incoming gradient G; adds m p to acc. Two
  // divisions: q = lambda / r (the mask's own quotient) and 1 / r.
  static __device__ __forceinline__ C grad(C v, C G, T g, T lam, T& acc) {
    const T r = absc(v);
    const T q = lam / r;
    const T mk = fmax(T(0), T(1) - q);
    const T p = fmadd(v.x, G.x, v.y * G.y);
    const T ir = T(1) / r;
    const T c = (mk > T(0) && lam > T(0)) ? q * (p * ir) * ir : T(0);
    acc = fmadd(mk, p, acc);
    return C{g * fmadd(c, v.x, mk * G.x), g * fmadd(c, v.y, mk * G.y)};
  }
};

// Elementwise forward over [segs, R, L] (L = N_out), grid (ceil(L / 256), segs * R).
template <typename T>
__global__ __launch_bounds__(256) void k_mask_fwd(const typename Complex<T>::type* __restrict__ y,
                                                  const T* __restrict__ gain, const T* __restrict__ lam,
                                                  typename Complex<T>::type* __restrict__ out, int R, int L) {
  using M = MaskMath<T>;
  const int m = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
  if (m >= L) return;
  const int64_t gr = blockIdx.y;
  const int k = static_cast<int>(gr % R);
  const int64_t i = gr * L + m;
  out[i] = M::apply(y[i], gain[k], lam[k]);
}

// Backward, one workgroup per row (segment, k): dL/dy elementwise, and the
// row's sum of m p by a fixed-order tree into part[gr] (the gain gradient's
// share of this row).
template <typename T>
__global__ __launch_bounds__(256) void k_mask_bwd(const typename Complex<T>::type* __restrict__ y,
                                                  const typename Complex<T>::type* __restrict__ gout,
                                                  const T* __restrict__ gain, const T* __restrict__ lam,
                                                  typename Complex<T>::type* __restrict__ gy, T* __restrict__ part,
                                                  int R, int L) {
  using C = typename Complex<T>::type;
  using M = MaskMath<T>;
  __shared__ T red[256];
  const int64_t gr = blockIdx.x;
  const int k = static_cast<int>(gr % R);
  const T lk = lam[k], gk = gain[k];
  const C* yr = y + gr * L;
  const C* gor = gout + gr * L;
  C* gyr = gy + gr * L;
  T acc = 0;
  for (int m = threadIdx.x; m < L; m += 256) gyr[m] = M::grad(yr[m], gor[m], gk, lk, acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[gr] = red[0];
}

// dL/dg_k = sum over segments of part[seg * R + k], one wave per k: lane l
// adds segments l, l + 64, l + 128, ... in that order, then the lanes combine
// by a fixed xor butterfly (the same order on every call).
template <typename T>
__global__ __launch_bounds__(64) void k_gain_sum(const T* __restrict__ part, T* __restrict__ dgain, int R,
                                                 int64_t segs) {
  const int k = static_cast<int>(blockIdx.x);
  const int l = static_cast<int>(threadIdx.x);
  T s = 0;
  for (int64_t b = l; b < segs; b += 64) s += part[b * R + k];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
  if (l == 0) dgain[k] = s;
}

}  // namespace qtam
